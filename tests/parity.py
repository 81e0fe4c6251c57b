"""Path-by-path comparison of tracker results (GPU path vs CPU oracle, or
one GPU launch shape vs another).

A path counts as converged when its final residual ||f(x)||_inf is at most
the absolute gate tol_residual (1e-10).  Two correct FP64 implementations
that evaluate f in different orders can land on opposite sides of that gate
for a root whose residual sits at the rounding floor (large |x|).  Such a
path is a borderline flip, not a mismatch, when both sides reached t = 1,
both residuals are within 10x the gate and the two endpoints agree within the
endpoint tolerance.  Anything else that differs is a hard mismatch."""
from __future__ import annotations

import numpy as np

REL = 1e-8
GATE = 1e-10


def close_rows(a, b, rel=REL):
    """Per row: ||a - b||_inf <= rel * max(1, ||b||_inf)."""
    if len(a) == 0:
        return np.zeros(0, bool)
    return np.abs(a - b).max(axis=1) <= rel * np.maximum(1.0, np.abs(b).max(axis=1))


def compare_paths(e_a, s_a, st_a, e_b, s_b, st_b, rel=REL, gate=GATE):
    """Returns (hard_mismatches, borderline_flips) as index arrays."""
    ca, cb = s_a == 0, s_b == 0
    both = ca & cb
    hard = list(np.nonzero(both)[0][~close_rows(e_a[both], e_b[both], rel)])
    flips = []
    for i in np.nonzero(ca != cb)[0]:
        ok = (st_a["t_final"][i] == 1.0 and st_b["t_final"][i] == 1.0
              and st_a["residual"][i] <= 10 * gate and st_b["residual"][i] <= 10 * gate
              and close_rows(e_a[i:i + 1], e_b[i:i + 1], rel)[0])
        (flips if ok else hard).append(i)
    return np.asarray(hard, np.int64), np.asarray(flips, np.int64)
