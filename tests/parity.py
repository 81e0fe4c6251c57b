"""Path-by-path comparison of tracker results (GPU path vs CPU oracle, or
one GPU launch shape vs another).

The parity bar: every path has the same converged / not-converged outcome
on both sides (so the converged counts and the not-converged counts are
identical), and both converged endpoints of a path agree within 1e-8
relative, ||x_a - x_b||_inf <= 1e-8 max(1, ||x_b||_inf).  Both sides end a
path reaching t = 1 with the same end game (double-double refinement to the
nearest double of the root, residual in double-double), so there is no
allowance for paths near the residual gate.

The sub-status of a path that does not converge (diverged past the radius,
step size below the minimum, too many steps) is reported, not gated: in
affine coordinates a path to a point at infinity may stop on the divergence
radius or on the minimum step depending on rounding.  What is checked of it
is that it is valid: a DIVERGED endpoint lies beyond the radius."""
from __future__ import annotations

import dataclasses
import os

import numpy as np

REL = 1e-8
GATE = 1e-10
DIV_RADIUS = 1e8
NTHREADS = min(16, os.cpu_count() or 1)


def close_rows(a, b, rel=REL):
    """Per row: ||a - b||_inf <= rel * max(1, ||b||_inf)."""
    if len(a) == 0:
        return np.zeros(0, bool)
    return np.abs(a - b).max(axis=1) <= rel * np.maximum(1.0, np.abs(b).max(axis=1))


@dataclasses.dataclass
class Parity:
    flips: np.ndarray    # converged on one side only
    far: np.ndarray      # converged on both sides, endpoints apart
    substat: np.ndarray  # not converged on both sides, sub-status differs

    @property
    def ok(self) -> bool:
        return len(self.flips) == 0 and len(self.far) == 0


def compare_paths(e_a, s_a, e_b, s_b, rel=REL) -> Parity:
    ca, cb = s_a == 0, s_b == 0
    both = np.nonzero(ca & cb)[0]
    far = both[~close_rows(e_a[both], e_b[both], rel)]
    flips = np.nonzero(ca != cb)[0]
    substat = np.nonzero(~ca & ~cb & (s_a != s_b))[0]
    return Parity(flips, far, substat)


def backward_error(system, X):
    """Relative backward error of each row x of X: ||f(x)||_inf over
    max_i sum_k |c_ik| |x^a_ik| (f in double: a diagnostic, not a gate)."""
    X = np.atleast_2d(np.asarray(X, np.complex128))
    out = np.zeros(len(X))
    eq = np.repeat(np.arange(system.n), np.diff(system.eq_ptr))
    for r, x in enumerate(X):
        with np.errstate(all="ignore"):
            mono = system.coeff * np.prod(x[None, :] ** system.exps, axis=1)
            f = np.zeros(system.n, complex)
            np.add.at(f, eq, mono)
            scale = np.zeros(system.n)
            np.add.at(scale, eq, np.abs(mono))
            out[r] = np.abs(f).max() / max(scale.max(), np.finfo(float).tiny)
    return out


def assert_parity(e_a, s_a, e_b, s_b, what, system=None, ids=None, log=None, rel=REL):
    """Asserts the parity bar; a, b: (endpoints [P, n], status [P]).  On a
    mismatch the message lists the first paths with both statuses and, when
    the system is given, both endpoints' relative backward errors."""
    p = compare_paths(e_a, s_a, e_b, s_b, rel)
    ids = np.arange(len(s_a)) if ids is None else np.asarray(ids)
    div_a = (s_a == 1) & ~(np.abs(e_a).max(axis=1) > DIV_RADIUS)
    div_b = (s_b == 1) & ~(np.abs(e_b).max(axis=1) > DIV_RADIUS)
    if log is not None:
        log(f"  {what}: converged {int((s_a == 0).sum())} / {int((s_b == 0).sum())}, "
            f"not converged {int((s_a != 0).sum())} / {int((s_b != 0).sum())}, "
            f"sub-status differences {len(p.substat)}")
    if not p.ok:
        lines = []
        for i in list(p.flips[:8]) + list(p.far[:8]):
            line = f"path {int(ids[i])}: status {int(s_a[i])} / {int(s_b[i])}"
            if system is not None:
                be = backward_error(system, np.stack([e_a[i], e_b[i]]))
                line += f", backward error {be[0]:.2e} / {be[1]:.2e}"
            lines.append(line)
        raise AssertionError(f"{what}: {len(p.flips)} converged-flag differences, "
                             f"{len(p.far)} endpoints apart\n  " + "\n  ".join(lines))
    assert not div_a.any() and not div_b.any(), f"{what}: DIVERGED endpoint inside the radius"
    return p


def assert_residuals(system, e, st, gate=GATE):
    """Every converged endpoint passes the residual gate, with f evaluated by
    the oracle's own (double-double) evaluator, not the tracker's report."""
    import oracle
    conv = np.asarray(st) == 0
    if not conv.any():
        return
    pts = np.asarray(e)[conv]
    if len(pts) > 4096:  # the oracle's evaluator releases the GIL: split over threads
        from concurrent.futures import ThreadPoolExecutor
        parts = np.array_split(pts, 64)
        with ThreadPoolExecutor(NTHREADS) as ex:
            res = np.concatenate(list(ex.map(lambda p: oracle.residuals_dd(system, p), parts)))
    else:
        res = oracle.residuals_dd(system, pts)
    bad = np.nonzero(~(res <= gate))[0]
    assert len(bad) == 0, f"{system.name}: {len(bad)} converged endpoints with residual " \
                          f"{res[bad[:4]]} above {gate}"


def match_sets(a, b, rel=REL, seed=0):
    """True when the rows of a and b pair off one to one with
    ||a_i - b_j||_inf <= rel max(1, ||b_j||_inf).  Candidates come from a
    sort on a random real projection (|proj(u) - proj(v)| <= ||u - v||_inf),
    so large sets match in n log n."""
    a = np.asarray(a, np.complex128).reshape(len(a), -1)
    b = np.asarray(b, np.complex128).reshape(len(b), -1)
    if a.shape != b.shape:
        return False
    if len(a) == 0:
        return True
    rng = np.random.default_rng(seed)
    w = rng.uniform(-1, 1, size=(2, a.shape[1]))
    w /= np.abs(w).sum()
    pa = a.real @ w[0] + a.imag @ w[1]
    pb = b.real @ w[0] + b.imag @ w[1]
    order = np.argsort(pb)
    pbs = pb[order]
    nb = np.maximum(1.0, np.abs(b).max(axis=1))
    used = np.zeros(len(b), bool)
    for i in np.argsort(pa):
        tol = rel * max(1.0, float(np.abs(a[i]).max())) * 2.0
        lo = np.searchsorted(pbs, pa[i] - tol, "left")
        hi = np.searchsorted(pbs, pa[i] + tol, "right")
        best, bj = np.inf, -1
        for j in order[lo:hi]:
            if used[j]:
                continue
            d = float(np.abs(a[i] - b[j]).max())
            if d <= rel * nb[j] and d < best:
                best, bj = d, j
        if bj < 0:
            return False
        used[bj] = True
    return True
