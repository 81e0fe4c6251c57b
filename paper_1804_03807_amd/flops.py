"""Algorithmic flop model of one tracking step (complex multiply = 6 flops,
complex add = 2), used to express measured throughput as FP64 FLOP/s.

Per evaluation of H, J_x at one point (reverse-mode differentiation of each
monomial, coefficient folded into the prefix products):
  * a term with k >= 2 factors: 3k - 3 complex multiplies (k prefix
    products, k - 1 partials, k - 2 suffix updates); k = 1: one multiply;
  * each factor with exponent e >= 2: e x^(e-1) costs 8 flops;
  * accumulation: 2 (k + 1) flops (value and k partials);
  * power table x_v^e, e <= e_max: 6 (e_max - 1) per variable;
  * homotopy assembly: start system x_i^{d_i} - 1 and its derivative
    (6 d_i + 4), H_i or H_t,i (20), J row scaling by t (2n) and the diagonal
    gamma (1-t) d_i x_i^{d_i-1} (8).
Per linear solve (LU with partial pivoting + two triangular solves):
  F_LU(n) = sum_{m=2..n} [3m + 6 + 6(m-1) + 8(m-1)^2] + 6,
  F_solve(n) = 8 n (n - 1) + 6 n.
The kernels solve by Gauss-Jordan elimination, which performs more
arithmetic than this count; achieved figures therefore understate the
executed FP64 rate.
"""
from __future__ import annotations

import numpy as np


def f_eval(system) -> int:
    ex = np.asarray(system.exps)
    n = int(system.n)
    total = 0
    for row in ex:
        k = int((row > 0).sum())
        high = int((row >= 2).sum())
        if k >= 2:
            total += 6 * (3 * k - 3)
        elif k == 1:
            total += 6
        total += 8 * high + 2 * (k + 1)
    emax = ex.max(axis=0)
    total += int(sum(6 * (max(1, int(e)) - 1) for e in emax))
    degs = system.degrees()
    total += int(sum(6 * int(d) + 4 + 20 + 2 * n + 8 for d in degs))
    return int(total)


def f_lu(n: int) -> int:
    return int(sum(3 * m + 6 + 6 * (m - 1) + 8 * (m - 1) ** 2 for m in range(2, n + 1)) + 6)


def f_solve(n: int) -> int:
    return int(8 * n * (n - 1) + 6 * n)


def per_eval_solve(system) -> int:
    """Flops of one evaluation followed by one linear solve."""
    return f_eval(system) + f_lu(system.n) + f_solve(system.n)


def run_flops(system, stats) -> float:
    """Algorithmic flops of a tracking run from per-path counters
    (evaluations and solves of predictor and corrector)."""
    ev = float(np.asarray(stats["evals"], dtype=np.float64).sum())
    so = float(np.asarray(stats["solves"], dtype=np.float64).sum())
    return ev * f_eval(system) + so * (f_lu(system.n) + f_solve(system.n))
