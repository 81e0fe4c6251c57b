"""Pins of the oracle's double-double tracker (the paper's "quality up",
Section 1, Section 5.1) to values computed with 50-digit arithmetic
(mpmath), never to the oracle itself: endpoints agree with the exact roots
to about 1e-30 relative, far beyond what double precision can reach."""
import itertools

import mpmath
import numpy as np

import oracle
import workloads as W

mpmath.mp.dps = 50


def _mp(z_hi, z_lo):
    return mpmath.mpc(z_hi.real, z_hi.imag) + mpmath.mpc(z_lo.real, z_lo.imag)


def test_dd_univariate_roots_to_30_digits(oracle_lib):
    s, poly = W.univariate(7, np.random.default_rng(27))
    hi, lo, st, _ = oracle.track_paths_dd(s, 0.6 - 0.8j)
    assert (st == 0).all()
    roots = mpmath.polyroots([mpmath.mpc(c.real, c.imag) for c in poly], maxsteps=300,
                             extraprec=300)
    used = set()
    for h, l in zip(hi[:, 0], lo[:, 0]):
        x = _mp(h, l)
        d, j = min((abs(x - r) / max(1, abs(r)), j) for j, r in enumerate(roots))
        assert d <= 1e-28 and j not in used
        used.add(j)


def _mp_system(s):
    """The stored system with its double coefficients taken exactly."""
    terms = []
    for i in range(s.n):
        eq = []
        for t in range(int(s.eq_ptr[i]), int(s.eq_ptr[i + 1])):
            c = s.coeff[t]
            eq.append((mpmath.mpc(c.real, c.imag), [int(v) for v in s.exps[t]]))
        terms.append(eq)

    def f(*x):
        out = []
        for eq in terms:
            v = mpmath.mpc(0)
            for c, a in eq:
                m = c
                for j, e in enumerate(a):
                    if e:
                        m *= x[j] ** e
                v += m
            out.append(v)
        return out
    return f


def test_dd_linear_products_to_30_digits(oracle_lib):
    """Products of linear forms, expanded in double: the roots of the stored
    system are found by 50-digit Newton (mpmath.findroot) from the
    closed-form roots of the unexpanded products, then compared."""
    n, degs = 3, [2, 3, 2]
    s, Ls, betas = W.linear_products(n, degs, np.random.default_rng(33))
    hi, lo, st, _ = oracle.track_paths_dd(s, np.exp(1.1j), n_threads=4)
    assert (st == 0).sum() == int(np.prod(degs))
    F = _mp_system(s)
    exact = []
    for choice in itertools.product(*[range(d) for d in degs]):
        M = np.array([Ls[i][choice[i]] for i in range(n)])
        r = np.array([betas[i][choice[i]] for i in range(n)])
        x0 = np.linalg.solve(M, r)
        root = mpmath.findroot(F, [mpmath.mpc(v.real, v.imag) for v in x0], tol=1e-45)
        exact.append([root[i] for i in range(n)])
    used = set()
    for k in range(len(st)):
        x = [_mp(hi[k, i], lo[k, i]) for i in range(n)]
        best, bj = None, -1
        for j, e in enumerate(exact):
            d = max(abs(x[i] - e[i]) for i in range(n)) / max(1, max(abs(e[i]) for i in range(n)))
            if best is None or d < best:
                best, bj = d, j
        assert best <= 1e-27 and bj not in used
        used.add(bj)


def test_dd_dense_bezout_and_nearest_double(oracle_lib):
    """All 32 paths of the dense n = 5 system converge; the high parts are
    the double tracker's endpoints, which its end game rounds to the nearest
    double of the root."""
    wl = W.dense_small()
    s, g = wl.systems[0], wl.gammas[0]
    hi, lo, st, stats = oracle.track_paths_dd(s, g, n_threads=4)
    assert (st == 0).all() and (stats["residual"] <= 1e-26).all()
    e, st2, _ = oracle.track_paths(s, g, n_paths=32)
    assert (st2 == 0).all()
    assert np.array_equal(hi, e)
    assert (np.abs(lo) <= np.abs(hi) * 2.0 ** -52).all()
