"""Pins of the CPU oracle to facts other than itself: symbolic expansion,
closed forms, library routines, invariants and the paper's worked example.

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a bad pivot rule, a wrong step
update) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import sympy as sp

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_point(rng, n, scale=1.0):
    return scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)


def _sympy_system(s):
    xs = sp.symbols(f"x1:{s.n + 1}")
    eqs = []
    for i in range(s.n):
        e = 0
        for t in range(int(s.eq_ptr[i]), int(s.eq_ptr[i + 1])):
            c = complex(s.coeff[t])
            mono = 1
            for j in range(s.n):
                mono *= xs[j] ** int(s.exps[t, j])
            e += (sp.Float(c.real, 30) + sp.I * sp.Float(c.imag, 30)) * mono
        eqs.append(sp.expand(e))
    return xs, eqs


def _sympy_eval(xs, eqs, x):
    sub = {xs[j]: sp.Float(x[j].real, 30) + sp.I * sp.Float(x[j].imag, 30) for j in range(len(xs))}
    f = np.array([complex(sp.N(e.subs(sub), 25)) for e in eqs])
    J = np.array([[complex(sp.N(sp.diff(e, xj).subs(sub), 25)) for xj in xs] for e in eqs])
    return f, J


@pytest.mark.parametrize("make", [
    lambda rng: W.dense_system(3, [3, 2, 3], rng),
    lambda rng: W.cyclic_system(5, rng),
    lambda rng: W.embedded_cyclic4(rng),
])
def test_eval_matches_symbolic_expansion(oracle_lib, make):
    rng = np.random.default_rng(11)
    s = make(rng)
    xs, eqs = _sympy_system(s)
    for _ in range(3):
        x = _rand_point(rng, s.n, 1.3)
        f_ref, J_ref = _sympy_eval(xs, eqs, x)
        f, J = oracle.eval_system(s, x)
        scale = max(1.0, np.abs(f_ref).max())
        assert np.abs(f - f_ref).max() <= 1e-13 * scale * 10
        assert np.abs(J - J_ref).max() <= 1e-13 * max(1.0, np.abs(J_ref).max()) * 10


def test_jacobian_central_difference(oracle_lib):
    """Holomorphic f: (f(x+ev) - f(x-ev)) / 2e = J v + O(e^2)."""
    rng = np.random.default_rng(12)
    s = W.dense_system(4, [3, 3, 2, 3], rng)
    x = _rand_point(rng, 4)
    v = _rand_point(rng, 4)
    _, J = oracle.eval_system(s, x)
    errs = []
    for eps in (1e-2, 5e-3):
        fp, _ = oracle.eval_system(s, x + eps * v)
        fm, _ = oracle.eval_system(s, x - eps * v)
        errs.append(np.abs((fp - fm) / (2 * eps) - J @ v).max())
    # second order: halving eps divides the error by about 4
    assert 3.0 < errs[0] / errs[1] < 5.0
    # and a complex direction (holomorphy, not just real differentiability)
    fp, _ = oracle.eval_system(s, x + 1e-3j * v)
    fm, _ = oracle.eval_system(s, x - 1e-3j * v)
    assert np.abs((fp - fm) / (2e-3j) - J @ v).max() < 1e-4


def test_euler_identity_homogeneous(oracle_lib):
    """For q homogeneous of degree d: sum_j x_j dq/dx_j = d q."""
    rng = np.random.default_rng(13)
    d = 3
    full = W.dense_system(4, [d] * 4, rng)
    keep = full.exps.astype(int).sum(axis=1) == d
    eq_ptr = [0]
    for i in range(4):
        a, b = full.eq_ptr[i], full.eq_ptr[i + 1]
        eq_ptr.append(eq_ptr[-1] + int(keep[a:b].sum()))
    hom = W.PolySystem(4, np.asarray(eq_ptr, np.int32), full.coeff[keep].copy(),
                       full.exps[keep].copy())
    hom.validate()
    x = _rand_point(rng, 4)
    f, J = oracle.eval_system(hom, x)
    assert np.abs(J @ x - d * f).max() < 1e-12 * max(1, np.abs(f).max())


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 12])
def test_lu_solve_matches_lapack(oracle_lib, n):
    rng = np.random.default_rng(100 + n)
    for _ in range(5):
        A = _rand_point(rng, n * n).reshape(n, n)
        b = _rand_point(rng, n)
        y = oracle.lu_solve(A, b)
        y_ref = np.linalg.solve(A, b)
        assert np.abs(y - y_ref).max() <= 1e-12 * max(1, np.abs(y_ref).max()) * np.linalg.cond(A)


def test_lu_needs_pivoting_and_detects_singular(oracle_lib):
    A = np.array([[0, 1, 2], [1, 0, 3], [4, 5, 0]], dtype=complex)
    b = np.array([1, 2, 3], dtype=complex)
    assert np.allclose(oracle.lu_solve(A, b), np.linalg.solve(A, b), atol=1e-14)
    A2 = np.array([[1e-30, 1], [1, 1]], dtype=complex)  # needs the row swap to be accurate
    assert np.allclose(oracle.lu_solve(A2, b[:2]), np.linalg.solve(A2, b[:2]), atol=1e-14)
    with pytest.raises(ZeroDivisionError):
        oracle.lu_solve(np.array([[1, 2], [2, 4]], dtype=complex), b[:2])


def test_newton_quadratic_at_planted_root(oracle_lib):
    """Constant terms shifted so that f(x*) = 0 (f(x*) from sympy); Newton
    with the oracle's evaluation and solve converges quadratically."""
    rng = np.random.default_rng(14)
    s = W.dense_system(3, [2, 3, 2], rng)
    xstar = _rand_point(rng, 3, 0.8)
    xs, eqs = _sympy_system(s)
    f_star, _ = _sympy_eval(xs, eqs, xstar)
    for i in range(3):
        const = int(s.eq_ptr[i])  # graded-lex order: the constant term comes first
        assert s.exps[const].sum() == 0
        s.coeff[const] -= f_star[i]
    x = xstar + 1e-2 * _rand_point(rng, 3)
    errs = [np.abs(x - xstar).max()]
    for _ in range(5):
        f, J = oracle.eval_system(s, x)
        x = x - oracle.lu_solve(J, f)
        errs.append(np.abs(x - xstar).max())
    assert errs[-1] < 1e-13
    for a, b in zip(errs[:3], errs[1:4]):
        if a > 1e-9:
            assert b <= 50 * a * a


def test_start_point_mixed_radix(oracle_lib):
    d = [2, 3, 4]
    for p in range(24):
        x = oracle.start_point(d, p)
        k = [p % 2, (p // 2) % 3, (p // 6) % 4]
        assert np.allclose(x, [np.exp(2j * np.pi * k[i] / d[i]) for i in range(3)], atol=1e-15)


def _match_sets(a, b, rel=1e-8):
    """Every point of a has exactly one point of b within rel, and vice versa."""
    if len(a) != len(b):
        return False
    used = np.zeros(len(b), bool)
    for p in a:
        d = np.abs(b - p).max(axis=1)
        j = int(np.argmin(np.where(used, np.inf, d)))
        if used[j] or d[j] > rel * max(1.0, np.abs(p).max()):
            return False
        used[j] = True
    return True


@pytest.mark.parametrize("d", [1, 2, 5, 8])
def test_track_univariate_matches_roots(oracle_lib, d):
    s, poly = W.univariate(d, np.random.default_rng(20 + d))
    e, st, _, pairs = oracle.solve(s, 0.6 - 0.8j)
    assert (st == oracle.CONVERGED).all() and len(pairs) == 0
    assert _match_sets(e, np.roots(poly).reshape(-1, 1))


def _decoupled_path(a, b, gamma, d, x0, ts):
    """Closed-form path of gamma(1-t)(x^d - 1) + t(a x^d - b) = 0 per
    coordinate: x(t)^d = (gamma(1-t) + t b)/(gamma(1-t) + t a), followed
    continuously from x0 over the grid ts."""
    out, x = [], x0.copy()
    for t in ts:
        r = (gamma * (1 - t) + t * b) / (gamma * (1 - t) + t * a)
        new = np.empty_like(x)
        for i in range(len(x)):
            cands = r[i] ** (1.0 / d[i]) * np.exp(2j * np.pi * np.arange(d[i]) / d[i])
            new[i] = cands[np.argmin(np.abs(cands - x[i]))]
        x = new
        out.append(x.copy())
    return out


def test_rk4_predictor_order_on_closed_form_path(oracle_lib):
    """Local error of the predictor against the exact path is O(h^5): halving
    h divides it by about 32.  Pins the tangent dx/dt = -J^{-1} H_t (its
    sign, H_t = f - gamma g) and the RK4 weights, which the corrector would
    otherwise hide."""
    degs = [3, 2]
    s, a, b = W.decoupled(degs, np.random.default_rng(22))
    gamma = np.exp(0.9j)
    t0 = 0.3
    x0 = np.array([np.exp(2j * np.pi / 3), -1.0 + 0j])
    grid = np.linspace(0, t0, 3001)
    xt0 = _decoupled_path(a, b, gamma, degs, x0, grid)[-1]
    errs = []
    for h in (0.01, 0.005, 0.0025):
        fine = np.linspace(t0, t0 + h, 401)
        exact = _decoupled_path(a, b, gamma, degs, xt0, fine)[-1]
        errs.append(np.abs(oracle.rk4_predict(s, gamma, xt0, t0, h) - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 24 < r1 < 40 and 24 < r2 < 40, errs


def test_step_control_on_linear_paths(oracle_lib):
    """Linear equations: every step is accepted, so the step sizes follow
    the control rule exactly: 0.01 three times, doubled after every three
    accepts (0.02, 0.04, 0.08), capped at h_max = 0.1, the last step clipped
    to end at t = 1 -> 3+3+3+3+5+1 = 18 steps."""
    s, a, b = W.decoupled([1, 1, 1], np.random.default_rng(23))
    e, st, stats = oracle.track_paths(s, np.exp(0.5j), n_paths=1)
    assert st[0] == oracle.CONVERGED
    assert stats["steps"][0] == 18 and stats["rejections"][0] == 0
    assert np.allclose(e[0], b / a, atol=1e-13)


def test_track_decoupled_closed_form(oracle_lib):
    degs = [2, 3, 1, 2]
    s, a, b = W.decoupled(degs, np.random.default_rng(21))
    e, st, _, _ = oracle.solve(s, np.exp(0.7j))
    assert (st == oracle.CONVERGED).all()
    import itertools
    roots = [(b[i] / a[i]) ** (1 / degs[i]) * np.exp(2j * np.pi * np.arange(degs[i]) / degs[i])
             for i in range(len(degs))]
    exact = np.array(list(itertools.product(*roots)))
    assert _match_sets(e, exact)


@pytest.mark.parametrize("n,degs", [(3, [2, 3, 2]), (4, [2, 2, 3, 2]), (6, [2, 2, 2, 2, 2, 3])])
def test_track_linear_products_closed_form(oracle_lib, n, degs):
    """f_i = prod_k (l_ik . x - beta_ik): every solution solves one n x n
    linear system, one factor per equation."""
    import itertools
    s, Ls, betas = W.linear_products(n, degs, np.random.default_rng(30 + n))
    exact = []
    for choice in itertools.product(*[range(d) for d in degs]):
        M = np.array([Ls[i][choice[i]] for i in range(n)])
        r = np.array([betas[i][choice[i]] for i in range(n)])
        exact.append(np.linalg.solve(M, r))
    e, st, _, pairs = oracle.solve(s, np.exp(1.1j), n_threads=4)
    assert (st == oracle.CONVERGED).sum() == int(np.prod(degs))
    assert _match_sets(e[st == 0], np.array(exact))


def test_dense_small_bezout(oracle_lib):
    """Generic dense system: exactly prod d_i = 32 finite regular solutions,
    all reached, residual <= 1e-10, pairwise distinct."""
    wl = W.dense_small()
    s = wl.systems[0]
    assert s.n_terms == 5 * W.n_terms_dense(5, 2) == 105
    e, st, stats, pairs = oracle.solve(s, wl.gammas[0])
    assert (st == oracle.CONVERGED).sum() == 32
    assert (stats["residual"] <= 1e-10).all()
    assert len(oracle.find_duplicates(e, st, rel=1e-6)) == 0


def test_cyclic2_closed_form(oracle_lib):
    rng = np.random.default_rng(40)
    s = W.cyclic_system(2, rng)
    a1, a2 = s.coeff[0], s.coeff[1]
    c = -s.coeff[3]
    e, st, _, _ = oracle.solve(s, np.exp(0.3j))
    assert (st == 0).sum() == 2
    x1 = np.sqrt(-a2 * c / a1) * np.array([1, -1])
    exact = np.stack([x1, -a1 * x1 / a2], axis=1)
    assert _match_sets(e, exact)


def test_cyclic3_by_elimination(oracle_lib):
    """Eliminate x1 (linear equation) and x3 by a resultant computed with
    symbolic coefficients: a univariate polynomial in x2 whose roots
    (numpy.roots) give every solution."""
    rng = np.random.default_rng(41)
    s = W.cyclic_system(3, rng)
    x1, x2, x3 = sp.symbols("x1 x2 x3")
    a1, a2, a3, b1, b2, b3, c = sp.symbols("a1 a2 a3 b1 b2 b3 c")
    e1 = a1 * x1 + a2 * x2 + a3 * x3
    e2 = b1 * x1 * x2 + b2 * x2 * x3 + b3 * x3 * x1
    e3 = x1 * x2 * x3 - c
    x1_expr = -(a2 * x2 + a3 * x3) / a1
    p2 = sp.expand(sp.numer(sp.together(e2.subs(x1, x1_expr))))
    p3 = sp.expand(sp.numer(sp.together(e3.subs(x1, x1_expr))))
    res = sp.Poly(sp.resultant(p2, p3, x3), x2)
    # generator layout: equation k has terms i = 0..2 with support starting at x_{i+1}
    vals = {a1: s.coeff[0], a2: s.coeff[1], a3: s.coeff[2],
            b1: s.coeff[3], b2: s.coeff[4], b3: s.coeff[5], c: -s.coeff[7]}
    assert tuple(s.exps[5]) == (1, 0, 1)  # x3 x1
    num = lambda e, extra={}: complex(sp.N(e.subs({**vals, **extra}), 25))
    coeffs = [num(cf) for cf in res.all_coeffs()]
    lead = next(i for i, cf in enumerate(coeffs) if abs(cf) > 1e-12)
    sols = []
    for r2 in np.roots(coeffs[lead:]):
        if abs(r2) < 1e-8:
            continue  # x2 = 0 cannot satisfy x1 x2 x3 = c
        q = sp.Poly(p2.subs(x2, r2), x3)
        cands = np.roots([num(cf) for cf in q.all_coeffs()])
        f3 = [abs(num(p3, {x2: r2, x3: cc})) for cc in cands]
        r3 = cands[int(np.argmin(f3))]
        sols.append([num(x1_expr, {x2: r2, x3: r3}), r2, r3])
    sols = np.array(sols)
    e, st, _, _ = oracle.solve(s, np.exp(2.1j))
    assert (st == 0).sum() == len(sols) == 6
    assert _match_sets(e[st == 0], sols, rel=1e-7)


def test_embedded_cyclic4_paper_example(oracle_lib):
    """Example 2.1: E_1(f(x), z_1) has 20 solutions, 4 with z_1 = 0 (generic
    points on the degree-4 curve of cyclic 4-roots).  24 total-degree paths."""
    gold = json.load(open(os.path.join(HERE, "golden", "embedded_cyclic4.json")))
    wl = W.embedded_cyclic4_workload()
    s = wl.systems[0]
    assert s.bezout() == 24
    e, st, stats, pairs = oracle.solve(s, wl.gammas[0])
    conv = e[st == oracle.CONVERGED]
    assert len(conv) == gold["solutions"]
    assert len(pairs) == 0
    zero = conv[np.abs(conv[:, 4]) <= 1e-8]
    assert len(zero) == gold["zero_slack_solutions"] == gold["curve_degree"]
    # those four satisfy cyclic 4-roots (unit coefficients) and the hyperplane
    for x in zero[:, :4]:
        x1, x2, x3, x4 = x
        cyc = [x1 + x2 + x3 + x4, x1 * x2 + x2 * x3 + x3 * x4 + x4 * x1,
               x1 * x2 * x3 + x2 * x3 * x4 + x3 * x4 * x1 + x4 * x1 * x2, x1 * x2 * x3 * x4 - 1]
        assert np.abs(cyc).max() < 1e-9
        hyp = s.coeff[s.eq_ptr[4]:s.eq_ptr[5]]
        assert abs(hyp[0] + hyp[1:5] @ x) < 1e-9


def test_cyclic12_bezout_count():
    gold = json.load(open(os.path.join(HERE, "golden", "bezout_counts.json")))
    s = W.cyclic_system(12, np.random.default_rng(0))
    assert s.bezout() == gold["cyclic12_bezout"] == math.factorial(12)
    assert W.cyclic8().total_paths == 40320


def test_gamma_invariance_cyclic5(oracle_lib):
    """The finite solution set does not depend on gamma."""
    s = W.cyclic_system(5, np.random.default_rng(50))
    e1, s1, _, p1 = oracle.solve(s, np.exp(0.4j), n_threads=4)
    e2, s2, _, p2 = oracle.solve(s, np.exp(2.9j), n_threads=4)
    c1, c2 = e1[s1 == 0], e2[s2 == 0]
    assert len(p1) == len(p2) == 0
    assert len(c1) == len(c2) == 70  # cyclic 5-roots: 70 isolated solutions
    assert _match_sets(c1, c2)


def test_forced_failure_statuses(oracle_lib):
    wl = W.dense_small()
    s = wl.systems[0]
    t = oracle.default_tolerances(max_steps=1)
    _, st, _ = oracle.track_paths(s, wl.gammas[0], n_paths=4, tol=t)
    assert (st == oracle.FAILED_MAXSTEPS).all()
    t = oracle.default_tolerances(h_min=0.5, h_init=0.3)
    _, st, _ = oracle.track_paths(s, wl.gammas[0], n_paths=4, tol=t)
    assert (st == oracle.FAILED_MINSTEP).all()
    t = oracle.default_tolerances(div_radius=1e-3)
    _, st, _ = oracle.track_paths(s, wl.gammas[0], n_paths=4, tol=t)
    assert (st == oracle.DIVERGED).all()


def test_work_crew_matches_single_thread(oracle_lib):
    wl = W.cyclic_workload(6, 9)
    s = wl.systems[0]
    e1, s1, st1 = oracle.track_paths(s, wl.gammas[0], n_paths=720, n_threads=1)
    e8, s8, st8 = oracle.track_paths(s, wl.gammas[0], n_paths=720, n_threads=8)
    assert np.array_equal(s1, s8) and np.array_equal(e1, e8)
    assert np.array_equal(st1["steps"], st8["steps"])


def _linear_product_roots(n, degs, Ls, betas):
    import itertools
    out = []
    for choice in itertools.product(*[range(d) for d in degs]):
        M = np.array([Ls[i][choice[i]] for i in range(n)])
        r = np.array([betas[i][choice[i]] for i in range(n)])
        out.append(np.linalg.solve(M, r))
    return np.array(out)


@pytest.mark.parametrize("n,degs", [(3, [2, 3, 2]), (5, [2, 2, 1, 3, 2])])
def test_general_start_system_linear_products(oracle_lib, n, degs):
    """Coefficient-parameter continuation: from the solved system g (a linear
    product system, start points = its closed-form roots) to another linear
    product system f of the same degrees.  Every path converges and the
    endpoints are f's closed-form roots."""
    g, Lg, bg = W.linear_products(n, degs, np.random.default_rng(60 + n))
    f, Lf, bf = W.linear_products(n, degs, np.random.default_rng(70 + n))
    start = _linear_product_roots(n, degs, Lg, bg)
    e, st, _ = oracle.track_paths(f, np.exp(0.4j), start=start, g=g, n_threads=4)
    assert (st == oracle.CONVERGED).all()
    assert _match_sets(e, _linear_product_roots(n, degs, Lf, bf))


def test_general_start_system_univariate(oracle_lib):
    """n = 1: from the roots of one random quintic to the roots of another
    (numpy.roots, companion eigenvalues)."""
    g, pg = W.univariate(5, np.random.default_rng(81))
    f, pf = W.univariate(5, np.random.default_rng(82))
    start = np.roots(pg).reshape(-1, 1)
    e, st, _ = oracle.track_paths(f, np.exp(2.2j), start=start, g=g)
    assert (st == oracle.CONVERGED).all()
    assert _match_sets(e, np.roots(pf).reshape(-1, 1))


def test_explicit_start_points_total_degree(oracle_lib):
    """Total-degree start system with the start points passed in (a shuffled
    subset of the roots of unity) tracks the same paths as the decoded ids."""
    wl = W.dense_small()
    s, gam = wl.systems[0], wl.gammas[0]
    ids = np.array([7, 0, 31, 12, 5], np.int64)
    degs = s.degrees()
    start = np.array([[np.exp(2j * np.pi * ((p // int(np.prod(degs[:i]))) % degs[i]) / degs[i])
                       for i in range(s.n)] for p in ids])
    e1, s1, _ = oracle.track_paths(s, gam, path_ids=ids)
    e2, s2, _ = oracle.track_paths(s, gam, start=start)
    assert (s1 == s2).all()
    assert np.abs(e1 - e2).max() <= 1e-12


def _lp_roots(n, degs, Ls, betas):
    import itertools
    out = []
    for choice in itertools.product(*[range(d) for d in degs]):
        M = np.array([Ls[i][choice[i]] for i in range(n)])
        r = np.array([betas[i][choice[i]] for i in range(n)])
        out.append(np.linalg.solve(M, r))
    return np.array(out)


@pytest.mark.parametrize("seed", [41, 42])
def test_duplicate_post_pass_recovers_jumped_paths(oracle_lib, seed):
    """Linear products of three linear forms in 4 unknowns: 81 closed-form
    roots.  Tracked with loose tolerances (h_max = 1, tol_corr = 0.3) several
    paths jump onto roots that other paths reach too; the post-pass finds
    those pairs and re-tracks both paths of each with h_max = 0.01 and
    tol_corr = 1e-10, after which the endpoint set is exactly the 81
    closed-form roots and no pair is left.  Re-tracking only one path of
    each pair, or re-tracking with the loose tolerances, leaves pairs and
    misses roots on these inputs."""
    n, degs = 4, [3, 3, 3, 3]
    s, Ls, betas = W.linear_products(n, degs, np.random.default_rng(seed))
    exact = _lp_roots(n, degs, Ls, betas)
    g = 1j * np.exp(0.3j)
    tol = oracle.default_tolerances(h_max=1.0, tol_corr=0.3)
    e0, s0, _ = oracle.track_paths(s, g, n_paths=81, tol=tol, n_threads=4)
    pairs = oracle.find_duplicates(e0, s0)
    assert len(pairs) >= 5  # the loose tracking jumps
    assert not _match_sets(e0[s0 == 0], exact)
    e, st, _, rem = oracle.solve(s, g, n_threads=4, tol=tol)
    assert len(rem) == 0
    assert (st == 0).sum() == 81
    assert _match_sets(e[st == 0], exact)
    # paths outside the pairs keep their first endpoints
    keep = np.setdiff1d(np.arange(81), np.unique(pairs.ravel()))
    assert np.array_equal(e[keep], e0[keep])


def test_find_duplicates_reports_exactly_the_planted_pairs(oracle_lib):
    """Near-copies planted at relative distance 3e-7 (a duplicate at the
    1e-6 test) and 5e-6 (not one), among well separated random points; paths
    that did not converge are ignored."""
    rng = np.random.default_rng(5)
    n, P = 4, 600
    x = (rng.standard_normal((P, n)) + 1j * rng.standard_normal((P, n))) * 3
    st = np.zeros(P, np.int32)
    st[::9] = 2
    planted = set()
    for k in range(0, P // 2, 17):  # sources and copies disjoint: no chains
        j = k + P // 2
        close = k % 2 == 1
        x[j] = x[k] * (1 + (3e-7 if close else 5e-6))
        if close and st[j] == 0 and st[k] == 0:
            planted.add((min(j, k), max(j, k)))
    got = {tuple(int(v) for v in p) for p in oracle.find_duplicates(x, st)}
    assert got == planted and len(planted) >= 5


def test_gamma_invariance_cyclic8(oracle_lib):
    """The cyclic-8 workload (40,320 paths) with its gamma and with another:
    the same number of finite endpoints, matched one to one within 1e-8."""
    import sys
    sys.path.insert(0, HERE)
    from parity import match_sets
    wl = W.cyclic8()
    s, g = wl.systems[0], complex(wl.gammas[0])
    nt = os.cpu_count() or 1
    e1, s1, _ = oracle.track_paths(s, g, n_paths=s.bezout(), n_threads=nt)
    e2, s2, _ = oracle.track_paths(s, np.exp(2j * np.pi * 0.377), n_paths=s.bezout(), n_threads=nt)
    c1, c2 = e1[s1 == 0], e2[s2 == 0]
    assert len(c1) == len(c2)
    assert match_sets(c1, c2)
