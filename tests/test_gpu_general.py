"""General start systems and explicit start points through the C ABI
(hp_track_paths with g and start): the problem statement's
track_paths(system, start_solutions, gamma, tolerances), including
coefficient-parameter continuation, against closed forms and the oracle."""
import itertools
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import REL, assert_parity, assert_residuals, close_rows

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_03807_amd as hp
    c = hp.Context(0)
    yield c
    c.close()


def lp_roots(n, degs, Ls, betas):
    out = []
    for choice in itertools.product(*[range(d) for d in degs]):
        M = np.array([Ls[i][choice[i]] for i in range(n)])
        r = np.array([betas[i][choice[i]] for i in range(n)])
        out.append(np.linalg.solve(M, r))
    return np.array(out)


def match_sets(a, b):
    if len(a) != len(b):
        return False
    used = np.zeros(len(b), bool)
    for p in a:
        d = np.abs(b - p).max(axis=1)
        d[used] = np.inf
        j = int(np.argmin(d))
        if not d[j] <= REL * max(1.0, np.abs(b[j]).max()):
            return False
        used[j] = True
    return True


@pytest.mark.parametrize("mode", ["batched", "plain"])
@pytest.mark.parametrize("n,degs", [(3, [2, 3, 2]), (5, [2, 2, 1, 3, 2])])
def test_linear_product_continuation(ctx, n, degs, mode):
    g, Lg, bg = W.linear_products(n, degs, np.random.default_rng(60 + n))
    f, Lf, bf = W.linear_products(n, degs, np.random.default_rng(70 + n))
    start = lp_roots(n, degs, Lg, bg)
    gam = np.exp(0.4j)
    log(f"case linear-product continuation n={n} paths={len(start)} mode={mode}")
    e, st, sts = ctx.track_paths(f, gam, start=start, g=g, mode=mode)
    assert (st == 0).all()
    assert match_sets(e, lp_roots(n, degs, Lf, bf))
    e_o, s_o, _ = oracle.track_paths(f, gam, start=start, g=g, n_threads=NTHREADS)
    assert_parity(e, st, e_o, s_o, f"linear products n={n}", f)
    assert_residuals(f, e, st)


def test_univariate_continuation(ctx):
    g, pg = W.univariate(5, np.random.default_rng(81))
    f, pf = W.univariate(5, np.random.default_rng(82))
    e, st, _ = ctx.track_paths(f, np.exp(2.2j), start=np.roots(pg).reshape(-1, 1), g=g)
    assert (st == 0).all()
    assert match_sets(e, np.roots(pf).reshape(-1, 1))


def test_explicit_start_points_total_degree(ctx):
    """Start points passed in (a shuffled subset of the roots of unity) give
    the paths of the decoded ids."""
    wl = W.dense_small()
    s, gam = wl.systems[0], complex(wl.gammas[0])
    e_all, s_all, st_all = ctx.track_paths(s, gam)
    ids = np.array([7, 0, 31, 12, 5, 5], np.int64)
    degs = s.degrees()
    start = np.array([[np.exp(2j * np.pi * ((p // int(np.prod(degs[:i]))) % degs[i]) / degs[i])
                       for i in range(s.n)] for p in ids])
    e, st, sts = ctx.track_paths(s, gam, start=start)
    assert (st == s_all[ids]).all()
    assert close_rows(e, e_all[ids], 1e-12).all()


def test_parameter_continuation_cyclic5(ctx):
    """Solve one random-coefficient cyclic-5 system, then move its 70 finite
    roots to those of another system on the same supports (generic: all 70
    paths converge); the endpoint set equals the total-degree solution of
    the target, and every path matches the oracle."""
    a = W.cyclic_workload(5, 50)
    b = W.cyclic_workload(5, 51)
    sa, sb = a.systems[0], b.systems[0]
    ea, sta, _ = ctx.track_paths(sa, complex(a.gammas[0]))
    start = ea[sta == 0]
    assert len(start) == 70
    gam = np.exp(1.3j)
    e, st, sts = ctx.track_paths(sb, gam, start=start, g=sa)
    log(f"  converged {int((st == 0).sum())} of {len(start)}")
    assert (st == 0).all()
    eb, stb, _ = ctx.track_paths(sb, complex(b.gammas[0]))
    assert match_sets(e, eb[stb == 0])
    e_o, s_o, _ = oracle.track_paths(sb, gam, start=start, g=sa, n_threads=NTHREADS)
    assert_parity(e, st, e_o, s_o, "cyclic5 continuation", sb)
    assert_residuals(sb, e, st)


def test_general_argument_errors(ctx):
    import paper_1804_03807_amd as hp
    from paper_1804_03807_amd import _lib
    s = W.dense_small().systems[0]
    g = W.dense_system(4, [2] * 4, np.random.default_rng(1))
    with pytest.raises(hp.HomotopyError):  # different n
        ctx.track_paths(s, 1j, start=np.ones((2, 5), complex), g=g)
    with pytest.raises(hp.HomotopyError):  # non-finite start point
        ctx.track_paths(s, 1j, start=np.full((1, 5), np.nan + 0j))
    v = hp._SysView(s)
    ends = np.zeros((1, 5), complex)
    stat = np.zeros(1, np.int32)
    tol = hp.default_tolerances()
    rc = _lib.load().hp_track_paths(ctx.handle, hp.ctypes.byref(v.c), hp.ctypes.byref(v.c), None, 1,
                                    hp._c64(1j), hp.ctypes.byref(tol), hp._ptr(ends), hp._ptr(stat),
                                    None, hp.HP_BATCHED)
    assert rc == _lib.HP_E_INVALID_ARG  # g without start points


def _continuation_case(ctx, n, seed_a, seed_b):
    """The finite roots of one random system on the cyclic-n supports (solved
    by total degree on the GPU) as start points for another such system."""
    a = W.cyclic_workload(n, seed_a)
    b = W.cyclic_workload(n, seed_b)
    sa, sb = a.systems[0], b.systems[0]
    ea, sta, _ = ctx.track_paths(sa, complex(a.gammas[0]))
    return sa, sb, ea[sta == 0]


@pytest.mark.parametrize("n,seeds", [(5, (50, 51)), (7, (52, 53))])
def test_parameter_continuation_specialised_kernel(ctx, n, seeds):
    """A plan for a start system on f's support (hp_plan_create_general) runs
    the specialised kernel's coefficient-parameter form (variant 300 + n):
    every path matches the oracle's continuation and the group kernels'
    continuation (hp_track_paths) to the parity bar, batched and plain
    results are bitwise equal, and the residual gate holds by the oracle's
    evaluator."""
    import torch
    import paper_1804_03807_amd as hp
    sa, sb, start = _continuation_case(ctx, n, *seeds)
    gam = complex(np.exp(1.3j))
    plan = ctx.plan(sb, gam, g=sa, start=start)
    P = len(start)
    out = {}
    for mode in ("batched", "plain"):
        e, st, sts = plan.outputs(P)
        plan.track_device(e, st, sts, mode=mode)
        torch.cuda.synchronize()
        t = ctx.last_timing()
        assert t["variant"] == 300 + n, (mode, t)
        out[mode] = (hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), hp.Plan.stats_to_numpy(sts))
    plan.close()
    e, st, sts = out["batched"]
    assert np.array_equal(e.view(np.float64), out["plain"][0].view(np.float64))
    assert np.array_equal(st, out["plain"][1])
    log(f"  cyclic-{n} continuation: converged {int((st == 0).sum())} of {P}")
    e_o, s_o, _ = oracle.track_paths(sb, gam, start=start, g=sa, n_threads=NTHREADS)
    assert_parity(e, st, e_o, s_o, f"cyclic{n} continuation (specialised)", sb)
    e_g, s_g, _ = ctx.track_paths(sb, gam, start=start, g=sa)
    assert ctx.last_timing()["variant"] < 100
    assert_parity(e, st, e_g, s_g, f"cyclic{n} continuation (specialised vs group)", sb)
    assert_residuals(sb, e, st)


def test_general_plan_other_support_runs_group_kernels(ctx):
    """A general plan whose start system has another support (linear
    products of other degrees per equation) takes the group kernels, and
    matches the oracle."""
    import torch
    import paper_1804_03807_amd as hp
    n = 3
    g, Lg, bg = W.linear_products(n, [2, 2, 3], np.random.default_rng(63))
    f, Lf, bf = W.linear_products(n, [2, 3, 2], np.random.default_rng(73))
    start = lp_roots(n, [2, 2, 3], Lg, bg)
    gam = complex(np.exp(0.4j))
    plan = ctx.plan(f, gam, g=g, start=start)
    e, st, sts = plan.outputs(len(start))
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    assert ctx.last_timing()["variant"] < 100
    plan.close()
    e_o, s_o, _ = oracle.track_paths(f, gam, start=start, g=g, n_threads=NTHREADS)
    assert_parity(hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), e_o, s_o, "linear products", f)
