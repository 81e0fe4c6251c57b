"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Every path has the same converged / not-converged
outcome on both sides (identical counts), converged endpoints match within
1e-8 relative (||x_gpu - x_ref||_inf <= 1e-8 max(1, ||x_ref||_inf)), and
every converged GPU endpoint passes the residual gate evaluated by the
oracle.  Sub-statuses of non-converged paths (diverged / failed) are
reported, not gated: in affine coordinates a path to a point at infinity may
stop on the divergence radius or on the minimum step depending on
rounding."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity, assert_residuals, match_sets

pytestmark = pytest.mark.gpu

REL = 1e-8
NTHREADS = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_03807_amd as hp
    c = hp.Context(0)
    yield c
    c.close()


def check_against_oracle(ctx, system, gamma, mode="batched", ids_sample=None):
    log(f"case {system.name} n={system.n} paths={system.bezout()} mode={mode}")
    e_g, s_g, st_g = ctx.track_paths(system, gamma, mode=mode)
    if ids_sample is None:
        ids_sample = np.arange(system.bezout())
    e_o, s_o, st_o = oracle.track_paths(system, gamma, path_ids=ids_sample, n_threads=NTHREADS)
    assert_parity(e_g[ids_sample], s_g[ids_sample], e_o, s_o, system.name, system, ids_sample,
                  log)
    assert_residuals(system, e_g, s_g)
    return e_g, s_g, st_g, e_o, s_o, st_o


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_dense_small_all_converge(ctx, mode):
    wl = W.dense_small()
    s = wl.systems[0]
    e_g, s_g, st_g, e_o, s_o, _ = check_against_oracle(ctx, s, wl.gammas[0], mode)
    assert (s_g == 0).sum() == (s_o == 0).sum() == 32
    assert (st_g["residual"] <= 1e-10).all()
    assert match_sets(e_g[s_g == 0], e_o[s_o == 0])


def test_plain_and_batched_agree_bitwise(ctx):
    wl = W.cyclic_workload(6, 9)
    s = wl.systems[0]
    e1, s1, st1 = ctx.track_paths(s, wl.gammas[0], mode="batched")
    e2, s2, st2 = ctx.track_paths(s, wl.gammas[0], mode="plain")
    assert np.array_equal(s1, s2)
    assert np.array_equal(e1, e2)
    assert np.array_equal(st1["steps"], st2["steps"])


def test_embedded_cyclic4_paper_example(ctx):
    wl = W.embedded_cyclic4_workload()
    s = wl.systems[0]
    e_g, s_g, _, e_o, s_o, _ = check_against_oracle(ctx, s, wl.gammas[0])
    conv = e_g[s_g == 0]
    assert len(conv) == 20
    assert int((np.abs(conv[:, 4]) <= 1e-8).sum()) == 4
    assert match_sets(conv, e_o[s_o == 0])


@pytest.mark.parametrize("d", [1, 3, 8])
def test_univariate_roots(ctx, d):
    s, poly = W.univariate(d, np.random.default_rng(20 + d))
    e, st, _ = ctx.track_paths(s, 0.6 - 0.8j)
    assert (st == 0).all()
    assert match_sets(e, np.roots(poly).reshape(-1, 1))
    assert_residuals(s, e, st)


def test_linear_products_closed_form(ctx):
    import itertools
    n, degs = 6, [2, 2, 2, 2, 2, 3]
    s, Ls, betas = W.linear_products(n, degs, np.random.default_rng(36))
    exact = []
    for choice in itertools.product(*[range(d) for d in degs]):
        M = np.array([Ls[i][choice[i]] for i in range(n)])
        r = np.array([betas[i][choice[i]] for i in range(n)])
        exact.append(np.linalg.solve(M, r))
    e, st, _ = ctx.track_paths(s, np.exp(1.1j))
    assert (st == 0).sum() == int(np.prod(degs))
    assert match_sets(e[st == 0], np.array(exact))
    assert_residuals(s, e, st)


@pytest.mark.parametrize("n,seed", [(5, 50), (6, 9), (7, 7)])
def test_cyclic_small_full_parity(ctx, n, seed):
    wl = W.cyclic_workload(n, seed)
    s = wl.systems[0]
    e_g, s_g, _, e_o, s_o, _ = check_against_oracle(ctx, s, wl.gammas[0])
    assert (s_g == 0).sum() == (s_o == 0).sum()
    assert match_sets(e_g[s_g == 0], e_o[s_o == 0])


def test_cyclic8_full_parity(ctx):
    """The benchmark workload: 40320 paths, every path against the oracle."""
    wl = W.cyclic8()
    s = wl.systems[0]
    e_g, s_g, st_g, e_o, s_o, st_o = check_against_oracle(ctx, s, wl.gammas[0])
    assert (s_g == 0).sum() == (s_o == 0).sum()
    assert match_sets(e_g[s_g == 0], e_o[s_o == 0])
    assert (st_g["residual"][s_g == 0] <= 1e-10).all()
    assert len(oracle.find_duplicates(e_g, s_g)) == 0


def _spec_plan_run(ctx, s, g):
    import torch
    import paper_1804_03807_amd as hp
    plan = ctx.plan(s, g)
    e, st, sts = plan.outputs(s.bezout())
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    variant = ctx.last_timing()["variant"]
    out = hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), hp.Plan.stats_to_numpy(sts)
    plan.close()
    return out, variant


def test_cyclic8_full_parity_specialised_plan(ctx):
    """The benchmark's configuration: a plan for the cyclic-8 workload runs on
    the kernel specialised to its support (variant 308, one persistent
    launch); all 40320 paths against the oracle."""
    wl = W.cyclic8()
    s, g = wl.systems[0], complex(wl.gammas[0])
    log(f"case cyclic8 specialised plan paths={s.bezout()}")
    (e_g, s_g, st_g), variant = _spec_plan_run(ctx, s, g)
    assert variant == 308
    e_o, s_o, st_o = oracle.track_paths(s, g, n_paths=s.bezout(), n_threads=NTHREADS)
    assert_parity(e_g, s_g, e_o, s_o, "cyclic8 / 308", s, log=log)
    assert_residuals(s, e_g, s_g)
    assert (st_g["residual"][s_g == 0] <= 1e-10).all()
    assert len(oracle.find_duplicates(e_g, s_g)) == 0


def test_cyclic8_gamma_invariance(ctx):
    """A second gamma moves every path but not the finite endpoint set: the
    GPU's converged endpoints with gamma' equal the oracle's with gamma (same
    count, matched one to one within 1e-8)."""
    wl = W.cyclic8()
    s, g = wl.systems[0], complex(wl.gammas[0])
    g2 = complex(np.exp(2j * np.pi * 0.377))
    log("case cyclic8 gamma invariance")
    (e2, s2, _), _ = _spec_plan_run(ctx, s, g2)
    e_o, s_o, _ = oracle.track_paths(s, g, n_paths=s.bezout(), n_threads=NTHREADS)
    log(f"  converged gamma'={int((s2 == 0).sum())} oracle(gamma)={int((s_o == 0).sum())}")
    assert (s2 == 0).sum() == (s_o == 0).sum()
    assert match_sets(e2[s2 == 0], e_o[s_o == 0])


def test_ids_list_matches_direct(ctx):
    import torch
    import paper_1804_03807_amd as hp
    wl = W.cyclic_workload(6, 9)
    s = wl.systems[0]
    ids = np.array([5, 700, 3, 3, 100, 719, 0], np.int64)
    plan = ctx.plan(s, wl.gammas[0])
    ea, sa, _ = plan.outputs(s.bezout())
    plan.track_device(ea, sa)  # every path, in id order
    e, st, sts = plan.outputs(len(ids))
    dids = torch.from_numpy(ids).cuda()
    plan.track_device(e, st, sts, ids=dids)
    torch.cuda.synchronize()
    e1, s1 = hp.Plan.endpoints_to_numpy(ea), sa.cpu().numpy()
    assert np.array_equal(st.cpu().numpy(), s1[ids])
    assert np.array_equal(hp.Plan.endpoints_to_numpy(e), e1[ids])
    plan.close()


def test_forced_failure_statuses(ctx):
    import paper_1804_03807_amd as hp
    wl = W.dense_small()
    s = wl.systems[0]
    _, st, _ = ctx.track_paths(s, wl.gammas[0], tol=hp.default_tolerances(max_steps=1))
    assert (st == hp.FAILED_MAXSTEPS).all()
    _, st, _ = ctx.track_paths(s, wl.gammas[0], tol=hp.default_tolerances(h_min=0.5, h_init=0.3))
    assert (st == hp.FAILED_MINSTEP).all()
    _, st, _ = ctx.track_paths(s, wl.gammas[0], tol=hp.default_tolerances(div_radius=1e-3))
    assert (st == hp.DIVERGED).all()


def test_invalid_arguments_raise(ctx):
    import paper_1804_03807_amd as hp
    s = W.cyclic_system(12, np.random.default_rng(0))
    bad = W.PolySystem(13, np.zeros(14, np.int32), np.zeros(0, np.complex128),
                       np.zeros((0, 13), np.uint8))
    with pytest.raises(hp.HomotopyError):
        ctx.track_paths(bad, 1.0, n_paths=1)
    with pytest.raises(hp.HomotopyError):
        ctx.track_paths(s, 0.0, n_paths=1)  # gamma must be nonzero
    e, st, _ = ctx.track_paths(W.dense_small().systems[0], 1j, n_paths=0)
    assert e.shape == (0, 5)


def test_context_destroyed_before_its_plan():
    """The C library keeps a context alive until its last plan is gone: a
    plan still tracks after its context was destroyed, and destroying it
    afterwards releases both."""
    import torch
    import paper_1804_03807_amd as hp
    wl = W.dense_small()
    s, g = wl.systems[0], complex(wl.gammas[0])
    c = hp.Context(0)
    plan = c.plan(s, g)
    c._L.hp_context_destroy(c.handle)  # the context first, directly through the C ABI
    c.handle = None
    e, st, sts = plan.outputs(s.bezout())
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    plan.close()


def test_solve_post_pass_against_oracle(ctx):
    """hp_solve's duplicate post-pass on a case where paths jump (linear
    products, 81 closed-form roots, loose tolerances h_max = 1, tol_corr =
    0.3): the tracking leaves duplicate pairs; hp_solve keeps every other
    path's endpoint, re-tracks both paths of each pair with h_max = 0.01 and
    tol_corr = 1e-10 exactly as the oracle does, and reports the pairs left,
    which the oracle's scan confirms."""
    import torch
    import paper_1804_03807_amd as hp
    n, degs = 4, [3, 3, 3, 3]
    s, Ls, betas = W.linear_products(n, degs, np.random.default_rng(41))
    g = 1j * np.exp(0.3j)
    tol = hp.default_tolerances(h_max=1.0, tol_corr=0.3)
    plan = ctx.plan(s, g, tol=tol)  # the kernel hp_solve runs
    e, st, sts = plan.outputs(81)
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    e0, s0 = hp.Plan.endpoints_to_numpy(e), st.cpu().numpy()
    plan.close()
    pairs = hp.find_duplicates(e0, s0)
    log(f"  loose tracking: {len(pairs)} duplicate pairs")
    assert len(pairs) > 0
    e1, s1, _, rem = ctx.solve(s, g, tol=tol)
    idx = np.unique(pairs.ravel())
    keep = np.setdiff1d(np.arange(81), idx)
    assert np.array_equal(e1[keep], e0[keep]) and np.array_equal(s1[keep], s0[keep])
    t2 = oracle.default_tolerances(h_max=0.01, tol_corr=1e-10)
    e_o, s_o, _ = oracle.track_paths(s, g, path_ids=idx.astype(np.int64), tol=t2,
                                     n_threads=NTHREADS)
    assert_parity(e1[idx], s1[idx], e_o, s_o, "re-tracked pairs", s, idx, log)
    assert rem == len(oracle.find_duplicates(e1, s1))
    # every converged endpoint is a distinct closed-form root (the loose
    # tracking itself may lose a path, so the set can be smaller than 81)
    import itertools
    exact = []
    for choice in itertools.product(*[range(d) for d in degs]):
        M = np.array([Ls[i][choice[i]] for i in range(n)])
        r = np.array([betas[i][choice[i]] for i in range(n)])
        exact.append(np.linalg.solve(M, r))
    exact = np.array(exact)
    hit = set()
    for x in e1[s1 == 0]:
        d = np.abs(exact - x).max(axis=1)
        j = int(np.argmin(d))
        assert d[j] <= 1e-8 * max(1.0, np.abs(exact[j]).max())
        hit.add(j)
    log(f"  after the post-pass: {int((s1 == 0).sum())} converged, {len(hit)} distinct roots")
    assert len(hit) == int((s1 == 0).sum()) - rem


def test_device_duplicate_scan_matches_host(ctx):
    """hp_find_duplicates_device reports the same pairs as the host scan
    (and the oracle's O(N^2) scan) on planted near-copies."""
    import torch
    import paper_1804_03807_amd as hp
    rng = np.random.default_rng(5)
    n, P = 6, 20000
    x = (rng.standard_normal((P, n)) + 1j * rng.standard_normal((P, n))) * 3
    st = np.zeros(P, np.int32)
    st[::9] = 2
    for k in range(0, P // 2, 97):
        x[k + P // 2] = x[k] * (1 + (3e-7 if k % 2 else 5e-6))
    ref = {tuple(int(v) for v in p) for p in hp.find_duplicates(x, st)}
    e_d = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    s_d = torch.from_numpy(st).cuda()
    pairs, found = ctx.find_duplicates_device(e_d, s_d, 1e-6, max_pairs=1 << 12)
    got = {tuple(int(v) for v in p) for p in pairs.cpu().numpy()}
    log(f"  pairs host {len(ref)} device {found}")
    assert found == len(ref) == len(got) and got == ref and len(ref) > 10
    sub = np.arange(0, P, 7)  # the oracle's scan on a subset
    assert {tuple(int(v) for v in p) for p in oracle.find_duplicates(x[sub], st[sub])} == \
        {tuple(int(v) for v in p) for p in hp.find_duplicates(x[sub], st[sub])}
    # max_pairs smaller than the number found: the count is still exact
    pairs2, found2 = ctx.find_duplicates_device(e_d, s_d, 1e-6, max_pairs=3)
    assert found2 == found and len(pairs2) == 3
