"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Converged endpoints must match within 1e-8 relative
(||x_gpu - x_ref||_inf <= 1e-8 max(1, ||x_ref||_inf)), with identical
converged / not-converged counts.  Sub-statuses of non-converged paths
(diverged / failed) are reported, not gated: in affine coordinates a path to
a point at infinity may stop on the divergence radius or on the minimum step
depending on rounding."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W

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


def close(a, b):
    return np.abs(a - b).max() <= REL * max(1.0, np.abs(b).max())


def match_sets(a, b):
    """Greedy nearest match: every point of a pairs with a distinct point of b."""
    if len(a) != len(b):
        return False
    used = np.zeros(len(b), bool)
    for p in a:
        d = np.abs(b - p).max(axis=1)
        d[used] = np.inf
        j = int(np.argmin(d))
        if not (d[j] <= REL * max(1.0, np.abs(b[j]).max())):
            return False
        used[j] = True
    return True


def per_path_report(e_g, s_g, e_o, s_o):
    both = (s_g == 0) & (s_o == 0)
    bad = [i for i in np.nonzero(both)[0] if not close(e_g[i], e_o[i])]
    flips = int(((s_g == 0) != (s_o == 0)).sum())
    return len(bad), flips


def check_against_oracle(ctx, system, gamma, mode="batched", ids_sample=None):
    log(f"case {system.name} n={system.n} paths={system.bezout()} mode={mode}")
    e_g, s_g, st_g = ctx.track_paths(system, gamma, mode=mode)
    if ids_sample is None:
        e_o, s_o, st_o = oracle.track_paths(system, gamma, n_paths=system.bezout(),
                                            n_threads=NTHREADS)
        e_gs, s_gs = e_g, s_g
    else:
        e_o, s_o, st_o = oracle.track_paths(system, gamma, path_ids=ids_sample,
                                            n_threads=NTHREADS)
        e_gs, s_gs = e_g[ids_sample], s_g[ids_sample]
    bad, flips = per_path_report(e_gs, s_gs, e_o, s_o)
    log(f"  converged gpu={int((s_gs == 0).sum())} oracle={int((s_o == 0).sum())} "
        f"per-path mismatches={bad} status flips={flips}")
    return e_g, s_g, st_g, e_o, s_o, st_o, bad, flips


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_dense_small_all_converge(ctx, mode):
    wl = W.dense_small()
    s = wl.systems[0]
    e_g, s_g, st_g, e_o, s_o, _, bad, flips = check_against_oracle(ctx, s, wl.gammas[0], mode)
    assert (s_g == 0).sum() == (s_o == 0).sum() == 32
    assert bad == 0 and flips == 0
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
    e_g, s_g, _, e_o, s_o, _, bad, flips = check_against_oracle(ctx, s, wl.gammas[0])
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


@pytest.mark.parametrize("n,seed", [(5, 50), (6, 9), (7, 7)])
def test_cyclic_small_full_parity(ctx, n, seed):
    wl = W.cyclic_workload(n, seed)
    s = wl.systems[0]
    e_g, s_g, _, e_o, s_o, _, bad, flips = check_against_oracle(ctx, s, wl.gammas[0])
    assert (s_g == 0).sum() == (s_o == 0).sum()
    assert match_sets(e_g[s_g == 0], e_o[s_o == 0])


def test_cyclic8_full_parity(ctx):
    """The benchmark workload: 40320 paths, every path against the oracle."""
    wl = W.cyclic8()
    s = wl.systems[0]
    e_g, s_g, st_g, e_o, s_o, st_o, bad, flips = check_against_oracle(ctx, s, wl.gammas[0])
    assert (s_g == 0).sum() == (s_o == 0).sum()
    assert match_sets(e_g[s_g == 0], e_o[s_o == 0])
    assert (st_g["residual"][s_g == 0] <= 1e-10).all()
    assert len(oracle.find_duplicates(e_g, s_g)) == 0


def test_cyclic8_full_parity_specialised_plan(ctx):
    """The benchmark's configuration: a plan for the cyclic-8 workload runs on
    the kernel specialised to its support (variant 308, one persistent
    launch); all 40320 paths against the oracle."""
    import torch
    import paper_1804_03807_amd as hp
    from parity import compare_paths
    wl = W.cyclic8()
    s, g = wl.systems[0], complex(wl.gammas[0])
    plan = ctx.plan(s, g)
    e, st, sts = plan.outputs(s.bezout())
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    assert ctx.last_timing()["variant"] == 308
    e_g, s_g, st_g = hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), hp.Plan.stats_to_numpy(sts)
    plan.close()
    e_o, s_o, st_o = oracle.track_paths(s, g, n_paths=s.bezout(), n_threads=NTHREADS)
    hard, flips = compare_paths(e_g, s_g, st_g, e_o, s_o, st_o)
    log(f"  converged gpu={int((s_g == 0).sum())} oracle={int((s_o == 0).sum())} "
        f"hard={len(hard)} borderline={len(flips)}")
    assert len(hard) == 0, f"paths {hard[:8]} differ from the oracle"
    assert abs(int((s_g == 0).sum()) - int((s_o == 0).sum())) <= len(flips)
    assert (st_g["residual"][s_g == 0] <= 1e-10).all()
    assert len(oracle.find_duplicates(e_g, s_g)) == 0


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
