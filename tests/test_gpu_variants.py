"""Every kernel variant (group kernels: n lanes per path; lane kernels: one
path per lane, Jacobian in LDS; kernels specialised to the system at run
time: one path per lane, Jacobian in registers) against the CPU oracle on
the same seeded inputs, in batched and plain mode."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity, assert_residuals

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
GROUP = [4, 8, 10, 12]
LANES = [100 + n for n in range(1, 9)] + [207, 208]
SPEC = [300 + n for n in range(1, 11)]
DENSE = [400, 411, 412]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_03807_amd as hp
    c = hp.Context(0)
    yield c
    c.close()


CASES = {
    "dense5": lambda: (W.dense_small().systems[0], complex(W.dense_small().gammas[0])),
    "cyclic4": lambda: (W.cyclic_workload(4, 41).systems[0], complex(W.cyclic_workload(4, 41).gammas[0])),
    "cyclic6": lambda: (W.cyclic_workload(6, 9).systems[0], complex(W.cyclic_workload(6, 9).gammas[0])),
    "cyclic7": lambda: (W.cyclic_workload(7, 7).systems[0], complex(W.cyclic_workload(7, 7).gammas[0])),
    "dense3_d3": lambda: (W.dense_system(3, [3, 3, 2], np.random.default_rng(33)), 0.6 + 0.8j),
    "dense8_d2": lambda: (W.dense_system(8, [2] * 8, np.random.default_rng(34)), np.exp(0.3j)),
    # a linear, a quadratic and a cubic equation (every block of the dense table)
    "dense3_d123": lambda: (W.dense_system(3, [1, 2, 3], np.random.default_rng(35)), np.exp(1.1j)),
    "dense11_d2": lambda: (W.dense_system(11, [2] * 11, np.random.default_rng(36)), np.exp(0.9j)),
    # the largest instantiations of the dense kernel, with cubic equations
    "dense9_d23": lambda: (W.dense_system(9, [2, 3, 2, 2, 3, 2, 2, 2, 3], np.random.default_rng(38)),
                           np.exp(0.7j)),
    "dense10_d3": lambda: (W.dense_system(10, [3, 2, 2, 3, 2, 2, 2, 3, 2, 3],
                                          np.random.default_rng(39)), np.exp(2.1j)),
    "dense11_d23": lambda: (W.dense_system(11, [3, 2, 2, 2, 3, 2, 2, 2, 2, 2, 3],
                                           np.random.default_rng(40)), np.exp(1.7j)),
    "cyclic9": lambda: (W.cyclic_workload(9, 42).systems[0], complex(W.cyclic_workload(9, 42).gammas[0])),
}
# cases tracked in full on the GPU but compared with the oracle on a stride
# sample of this many paths (the oracle would take minutes on all of them)
SAMPLE = {"dense10_d3": 2000, "dense11_d23": 2000, "cyclic9": 20000}
# which variants run a case: the large cases only on their default kernels
ONLY = {"dense9_d23": {400, 10}, "dense10_d3": {400, 10}, "dense11_d23": {411, 12},
        "cyclic9": {309, 10}}
_oracle_cache = {}


def sample_ids(name, s):
    P = s.bezout()
    return W.stride_sample(P, SAMPLE[name]) if name in SAMPLE else np.arange(P)


def oracle_ref(name, s, g):
    if name not in _oracle_cache:
        _oracle_cache[name] = oracle.track_paths(s, g, path_ids=sample_ids(name, s),
                                                 n_threads=NTHREADS)
    return _oracle_cache[name]


def run_variant(ctx, s, g, code, mode):
    import torch
    import paper_1804_03807_amd as hp
    plan = ctx.plan(s, g)
    plan.set_variant(code)
    P = s.bezout()
    e, st, sts = plan.outputs(P)
    plan.track_device(e, st, sts, mode=mode)
    torch.cuda.synchronize()
    t = ctx.last_timing()
    out = (hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), hp.Plan.stats_to_numpy(sts))
    plan.close()
    return out, t


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("code", GROUP + LANES + SPEC + DENSE)
def test_variant_matches_oracle(ctx, name, code):
    s, g = CASES[name]()
    if name in ONLY and code not in ONLY[name]:
        pytest.skip("large case: run on its default kernels only")
    if code in DENSE:
        if (s.n > 10 if code == 400 else s.n != code - 400) or max(s.degrees()) > 3:
            pytest.skip("dense kernel 400: n <= 10; 411, 412: n = 11, 12; total degree <= 3")
    elif (code >= 100 and code % 100 != s.n) or code % 100 < s.n:
        pytest.skip("variant not compiled for this n")
    log(f"case {name} n={s.n} paths={s.bezout()} variant={code}")
    (e, st, sts), t = run_variant(ctx, s, g, code, "batched")
    assert t["variant"] == code
    ids = sample_ids(name, s)
    e_o, s_o, _ = oracle_ref(name, s, g)
    assert_parity(e[ids], st[ids], e_o, s_o, f"{name} / {code}", s, ids, log)
    assert_residuals(s, e, st)
    assert (sts["residual"][st == 0] <= 1e-10).all()


@pytest.mark.parametrize("name,code", [("cyclic4", 104), ("cyclic6", 106), ("dense8_d2", 208),
                                       ("cyclic6", 306), ("dense8_d2", 308)])
def test_lane_plain_equals_batched(ctx, name, code):
    s, g = CASES[name]()
    (e1, s1, t1), _ = run_variant(ctx, s, g, code, "batched")
    (e2, s2, t2), tp = run_variant(ctx, s, g, code, "plain")
    assert tp["launches"] > 1
    assert np.array_equal(s1, s2)
    assert np.array_equal(e1, e2)
    assert np.array_equal(t1["steps"], t2["steps"])


def test_unknown_variant_rejected(ctx):
    import paper_1804_03807_amd as hp
    s, g = CASES["cyclic6"]()
    plan = ctx.plan(s, g)
    for bad in (5, 104, 108, 207, 300, 305, 309, 311, 400, 410, 411, 413, -1):
        with pytest.raises(hp.HomotopyError):
            plan.set_variant(bad)
    plan.close()


def test_autotune_chooses_a_valid_variant(ctx, tmp_path, monkeypatch):
    """tune=1 times every candidate variant on a sample, keeps the fastest,
    records it in $HP_TUNE_CACHE; a second plan reads the cache; the tuned
    plan's results match the oracle."""
    import torch
    import paper_1804_03807_amd as hp
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HP_TUNE_CACHE", str(cache))
    s, g = CASES["cyclic6"]()
    plan = ctx.plan(s, g, tune=True)
    P = s.bezout()
    e, st, sts = plan.outputs(P)
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    t = ctx.last_timing()
    code = t["variant"]
    choice = plan.tuning()
    log(f"autotuned variant {code}, choice {choice}")
    assert code in GROUP + LANES + SPEC + DENSE
    assert code < 100 or code % 100 == s.n
    assert choice["variant"] == code and choice["cached"] == 0 and choice["candidates"] >= 4
    assert choice["paths_per_wave"] == t["paths_per_wave"]
    assert choice["waves_per_simd"] == t["waves_per_simd"]
    assert choice["lanes_per_path"] == t["lanes_per_path"] == (s.n if code < 100 else 1)
    assert 0 < choice["ms"] <= choice["ms_default"]
    text = cache.read_text().split()  # key, variant, paths per wavefront (0: 64), waves per SIMD
    assert len(text) == 4 and int(text[1]) == code and int(text[3]) == choice["waves_per_simd"]
    e_o, s_o, _ = oracle_ref("cyclic6", s, g)
    assert_parity(hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), e_o, s_o, "autotuned", s)
    plan.close()
    plan2 = ctx.plan(s, g, tune=True)  # cached: same choice
    e2, st2, _ = plan2.outputs(P)
    plan2.track_device(e2, st2)
    torch.cuda.synchronize()
    assert ctx.last_timing()["variant"] == code
    assert plan2.tuning()["cached"] == 1
    plan2.close()


@pytest.mark.parametrize("name", ["cyclic6", "dense8_d2", "dense11_d2"])
def test_launch_shape_keeps_results(ctx, name):
    """The autotuner's launch shapes (32 of 64 lanes holding paths, a cap of
    one wavefront per SIMD) leave every path's result bit for bit as it is:
    paths are tracked independently."""
    import torch
    import paper_1804_03807_amd as hp
    s, g = CASES[name]()
    P = s.bezout()
    plan = ctx.plan(s, g)
    if name != "cyclic6":
        plan.set_variant(400 if s.n <= 10 else 400 + s.n)
    ref = None
    for lp, wps in [(0, 0), (32, 0), (0, 1), (48, 1), (32, 2)]:
        plan.set_launch(lp, wps)
        e, st, sts = plan.outputs(P)
        plan.track_device(e, st, sts)
        torch.cuda.synchronize()
        t = ctx.last_timing()
        assert t["paths_per_wave"] == (lp or 64) and t["waves_per_simd"] == wps
        out = (hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), sts.cpu().numpy().tobytes())
        if ref is None:
            ref = out
            continue
        assert np.array_equal(out[0].view(np.float64), ref[0].view(np.float64)), (lp, wps)
        assert np.array_equal(out[1], ref[1]) and out[2] == ref[2], (lp, wps)
    with pytest.raises(hp.HomotopyError):
        plan.set_launch(65, 0)
    with pytest.raises(hp.HomotopyError):
        plan.set_launch(0, -1)
    plan.set_variant(GROUP[1] if s.n <= 8 else GROUP[-1])
    with pytest.raises(hp.HomotopyError):
        plan.set_launch(32, 0)  # group kernels: paths per wavefront fixed by n
    plan.close()


def test_tune_batch(ctx, tmp_path, monkeypatch):
    """hp_tune_batch times the variants that run a whole batch with every
    launch shape and caches the fastest; hp_track_batch on that batch then
    launches with it, and its results match the untuned launch's."""
    monkeypatch.setenv("HP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    rng = np.random.default_rng(606)
    systems = [W.dense_system(int(n), [2] * int(n), rng) for n in rng.integers(3, 8, size=24)]
    gammas = W.unit_circle(rng, len(systems))
    ref = ctx.track_batch(systems, gammas)
    t_ref = ctx.last_timing()
    choice = ctx.tune_batch(systems, gammas)
    log(f"untuned variant {t_ref['variant']}; batch choice {choice}")
    assert choice["candidates"] >= 4 and choice["cached"] == 0
    assert choice["variant"] in GROUP + [400]
    out = ctx.track_batch(systems, gammas)
    t = ctx.last_timing()
    assert t["variant"] == choice["variant"]
    assert t["paths_per_wave"] == choice["paths_per_wave"]
    assert t["waves_per_simd"] == choice["waves_per_simd"]
    same_kernel = choice["variant"] == t_ref["variant"]
    for k, (s, (e, st, _), (e0, st0, _)) in enumerate(zip(systems, out, ref)):
        if same_kernel:
            assert np.array_equal(e.view(np.float64), e0.view(np.float64)) and np.array_equal(st, st0)
        else:
            assert_parity(e, st, e0, st0, f"batch system {k}", s)


@pytest.mark.parametrize("name", ["cyclic6", "dense8_d2"])
def test_plan_default_is_specialised(ctx, name):
    """Without tuning, a plan for n <= 10 runs on the kernel specialised to
    its system (variant 300 + n), 64 paths per wavefront."""
    import torch
    s, g = CASES[name]()
    plan = ctx.plan(s, g)
    e, st, sts = plan.outputs(s.bezout())
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    t = ctx.last_timing()
    assert t["variant"] == 300 + s.n
    assert t["paths_per_wave"] == 64
    plan.close()


def test_dense12_sampled(ctx):
    """The n = 12 dense kernel (412, the default for such a system) on a
    serving-size system of mixed degrees: a stride sample of 2,000 paths
    against the oracle, every converged endpoint through the oracle's
    residual gate."""
    import torch
    import paper_1804_03807_amd as hp
    rng = np.random.default_rng(37)
    s = W.dense_system(12, rng.integers(2, 4, size=12), rng)
    g = np.exp(0.4j)
    P = s.bezout()
    plan = ctx.plan(s, g)
    e, st, sts = plan.outputs(P)
    plan.track_device(e, st, sts)
    torch.cuda.synchronize()
    assert ctx.last_timing()["variant"] == 412
    e, st, sts = hp.Plan.endpoints_to_numpy(e), st.cpu().numpy(), hp.Plan.stats_to_numpy(sts)
    plan.close()
    sample = W.stride_sample(P, 2000)
    log(f"dense12 paths={P} sample={len(sample)}")
    e_o, s_o, _ = oracle.track_paths(s, g, path_ids=sample, n_threads=NTHREADS)
    assert_parity(e[sample], st[sample], e_o, s_o, "dense12 / 412", s, sample, log)
    assert_residuals(s, e, st)
