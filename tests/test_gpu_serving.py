"""GPU tests of the serving loop (hp_server_*): continuous batching of solve
requests of different sizes, admitted by HBM budget.

* every request's result in the mix equals its result alone (the request
  served by itself), endpoint by endpoint within 1e-8 relative and with
  identical statuses; each request runs on the kernel family it gets alone
  (its specialised kernel, the dense kernel or a group kernel);
* a request whose outputs exceed the budget is tracked chunk by chunk and
  still equals the whole-system result; the arena never exceeds the budget;
* sampled paths of mixed requests match the CPU oracle."""
import os
import sys
import threading
import time

import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
SLOT_BYTES = 12 * 16 + 4 + 40  # endpoint slot of the widest system + status + stats


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_03807_amd as hp
    c = hp.Context(0)
    yield c
    c.close()


def small_requests(count, max_paths):
    out = []
    rid = 0
    while len(out) < count:
        s, g = W.serving_request(rid)
        if s.bezout() <= max_paths:
            out.append((rid, s, g))
        rid += 1
    return out


def served_alone(ctx, s, g):
    """The request's result from a server that holds nothing else."""
    import paper_1804_03807_amd as hp
    srv = hp.Server(ctx, 1 << 30)
    try:
        e, st, sts, _ = srv.wait(srv.submit(s, g), stats=True)
        return e, st, sts
    finally:
        srv.close()


def assert_same(res, ref, what):
    """res, ref: (endpoints, status, stats) of the same request."""
    assert_parity(res[0], res[1], ref[0], ref[1], what)


def test_alone_equals_mix(ctx):
    import paper_1804_03807_amd as hp
    reqs = small_requests(12, 6000)
    log("requests", [(r, s.name, s.bezout()) for r, s, _ in reqs])
    alone = {r: served_alone(ctx, s, g) for r, s, g in reqs}
    srv = hp.Server(ctx, 1 << 30)
    try:
        ids = [(r, srv.submit(s, g)) for r, s, g in reqs]
        bitwise = 0
        for r, q in ids:
            e, st, sts, lat = srv.wait(q, stats=True)
            assert lat > 0
            assert_same((e, st, sts), alone[r], f"request {r}")
            bitwise += int(np.array_equal(e, alone[r][0]))
        log(f"bitwise-identical requests: {bitwise}/{len(ids)}")
        assert srv.peak_bytes() <= 1 << 30
    finally:
        srv.close()


def test_arrivals_during_work_overlap(ctx):
    """Requests submitted from another thread while earlier ones run; all
    complete with the alone result."""
    import paper_1804_03807_amd as hp
    reqs = small_requests(24, 6000)
    alone = {r: served_alone(ctx, s, g) for r, s, g in reqs}
    arr = W.poisson_arrivals(len(reqs), rate=200.0)
    srv = hp.Server(ctx, 1 << 30)
    ids = {}
    try:
        def producer():
            t0 = time.perf_counter()
            for (r, s, g), ta in zip(reqs, arr):
                while time.perf_counter() - t0 < ta:
                    time.sleep(0.0005)
                ids[r] = srv.submit(s, g)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        lats = []
        for r, s, g in reqs:
            e, st, sts, lat = srv.wait(ids[r], stats=True)
            lats.append(lat)
            assert_same((e, st, sts), alone[r], f"request {r}")
        log(f"latency ms p50={np.percentile(lats, 50):.2f} p99={np.percentile(lats, 99):.2f}")
    finally:
        srv.close()


def test_over_budget_request_is_chunked(ctx):
    """Budget holds ~8.9k path slots; cyclic-8 (40320 paths) must run in
    chunks beside a small request and equal the whole-system result."""
    import paper_1804_03807_amd as hp
    wl = W.cyclic8()
    sys8, g8 = wl.systems[0], complex(wl.gammas[0])
    ref8 = served_alone(ctx, sys8, g8)
    (r1, s1, g1), = small_requests(1, 1000)
    ref1 = served_alone(ctx, s1, g1)
    budget = 2 * 1000 * 1000
    srv = hp.Server(ctx, budget)
    try:
        q8 = srv.submit(sys8, g8)
        q1 = srv.submit(s1, g1)
        e, st, sts, _ = srv.wait(q8, stats=True)
        assert_same((e, st, sts), ref8, "cyclic8 chunked")
        e, st, sts, _ = srv.wait(q1, stats=True)
        assert_same((e, st, sts), ref1, "small request beside chunks")
        peak = srv.peak_bytes()
        log(f"peak resident bytes {peak} budget {budget}")
        assert 0 < peak <= budget
    finally:
        srv.close()


def test_budget_too_small_rejected(ctx):
    import paper_1804_03807_amd as hp
    with pytest.raises(hp.HomotopyError):
        hp.Server(ctx, 1024)


def test_mix_matches_oracle_sample(ctx):
    import paper_1804_03807_amd as hp
    reqs = small_requests(6, 6000)
    srv = hp.Server(ctx, 1 << 30)
    try:
        ids = [(srv.submit(s, g), s, g) for _, s, g in reqs]
        for q, s, g in ids:
            e, st, sts, _ = srv.wait(q, stats=True)
            sample = W.stride_sample(s.bezout(), 64)
            e_o, s_o, _ = oracle.track_paths(s, g, path_ids=sample, n_threads=NTHREADS)
            assert_parity(e[sample], st[sample], e_o, s_o, s.name, s, sample, log)
    finally:
        srv.close()


def test_sliced_equals_unsliced_bitwise(ctx):
    """With a budget of 4 steps per wavefront and epoch, paths of the
    specialised and dense kernel families are suspended to their slots and
    resumed in later epochs many times over; every request still ends bit for
    bit (endpoints, statuses, every counter) as when each queue runs to the
    end."""
    import paper_1804_03807_amd as hp
    reqs = small_requests(10, 6000)
    log("requests", [(r, s.name, s.bezout()) for r, s, _ in reqs])
    ref = {}
    srv = hp.Server(ctx, 1 << 30)
    try:
        srv.set_slice(0.0, 0)
        for r, s, g in reqs:
            ref[r] = srv.wait(srv.submit(s, g), stats=True)
        assert srv.info()["carried"] == 0
    finally:
        srv.close()
    srv = hp.Server(ctx, 1 << 30)
    try:
        srv.set_slice(0.0, 4)
        ids = [(r, srv.submit(s, g)) for r, s, g in reqs]
        for r, q in ids:
            e, st, sts, _ = srv.wait(q, stats=True)
            e0, st0, sts0, _ = ref[r]
            assert np.array_equal(st, st0), f"request {r}: statuses differ"
            assert np.array_equal(e.view(np.float64), e0.view(np.float64)), f"request {r}: endpoints"
            for k in ("steps", "rejections", "newton_iters", "evals", "solves", "t_final",
                      "residual"):
                assert np.array_equal(sts[k], sts0[k]), f"request {r}: stats {k}"
        info = srv.info()
        log("sliced server", info)
        assert info["fixed_steps"] == 4 and info["epochs"] > 10 and info["carried"] > 0
    finally:
        srv.close()


def test_adaptive_slice_bounds_epochs(ctx):
    """The adaptive step budget keeps epochs near the slice time: with a 5 ms
    slice, a cyclic-8 request (40,320 paths) runs over many epochs, and a
    small request submitted behind it finishes long before it."""
    import paper_1804_03807_amd as hp
    wl = W.cyclic8()
    sys8, g8 = wl.systems[0], complex(wl.gammas[0])
    (r1, s1, g1), = small_requests(1, 1000)
    ref1 = served_alone(ctx, s1, g1)
    srv = hp.Server(ctx, 1 << 30)
    try:
        srv.set_slice(5.0, 0)
        q8 = srv.submit(sys8, g8)
        time.sleep(0.05)
        q1 = srv.submit(s1, g1)
        e, st, sts, lat1 = srv.wait(q1, stats=True)
        assert_same((e, st, sts), ref1, "small request behind cyclic-8")
        _, st8, _, lat8 = srv.wait(q8, stats=True)
        info = srv.info()
        log(f"latency small {lat1:.1f} ms, cyclic-8 {lat8:.1f} ms; {info}")
        assert (st8 == 0).sum() > 0
        assert info["epochs"] > 5 and info["budget_max"] > 0
        assert lat1 < lat8
    finally:
        srv.close()


def test_submit_does_not_compile(ctx):
    """A request on a support not seen before returns from submit at once;
    its specialised kernel compiles on the server's own thread."""
    import paper_1804_03807_amd as hp
    rng = np.random.default_rng(20261203)
    s = W.embed(W.cyclic_system(5, rng), 1, rng, name="embedded_cyclic5")
    g = complex(W.unit_circle(rng))
    srv = hp.Server(ctx, 1 << 30)
    try:
        t0 = time.perf_counter()
        q = srv.submit(s, g)
        t_submit = time.perf_counter() - t0
        e, st, sts, lat = srv.wait(q, stats=True)
        log(f"submit {t_submit * 1e3:.1f} ms, request latency {lat:.0f} ms")
        assert t_submit < 0.5
        sample = W.stride_sample(s.bezout(), 48)
        e_o, s_o, _ = oracle.track_paths(s, g, path_ids=sample, n_threads=NTHREADS)
        assert_parity(e[sample], st[sample], e_o, s_o, s.name, s, sample, log)
    finally:
        srv.close()


def test_families_and_tolerances_mixed(ctx):
    """One server holds a request on the group kernels (a dense system of
    degree 4 with 1,638 factors: too many for a specialised kernel, too high
    a degree for the dense ones), one on a specialised
    kernel, one on the dense kernel, and one with other tolerances (served
    in epochs of its own), under a 4-step slice that is switched to the
    adaptive one half way; every result equals the request served alone
    with slicing off, bit for bit."""
    import paper_1804_03807_amd as hp
    rng = np.random.default_rng(1203)
    reqs = [
        (W.dense_system(6, [4, 4, 4, 2, 2, 2], rng), complex(np.exp(0.3j)), None),
        (W.cyclic_system(6, rng), complex(np.exp(1.1j)), None),
        (W.dense_system(4, [2, 3, 2, 2], rng), complex(np.exp(2.2j)), None),
        (W.cyclic_system(5, rng), complex(np.exp(0.7j)), hp.default_tolerances(tol_corr=1e-9)),
    ]
    ref = []
    for s, g, tol in reqs:
        srv = hp.Server(ctx, 1 << 30)
        try:
            srv.set_slice(0.0, 0)
            ref.append(srv.wait(srv.submit(s, g, tol), stats=True))
        finally:
            srv.close()
    srv = hp.Server(ctx, 1 << 30)
    try:
        srv.set_slice(0.0, 4)
        ids = [srv.submit(s, g, tol) for s, g, tol in reqs]
        time.sleep(0.02)
        srv.set_slice(50.0, 0)
        for k, q in enumerate(ids):
            e, st, sts, _ = srv.wait(q, stats=True)
            e0, st0, sts0, _ = ref[k]
            assert np.array_equal(st, st0), f"request {k}: statuses"
            assert np.array_equal(e.view(np.float64), e0.view(np.float64)), f"request {k}: endpoints"
            assert np.array_equal(sts["steps"], sts0["steps"]), f"request {k}: steps"
        log("mixed families", srv.info())
    finally:
        srv.close()


def test_destroy_with_requests_in_flight(ctx):
    """Destroying a server while requests are queued, compiling and running
    returns (the worker and compile threads stop); a new server on the same
    context then serves normally."""
    import paper_1804_03807_amd as hp
    srv = hp.Server(ctx, 1 << 30)
    srv.set_slice(0.0, 4)
    for r, s, g in small_requests(6, 6000):
        srv.submit(s, g)
    rng = np.random.default_rng(77)
    srv.submit(W.embed(W.cyclic_system(6, rng), 1, rng, name="embedded_cyclic6"), 0.6 + 0.8j)
    time.sleep(0.05)
    t0 = time.perf_counter()
    srv.close()
    log(f"destroy took {(time.perf_counter() - t0) * 1e3:.0f} ms")
    (r, s, g), = small_requests(1, 1000)
    srv = hp.Server(ctx, 1 << 30)
    try:
        e, st, sts, _ = srv.wait(srv.submit(s, g), stats=True)
        ref = served_alone(ctx, s, g)
        assert_same((e, st, sts), ref, "after a destroyed server")
    finally:
        srv.close()
