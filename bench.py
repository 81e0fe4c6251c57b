"""Benchmark: paths/s of the batched (persistent) tracker vs the plain
(one launch per step) tracker on one MI355X, with the roofline of the
tracking kernel and the CPU oracle timed on the host beside it.

Workload (default): random-coefficient system on the cyclic-8 supports,
all 8! = 40320 total-degree paths of gamma(1-t)(x^d - 1) + t f, complex
FP64 (seeded, synthetic; stands in for the paper's cyclic 8-roots runs).
A "step" is one solve of the whole system: every path tracked to its end.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk

# HBM bytes per launch of the kernel the bench times (the plan's default:
# the kernel specialised to the cyclic-8 support, variant 308) from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each
# scaled by what the counter reads for a 256 MiB device copy (FETCH_SIZE
# reads half the copied bytes, WRITE_SIZE all of them).  Valid only for the
# kernel sources they were taken on; reported as null once those change.
TRAFFIC_PROFILE = {
    "workload": "cyclic8",
    "variant": 308,
    "sources_sha256": {
        "spec_track.hpp": "bb636574221bdf00805a21bbf4a783b4222c9c83e6ae6b0d1ef22211410816f1",
        "lane_track.hpp": "d88e396d1469da3c3c901e2aaa6170c2cb2c893162686c6fafd3989921cf3ff4",
        "hp_device.hpp": "f785014ca74114e45d5b32364f08af0b41660996c35cbf08085ef6fbc53b0a3e",
        "hp_internal.hpp": "fcdd9f4c568f1d13ef2e0d021aee18cbcf41be765e41d7bf5a60016e6757857e",
        "hp_jit.cpp": "161eb0b1682f3e9c2e6298568b857aa590840c85fd0c98555fde715ce4f31b59",
        "reg_lu.hpp": "488a287cfdfca4d8c1b616ad7aa2ae6bd41dfae4f8f485f55d55bd2819711eb2",
    },
    "fetch_kib": 571.0, "fetch_scale": 262144 / 131093.125,
    "write_kib": 6812.9375, "write_scale": 262144 / 262144,
}

WORKLOADS = {
    "cyclic8": ("cyclic8: random unit-circle coefficients on the cyclic 8-roots supports, "
                "40320 total-degree paths, complex fp64, seed 2"),
    "cyclic10": ("cyclic10: random unit-circle coefficients on the cyclic 10-roots supports, "
                 "3628800 total-degree paths, complex fp64, seed 5"),
    "dense5": "dense5_d2: dense random n=5 quadratics, 32 paths, seed 1",
}


def load_workload(name):
    import workloads as W
    if name == "cyclic8":
        return W.cyclic8()
    if name == "cyclic10":
        return W.cyclic10()
    if name == "dense5":
        return W.dense_small()
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(workload, variant):
    """HBM bytes per launch from the counter profile, or None when the kernel
    sources differ from the profiled ones or the workload or kernel variant
    is another one."""
    import hashlib
    T = TRAFFIC_PROFILE
    if workload != T["workload"] or variant != T["variant"] or not T["sources_sha256"]:
        return None
    csrc = os.path.join(ROOT, "paper_1804_03807_amd", "csrc")
    for name, digest in T["sources_sha256"].items():
        with open(os.path.join(csrc, name), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    return T["fetch_kib"] * 1024 * T["fetch_scale"] + T["write_kib"] * 1024 * T["write_scale"]


def serving_run(ctx, n_requests, budget_bytes, load=0.8):
    """Serving sample: the first n_requests of the seeded request stream.
    Saturated pass (all submitted at once) gives the saturated request rate;
    then a Poisson stream at load x that rate; latency = completion - arrival."""
    import threading
    import paper_1804_03807_amd as hp
    import workloads as W
    reqs = [W.serving_request(i) for i in range(n_requests)]
    paths = sum(s.bezout() for s, _ in reqs)
    # the server runs sparse requests with n <= 10 on the kernel specialised
    # to their support; a deployment compiles its supports ahead (hiprtc,
    # kept for the process), which is timed here apart from the serving runs
    t0 = time.perf_counter()
    for s, _ in reqs:
        if s.n <= 10 and max(s.degrees()) > 3:
            try:
                hp.spec_compile(s)
            except hp.HomotopyError:
                pass  # too large for a specialised kernel: group kernels
    compile_ms = (time.perf_counter() - t0) * 1e3

    def run(arrivals):
        srv = hp.Server(ctx, budget_bytes)
        ids = [None] * len(reqs)
        t0 = time.perf_counter()

        def producer():
            for i, ((s, g), ta) in enumerate(zip(reqs, arrivals)):
                while time.perf_counter() - t0 < ta:
                    time.sleep(0.0002)
                ids[i] = srv.submit(s, g)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        lat, conv = [], 0
        for q in ids:
            _, st, _, ms = srv.wait(q)
            lat.append(ms)
            conv += int((st == 0).sum())
        makespan = time.perf_counter() - t0
        peak = srv.peak_bytes()
        srv.close()
        return np.asarray(lat), makespan, peak, conv

    lat_sat, span_sat, _, _ = run(np.zeros(len(reqs)))
    rate_sat = len(reqs) / span_sat
    lam = load * rate_sat
    lat, span, peak, conv = run(W.poisson_arrivals(len(reqs), lam))
    return {"requests": len(reqs), "paths": paths, "converged": conv,
            "spec_compile_ms": compile_ms,
            "sample": f"request ids 0..{len(reqs) - 1} of the seeded stream (seed 4)",
            "saturated_requests_per_s": rate_sat, "lambda_requests_per_s": lam,
            "paths_per_s": paths / span, "makespan_s": span,
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99))},
            "saturated_latency_ms": {"p50": float(np.percentile(lat_sat, 50)),
                                     "p99": float(np.percentile(lat_sat, 99))},
            "hbm_budget_bytes": budget_bytes, "peak_resident_bytes": peak}


def batch_run(ctx, n_systems=256):
    """Many dense systems (n 3..10, degrees 2..3 per equation, seed 3) in one
    persistent launch with one refill queue per system."""
    import workloads as W
    wl = W.dense_batch(n_systems, seed=3)
    gam = [complex(g) for g in wl.gammas]
    from paper_1804_03807_amd import flops
    ctx.track_batch(wl.systems, gam, stats=False)  # warm-up (code load, tables)
    t0 = time.perf_counter()
    res = ctx.track_batch(wl.systems, gam, stats=True)
    dt = time.perf_counter() - t0
    tm = ctx.last_timing()
    conv = sum(int((st == 0).sum()) for _, st, _ in res)
    flop = sum(flops.run_flops(sy, sts) for sy, (_, _, sts) in zip(wl.systems, res))
    tfs = flop / (tm["kernel_ms"] * 1e-3) / 1e12
    return {"systems": n_systems, "paths": wl.total_paths, "converged": conv,
            "kernel_ms": tm["kernel_ms"], "paths_per_s": wl.total_paths / (tm["kernel_ms"] * 1e-3),
            "end_to_end_ms": dt * 1e3, "kernel_variant": tm["variant"],
            "achieved_tflops": tfs, "frac_of_fp64_peak": tfs / FP64_PEAK_TFLOPS}


def cyclic10_run(ctx):
    """All 10! = 3,628,800 paths of the cyclic-10 supports (seed 5): the
    persistent tracker with divergence truncation, then the duplicate pass."""
    import workloads as W
    import paper_1804_03807_amd as hp
    wl = W.cyclic10()
    s, g = wl.systems[0], complex(wl.gammas[0])
    # the kernel specialised to the support, compiled ahead (hiprtc; kept for
    # the process), so that the timed solve does not include its compilation
    t0 = time.perf_counter()
    hp.spec_compile(s)
    compile_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    e, st, sts, remaining = ctx.solve(s, g)
    dt = time.perf_counter() - t0
    tm = ctx.last_timing()
    from paper_1804_03807_amd import flops
    conv = st == 0
    tfs = flops.run_flops(s, sts) / (dt) / 1e12
    return {"paths": s.bezout(), "converged": int(conv.sum()),
            "achieved_tflops_end_to_end": tfs, "frac_of_fp64_peak_end_to_end": tfs / FP64_PEAK_TFLOPS,
            "diverged": int((st == 1).sum()), "failed": int((st >= 2).sum()),
            "duplicate_pairs_left": remaining,
            "residual_gate_ok": bool((sts["residual"][conv] <= 1e-10).all()),
            "solve_ms": dt * 1e3, "paths_per_s": s.bezout() / dt,
            "kernel_variant": tm["variant"], "spec_compile_ms": compile_ms}


def cpu_baseline(system, gamma, seconds_target=15.0):
    """The oracle as it stands, on a stride sample of path ids, with every
    host thread; extrapolated to paths/s."""
    import oracle
    threads = os.cpu_count() or 1
    total = system.bezout()
    # calibrate on a small sample, then size the main sample to ~seconds_target
    ids = np.arange(0, total, max(1, total // 256), dtype=np.int64)
    t0 = time.perf_counter()
    oracle.track_paths(system, gamma, path_ids=ids, n_threads=threads)
    rate = len(ids) / max(1e-6, time.perf_counter() - t0)
    want = int(min(total, max(len(ids), rate * seconds_target)))
    stride = max(1, total // want)
    ids = np.arange(0, total, stride, dtype=np.int64)
    t0 = time.perf_counter()
    _, st, _ = oracle.track_paths(system, gamma, path_ids=ids, n_threads=threads)
    dt = time.perf_counter() - t0
    # one thread on a sixteenth of the sample
    ids1 = ids[::16]
    t1 = time.perf_counter()
    oracle.track_paths(system, gamma, path_ids=ids1, n_threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": len(ids) / dt, "unit": "paths/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}-th path id ({len(ids)} of {total} paths), "
                      f"{threads} threads, {dt:.1f} s",
            "one_thread_value": len(ids1) / dt1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cyclic8", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", type=int, default=0,
                    help="force a kernel variant code (homotopy.h, hp_plan_set_variant)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=32,
                    help="requests in the serving sample (0: skip)")
    ap.add_argument("--serving-budget-gib", type=float, default=16.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 256-system batch and the cyclic-10 runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device copy (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); paths are independent "
              "and would shard by path-id range across GPUs, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1804_03807_amd as hp
    from paper_1804_03807_amd import flops

    wl = load_workload(args.workload)
    system, gamma = wl.systems[0], complex(wl.gammas[0])
    P = system.bezout()
    ctx = hp.Context(0)
    t0 = time.perf_counter()
    plan = ctx.plan(system, gamma, tune=args.tune)  # compiles the specialised kernel
    plan_ms = (time.perf_counter() - t0) * 1e3
    if args.variant:
        plan.set_variant(args.variant)
    e, st, sts = plan.outputs(P)
    stream = torch.cuda.current_stream()

    def one():
        plan.track_device(e, st, sts, mode="batched", stream=stream)
        return ctx.last_timing()

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    times, kms = [], []
    t_all0 = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        tm = one()
        times.append((time.perf_counter() - t0) * 1e3)
        kms.append(tm["kernel_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all0
    timing = ctx.last_timing()

    status = st.cpu().numpy()
    stats = hp.Plan.stats_to_numpy(sts)
    conv = status == hp.CONVERGED
    resid_ok = bool((stats["residual"][conv] <= 1e-10).all())
    value = P * args.steps / elapsed
    flop = flops.run_flops(system, stats)
    kmean = float(np.mean(kms))
    achieved = flop / (kmean * 1e-3) / 1e12

    out = {
        "metric": "paths/sec at endpoint residual<=1e-10, batched vs plain; p50/p99 solve latency",
        "value": value,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "paths": P, "n": system.n,
                   "mode": "batched (persistent, device refill queue)",
                   "kernel_variant": {"max_n": timing["max_n"],
                                      "paths_per_wave": timing["paths_per_wave"], "code": timing["variant"],
                                      "groups": timing["groups"]},
                   "plan_create_ms": plan_ms},
        "converged": int(conv.sum()),
        "not_converged": int((~conv).sum()),
        "converged_per_s": int(conv.sum()) * args.steps / elapsed,
        "residual_gate_ok": resid_ok,
        "latency_ms": {"p50": float(np.percentile(times, 50)),
                       "p99": float(np.percentile(times, 99))},
        "kernel_ms_mean": kmean,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(args.workload, timing["variant"]),
                     "flops_per_launch": flop},
    }
    if not resid_ok:
        out["value_invalid"] = "a converged endpoint failed the residual gate"

    if not args.no_plain:
        t0 = time.perf_counter()
        plan.track_device(e, st, sts, mode="plain", stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tp = ctx.last_timing()
        out["plain"] = {"value": P / dt, "unit": "paths/s", "launches": tp["launches"],
                        "ms": dt * 1e3}
        out["batched_over_plain"] = value / (P / dt)

    if not args.no_extra:
        out["batch256"] = batch_run(ctx)
        out["cyclic10"] = cyclic10_run(ctx)

    if args.serving_requests > 0:
        out["serving"] = serving_run(ctx, args.serving_requests,
                                     int(args.serving_budget_gib * (1 << 30)))

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(system, gamma)

    print(json.dumps(out), flush=True)
    plan.close()
    ctx.close()


if __name__ == "__main__":
    main()
