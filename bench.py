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
    return {"value": len(ids) / dt, "unit": "paths/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}-th path id ({len(ids)} of {total} paths), "
                      f"{threads} threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cyclic8", choices=sorted(WORKLOADS))
    ap.add_argument("--waves", type=int, default=0, help="force a kernel variant (waves/group)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", action="store_true")
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
    plan = ctx.plan(system, gamma, tune=args.tune)
    if args.waves:
        plan.set_variant(args.waves)
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
                                      "waves_per_group": timing["waves_per_group"],
                                      "groups": timing["groups"]}},
        "converged": int(conv.sum()),
        "not_converged": int((~conv).sum()),
        "residual_gate_ok": resid_ok,
        "latency_ms": {"p50": float(np.percentile(times, 50)),
                       "p99": float(np.percentile(times, 99))},
        "kernel_ms_mean": kmean,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
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

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(system, gamma)

    print(json.dumps(out), flush=True)
    plan.close()
    ctx.close()


if __name__ == "__main__":
    main()
