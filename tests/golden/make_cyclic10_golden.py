"""Writes the oracle's result for every path of the cyclic-10 workload
(random coefficients on the cyclic 10-roots supports, seed 5, 10! = 3,628,800
total-degree paths): the status of each path and the endpoints of the
converged ones, before any duplicate post-pass.

Calls only ``oracle`` and ``workloads``; nothing here comes from the HIP
path.  Takes over an hour on 8 host threads:

    python tests/golden/make_cyclic10_golden.py [n_threads]

Output: ``cyclic10_seed5.npz`` (status int8 per path id, ids and endpoints of
the converged paths, and one bit per path, packed: the path stopped in the end
zone t >= 1 - 1e-9) and ``cyclic10_seed5.json`` (status histogram, the
smallest t at which a FAILED_MINSTEP path stopped, the digest of the oracle
source the values were made with, run time).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CHUNK = 1 << 17


def oracle_digest() -> str:
    h = hashlib.sha256()
    for name in ("oracle.c", "oracle.h"):
        with open(os.path.join(ROOT, "oracle", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def main():
    n_threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.build()
    wl = W.cyclic10()
    s, gamma = wl.systems[0], wl.gammas[0]
    P = s.bezout()
    status = np.zeros(P, np.int8)
    t_final = np.zeros(P, np.float64)
    xnorm = np.zeros(P, np.float64)
    conv_ids, conv_x = [], []
    t0 = time.time()
    for lo in range(0, P, CHUNK):
        ids = np.arange(lo, min(P, lo + CHUNK), dtype=np.int64)
        e, st, stats = oracle.track_paths(s, gamma, path_ids=ids, n_threads=n_threads)
        status[ids] = st
        t_final[ids] = stats["t_final"]
        xnorm[ids] = np.abs(e).max(axis=1)
        c = st == oracle.CONVERGED
        conv_ids.append(ids[c])
        conv_x.append(e[c])
        done = lo + len(ids)
        print(f"{done}/{P} paths, {time.time() - t0:.0f} s, converged so far "
              f"{sum(len(a) for a in conv_ids)}", flush=True)
    conv_ids = np.concatenate(conv_ids)
    conv_x = np.concatenate(conv_x)
    hist = np.bincount(status, minlength=5).tolist()
    write(status, conv_ids, conv_x, t_final, xnorm, hist, n_threads, time.time() - t0)


ENDZONE = 1e-9


def write(status, conv_ids, conv_x, t_final, xnorm, hist, n_threads, seconds):
    np.savez_compressed(os.path.join(HERE, "cyclic10_seed5.npz"), status=status,
                        conv_ids=conv_ids, conv_x=conv_x,
                        endzone=np.packbits(t_final >= 1.0 - ENDZONE))
    ms = status == 2
    meta = {
        "workload": "cyclic-10 supports, random unit-circle coefficients, seed 5; "
                    "total-degree homotopy, 3,628,800 paths, default tolerances",
        "made_by": "tests/golden/make_cyclic10_golden.py (oracle only)",
        "oracle_sha256": oracle_digest(),
        "status_histogram": hist,
        "status_names": ["CONVERGED", "DIVERGED", "FAILED_MINSTEP", "FAILED_MAXSTEPS",
                         "FAILED_NEWTON_T1"],
        "converged": int(hist[0]),
        "endzone": f"t_final >= 1 - {ENDZONE:g}",
        "minstep_min_t_final": float(t_final[ms].min()) if ms.any() else None,
        "minstep_norm_range": [float(xnorm[ms].min()), float(xnorm[ms].max())] if ms.any() else None,
        "n_threads": n_threads,
        "seconds": round(seconds, 1),
    }
    with open(os.path.join(HERE, "cyclic10_seed5.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
