"""The double-double tracker on the GPU (hp_track_paths_dd) against the
oracle's double-double tracker on the same inputs: identical converged /
not-converged outcomes, and converged endpoints (hi + lo) that agree within
1e-20 relative (both run the final Newton to 1e-26); against 50-digit roots
for a univariate system; and the high parts equal the double tracker's
endpoints, which its end game rounds to the nearest double of the root."""
import os
import sys

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
REL_DD = 1e-20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_03807_amd as hp
    c = hp.Context(0)
    yield c
    c.close()


def dd_close(hi_a, lo_a, hi_b, lo_b, rel=REL_DD):
    d = np.abs((hi_a - hi_b) + (lo_a - lo_b)).max(axis=1)
    return d <= rel * np.maximum(1.0, np.abs(hi_b).max(axis=1))


CASES = {
    "dense5": lambda: (W.dense_small().systems[0], complex(W.dense_small().gammas[0]), None),
    "cyclic5": lambda: (W.cyclic_workload(5, 50).systems[0],
                        complex(W.cyclic_workload(5, 50).gammas[0]), None),
    "dense8_d2": lambda: (W.dense_system(8, [2] * 8, np.random.default_rng(34)), np.exp(0.3j), None),
    "cyclic7": lambda: (W.cyclic_workload(7, 7).systems[0], complex(W.cyclic_workload(7, 7).gammas[0]),
                        700),
    "dense11_d2": lambda: (W.dense_system(11, [2] * 11, np.random.default_rng(36)), np.exp(0.9j), 300),
}


@pytest.mark.parametrize("name", list(CASES))
def test_dd_tracker_matches_oracle(ctx, name):
    s, g, sample = CASES[name]()
    P = s.bezout()
    log(f"case {name} n={s.n} paths={P}")
    hi, lo, st, sts = ctx.track_paths_dd(s, g)
    t = ctx.last_timing()
    log(f"  kernel {t['kernel_ms']:.2f} ms, converged {int((st == 0).sum())} of {P}")
    ids = np.arange(P) if sample is None else W.stride_sample(P, sample)
    ho, lo_o, so, _ = oracle.track_paths_dd(s, g, path_ids=ids, n_threads=NTHREADS)
    assert np.array_equal(st[ids] == 0, so == 0), np.nonzero((st[ids] == 0) != (so == 0))[0][:8]
    both = (st[ids] == 0) & (so == 0)
    ok = dd_close(hi[ids][both], lo[ids][both], ho[both], lo_o[both])
    assert ok.all(), ids[both][~ok][:8]
    assert (sts["residual"][st == 0] <= 1e-20).all()
    # the high parts are the nearest doubles of the roots: the double
    # tracker's endpoints (where it converges as well)
    e, sd, _ = ctx.track_paths(s, g)
    c = (sd == 0) & (st == 0)
    log(f"  high parts equal to the double tracker's endpoints: {int((hi[c] == e[c]).all(axis=1).sum())} of {int(c.sum())}")
    assert (hi[c] == e[c]).all(axis=1).mean() >= 0.99


def test_dd_univariate_roots_to_28_digits(ctx):
    mpmath.mp.dps = 50
    s, poly = W.univariate(8, np.random.default_rng(28))
    hi, lo, st, _ = ctx.track_paths_dd(s, 0.6 - 0.8j)
    assert (st == 0).all()
    roots = mpmath.polyroots([mpmath.mpc(c.real, c.imag) for c in poly], maxsteps=300,
                             extraprec=300)
    for h, l in zip(hi[:, 0], lo[:, 0]):
        x = mpmath.mpc(h.real, h.imag) + mpmath.mpc(l.real, l.imag)
        assert min(abs(x - r) / max(1, abs(r)) for r in roots) <= 1e-28
