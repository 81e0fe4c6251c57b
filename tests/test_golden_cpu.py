"""The stored oracle results (tests/golden/*.npz, written by the committed
scripts beside them that call only the oracle) still agree with the oracle
as it stands: a sample of stored paths is tracked again and must come out
identical (the oracle is deterministic per path)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
C10 = os.path.join(HERE, "golden", "cyclic10_seed5.npz")


@pytest.mark.skipif(not os.path.exists(C10), reason="cyclic-10 golden not written yet")
def test_cyclic10_golden_matches_oracle(oracle_lib):
    z = np.load(C10)
    meta = json.load(open(C10.replace(".npz", ".json")))
    status, conv_ids, conv_x = z["status"], z["conv_ids"], z["conv_x"]
    assert len(status) == 3628800
    assert np.bincount(status, minlength=5).tolist() == meta["status_histogram"]
    assert np.array_equal(np.nonzero(status == 0)[0], conv_ids)
    assert len(conv_x) == meta["converged"]
    wl = W.cyclic10()
    s, g = wl.systems[0], complex(wl.gammas[0])
    ids = np.unique(np.concatenate([W.stride_sample(len(status), 120), conv_ids[::900]]))
    e, st, _ = oracle.track_paths(s, g, path_ids=ids, n_threads=os.cpu_count() or 1)
    assert np.array_equal(st, status[ids].astype(np.int32))
    where = np.searchsorted(conv_ids, ids[st == 0])
    assert np.array_equal(e[st == 0], conv_x[where])
    # every FAILED_MINSTEP path stopped in the end zone
    endzone = np.unpackbits(z["endzone"])[:len(status)].astype(bool)
    assert endzone[status == 2].all()
    assert meta["minstep_min_t_final"] >= 1 - 1e-9
