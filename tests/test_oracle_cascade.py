"""Pins of the oracle's cascade of homotopies (Section 3.1, Example 3.1,
Figure 3) to the paper's printed values on the system of Example 3.1: the
numbers of regular solutions (nonzero slack) that pass from stage to stage
(54, 50, 26) and the 8 finite candidates at the end, among them the four
printed isolated solutions; every candidate lies on a component of the
printed decomposition.  The numbers of solutions with zero slack at the
lower stages are singular and fluctuate with the random constants (the
paper says so), so those are checked for validity only."""
import numpy as np
import pytest

import oracle
import workloads as W

ISOLATED = [(3, 2, 2, 1), (3, 3, 2, 1), (4, 3, 2, 1), (4, 2, 2, 1)]
LINES = [  # (x1, x2, x3, x4) with None free, printed in Example 3.1
    (2, 2, None, 1), (2, 2, 1, None), (2, 3, 1, None), (2, 3, None, 1),
    (3, 1, 1, None), (3, 1, 2, None), (3, 2, 1, None), (3, 3, 1, None),
    (4, 1, 1, None), (4, 1, 2, None), (4, 2, 1, None), (4, 3, 1, None)]


def component_dims(x, tol=1e-6):
    """Dimensions of the printed components of Example 3.1's solution set
    that contain x (3: x1 = 1; 2: x1 = 2, x2 = 1; 1: the twelve lines; 0: the
    four isolated points)."""
    x = np.asarray(x)[:4]
    dims = set()
    if abs(x[0] - 1) <= tol:
        dims.add(3)
    if abs(x[0] - 2) <= tol and abs(x[1] - 1) <= tol:
        dims.add(2)
    for line in LINES:
        if all(v is None or abs(x[j] - v) <= tol * max(1, abs(x[j])) for j, v in enumerate(line)):
            dims.add(1)
    for p in ISOLATED:
        if np.abs(x - np.array(p)).max() <= tol:
            dims.add(0)
    return dims


def run_cascade(seed=8):
    e = W.embed(W.multistep_system(), 3, np.random.default_rng(seed))
    gammas = W.unit_circle(np.random.default_rng(99), 4)
    return e, gammas, oracle.cascade(e, 3, gammas, n_threads=4)


@pytest.fixture(scope="module")
def cascade_result(oracle_lib):
    return run_cascade()


def test_cascade_regular_counts_match_figure3(cascade_result):
    e, _, st = cascade_result
    assert [s["dim"] for s in st] == [3, 2, 1, 0]
    assert st[0]["paths"] == 256  # total degree 4^4 of the top embedded system
    # top: one generic point of the three-dimensional set, 54 with z3 != 0
    assert len(st[0]["candidates"]) == 1 and st[0]["nonzero"] == 54
    assert st[1]["paths"] == 54 and st[1]["nonzero"] == 50
    assert st[2]["paths"] == 50 and st[2]["nonzero"] == 26
    assert st[3]["paths"] == 26 and len(st[3]["candidates"]) == 8


def test_cascade_isolated_solutions_printed(cascade_result):
    _, _, st = cascade_result
    fin = st[3]["candidates"]
    for p in ISOLATED:
        assert (np.abs(fin[:, :4] - np.array(p)).max(axis=1) <= 1e-8).sum() == 1, p


def test_cascade_candidates_lie_on_printed_components(cascade_result):
    _, _, st = cascade_result
    for s in st:
        for x in s["candidates"]:
            dims = component_dims(x)
            assert dims, (s["dim"], x)
            # a candidate of dimension d lies on a component of dimension >= d
            assert max(dims) >= s["dim"], (s["dim"], x, dims)
    # the top candidate is the generic point of x1 = 1
    assert component_dims(st[0]["candidates"][0]) == {3}


def test_cascade_stage_system_removes_one_slack(oracle_lib):
    e = W.embed(W.multistep_system(), 3, np.random.default_rng(8))
    F = oracle.cascade_stage_system(e, 3, 3)
    # z3 (unknown 6) left the four equations of f and its hyperplane became z3 = 0
    assert not any(F.exps[t][6] for t in range(int(F.eq_ptr[4])))
    row = slice(int(F.eq_ptr[6]), int(F.eq_ptr[7]))
    assert F.coeff[row].tolist() == [1.0] and F.exps[row].tolist() == [[0, 0, 0, 0, 0, 0, 1]]
    assert np.array_equal(F.coeff[int(F.eq_ptr[4]):int(F.eq_ptr[6])],
                          e.coeff[int(e.eq_ptr[4]):int(e.eq_ptr[6])])
