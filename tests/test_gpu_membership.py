"""The homotopy membership test on the GPU (hp_membership_test, Section 4.1)
against the oracle and the closed forms of Example 4.1 and of the
three-dimensional set of Example 3.1's system (Example 4.2)."""
import os
import sys

import numpy as np
import pytest

import oracle
from parity import assert_parity
from test_oracle_membership import _ex41, _three_dim_set

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_03807_amd as hp
    c = hp.Context(0)
    yield c
    c.close()


def test_example41_on_gpu(ctx):
    e, (c0, c1, c2), witness = _ex41()
    tests = np.array([[2, 0, 0], [1.0, 0.7 - 0.2j, 0.0]], complex)
    E, S, M = ctx.membership_test(e, 1, witness, tests)
    log(f"  member {M.tolist()}, endpoints {E[:, 0]}")
    assert M.tolist() == [False, True]
    assert np.abs(E[0, 0] - np.array([1.0, c1 / c2, 0.0])).max() <= 1e-12
    Eo, So, Mo = oracle.membership_test(e, 1, witness, tests)
    assert Mo.tolist() == M.tolist()
    assert_parity(E.reshape(-1, 3), S.ravel(), Eo.reshape(-1, 3), So.ravel(), "example 4.1", e)


def test_three_dim_set_on_gpu(ctx):
    e, C, witness = _three_dim_set()
    isolated = [(3, 2, 2, 1), (3, 3, 2, 1), (4, 3, 2, 1), (4, 2, 2, 1)]
    on_set = [(1, 2, 3, -1), (1, 0.5j, 2, 2 - 1j)]
    tests = np.array([list(p) + [0, 0, 0] for p in isolated + on_set], complex)
    E, S, M = ctx.membership_test(e, 3, witness, tests)
    assert M.tolist() == [False] * 4 + [True] * 2
    Eo, So, Mo = oracle.membership_test(e, 3, witness, tests, n_threads=NTHREADS)
    assert Mo.tolist() == M.tolist()
    assert_parity(E.reshape(-1, 7), S.ravel(), Eo.reshape(-1, 7), So.ravel(), "example 4.2 (3D set)",
                  e)


def test_membership_rejects_nonlinear_hyperplane(ctx):
    import paper_1804_03807_amd as hp
    e, _, witness = _ex41()
    with pytest.raises(hp.HomotopyError):
        ctx.membership_test(e, 2, witness, [[2, 0, 0]])  # the second equation is not linear
