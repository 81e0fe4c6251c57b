"""Pins of the oracle's homotopy membership test (Section 4.1) to closed
forms: the printed outcome of Example 4.1 (the double point (2, 0) is not on
the line x1 = 1) with the endpoint the moved hyperplane gives, a point of
the line found to be on it, and the three-dimensional set x1 = 1 of the
cascade example (Example 3.1, continued in Example 4.2) against its four
regular isolated solutions and points with x1 = 1."""
import numpy as np

import oracle
import workloads as W


def _ex41(seed=7):
    e = W.embed(W.membership_example(), 1, np.random.default_rng(seed))
    a, b = int(e.eq_ptr[2]), int(e.eq_ptr[3])
    c = {tuple(int(v) for v in e.exps[t]): complex(e.coeff[t]) for t in range(a, b)}
    c0, c1, c2 = c[(0, 0, 0)], c[(1, 0, 0)], c[(0, 1, 0)]
    witness = np.array([[1.0, -(c0 + c1) / c2, 0.0]])  # the line x1 = 1 at the hyperplane
    return e, (c0, c1, c2), witness


def test_moved_hyperplane_constant(oracle_lib):
    """Moving the hyperplane through (2, 0, 0) replaces c0 by c3 = -2 c1."""
    e, (c0, c1, c2), _ = _ex41()
    f = oracle.moved_hyperplanes(e, 1, [2, 0, 0])
    a, b = int(f.eq_ptr[2]), int(f.eq_ptr[3])
    const = [complex(f.coeff[t]) for t in range(a, b) if f.exps[t].sum() == 0]
    assert np.allclose(const, [-2 * c1], rtol=1e-15, atol=0)
    assert np.array_equal(f.coeff[:a], e.coeff[:a])  # the other equations are untouched


def test_example41_point_not_on_line(oracle_lib):
    """The printed outcome: the path from the generic point ends at another
    generic point of the line, (1, c1/c2, 0), not at (2, 0, 0)."""
    e, (c0, c1, c2), witness = _ex41()
    E, S, M = oracle.membership_test(e, 1, witness, [[2, 0, 0]])
    assert S[0, 0] == oracle.CONVERGED and not M[0]
    assert np.abs(E[0, 0] - np.array([1.0, c1 / c2, 0.0])).max() <= 1e-12


def test_example41_point_on_line(oracle_lib):
    e, _, witness = _ex41()
    y = np.array([1.0, 0.7 - 0.2j, 0.0])
    E, S, M = oracle.membership_test(e, 1, witness, [y])
    assert M[0] and np.abs(E[0, 0] - y).max() <= 1e-12


def _three_dim_set(seed=8):
    """Example 3.1's system embedded for its top dimension 3; the generic
    point of the three-dimensional set x1 = 1 (degree 1) where the three
    hyperplanes cut it (z = 0)."""
    e = W.embed(W.multistep_system(), 3, np.random.default_rng(seed))
    C = np.zeros((3, 5), complex)  # c_j0, c_j1 .. c_j4
    for j in range(3):
        i = 4 + j
        for t in range(int(e.eq_ptr[i]), int(e.eq_ptr[i + 1])):
            ex = e.exps[t]
            if ex.sum() == 0:
                C[j, 0] = e.coeff[t]
            elif ex[:4].sum() == 1:
                C[j, 1 + int(np.argmax(ex[:4]))] = e.coeff[t]
    rest = np.linalg.solve(C[:, 2:], -(C[:, 0] + C[:, 1]))
    return e, C, np.concatenate([[1.0], rest, [0, 0, 0]]).reshape(1, 7)


def test_three_dim_set_membership(oracle_lib):
    e, C, witness = _three_dim_set()
    isolated = [(3, 2, 2, 1), (3, 3, 2, 1), (4, 3, 2, 1), (4, 2, 2, 1)]  # printed in Example 3.1
    on_set = [(1, 2, 3, -1), (1, 0.5j, 2, 2 - 1j)]
    tests = np.array([list(p) + [0, 0, 0] for p in isolated + on_set], complex)
    E, S, M = oracle.membership_test(e, 3, witness, tests)
    assert (S == oracle.CONVERGED).all()
    assert M.tolist() == [False] * 4 + [True] * 2
    for k, y in enumerate(tests[:4]):
        # the moved hyperplanes cut x1 = 1 where c_j . (1, x2, x3, x4) = c_j . y
        rhs = C[:, 1:] @ y[:4] - C[:, 1]
        x = np.linalg.solve(C[:, 2:], rhs)
        assert np.abs(E[k, 0] - np.concatenate([[1.0], x, [0, 0, 0]])).max() <= 1e-10
