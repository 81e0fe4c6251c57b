"""Pins of the oracle's end game: the double-double arithmetic, the
double-double evaluation of f, the Newton refinement to the nearest double
of a root and the residual taken there, each against exact rational
arithmetic (fractions.Fraction) or arbitrary precision (mpmath), never
against the oracle itself."""
import math
from fractions import Fraction as Fr

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W


def _fr(x):
    return Fr(float(x))


def _rel(approx_hi, approx_lo, exact):
    got = _fr(approx_hi) + _fr(approx_lo)
    if exact == 0:
        return abs(float(got))
    return abs(float((got - exact) / exact))


def _rand_dd(rng):
    hi = rng.standard_normal() * 10.0 ** rng.integers(-3, 4)
    lo = hi * 2.0 ** -54 * rng.uniform(-1, 1)
    s = hi + lo  # normalise: hi is the nearest double of hi + lo
    return s, float(_fr(hi) + _fr(lo) - _fr(s))


def test_dd_sum_and_product_against_rationals(oracle_lib):
    rng = np.random.default_rng(101)
    for _ in range(2000):
        a_hi, a_lo = _rand_dd(rng)
        b_hi, b_lo = _rand_dd(rng)
        if rng.random() < 0.2:  # near cancellation in the sum
            b_hi, b_lo = -a_hi * (1 + 2.0 ** -40), -a_lo
        (s_hi, s_lo), (p_hi, p_lo) = oracle.dd_ops(a_hi, a_lo, b_hi, b_lo)
        A = _fr(a_hi) + _fr(a_lo)
        B = _fr(b_hi) + _fr(b_lo)
        # sum: accurate double-double addition, error <= 2^-104 |A + B|
        # (cancellation included) plus nothing else
        assert abs(_fr(s_hi) + _fr(s_lo) - (A + B)) <= Fr(1, 2 ** 104) * abs(A + B) + Fr(1, 2 ** 1070)
        # product: error <= 2^-102 |A B| (the dropped lo*lo term and the
        # roundings of the cross terms)
        assert abs(_fr(p_hi) + _fr(p_lo) - A * B) <= Fr(1, 2 ** 102) * abs(A * B)
        # normalised: |lo| <= ulp(hi) / 2
        for hi, lo in ((s_hi, s_lo), (p_hi, p_lo)):
            assert abs(lo) <= math.ulp(hi) / 2


def _exact_eval(s, x_hi, x_lo):
    """f at the exact complex rational point x_hi + x_lo, as pairs of Fractions."""
    xr = [(_fr(x_hi[j].real) + _fr(x_lo[j].real), _fr(x_hi[j].imag) + _fr(x_lo[j].imag))
          for j in range(s.n)]
    out, scale = [], []
    for i in range(s.n):
        re, im, mag = Fr(0), Fr(0), 0.0
        for t in range(int(s.eq_ptr[i]), int(s.eq_ptr[i + 1])):
            c = complex(s.coeff[t])
            vr, vi = _fr(c.real), _fr(c.imag)
            for j in range(s.n):
                for _ in range(int(s.exps[t, j])):
                    vr, vi = vr * xr[j][0] - vi * xr[j][1], vr * xr[j][1] + vi * xr[j][0]
            re += vr
            im += vi
            mag += abs(complex(float(vr), float(vi)))
        out.append((re, im))
        scale.append(mag)
    return out, scale


@pytest.mark.parametrize("make", [
    lambda rng: W.dense_system(3, [3, 2, 3], rng),
    lambda rng: W.cyclic_system(6, rng),
])
def test_eval_dd_against_rationals(oracle_lib, make):
    rng = np.random.default_rng(103)
    s = make(rng)
    for _ in range(4):
        x_hi = (rng.standard_normal(s.n) + 1j * rng.standard_normal(s.n)) * 1.7
        x_lo = x_hi * 2.0 ** -55 * (rng.uniform(-1, 1, s.n) + 1j * rng.uniform(-1, 1, s.n))
        x_hi = x_hi + x_lo  # keep the pair normalised
        x_lo = np.array([complex(float(_fr(a.real) + _fr(b.real) - _fr(c.real)),
                                 float(_fr(a.imag) + _fr(b.imag) - _fr(c.imag)))
                         for a, b, c in zip(x_hi - x_lo, x_lo, x_hi)])
        f_hi, f_lo = oracle.eval_system_dd(s, x_hi, x_lo)
        exact, scale = _exact_eval(s, x_hi, x_lo)
        for i in range(s.n):
            got_re = _fr(f_hi[i].real) + _fr(f_lo[i].real)
            got_im = _fr(f_hi[i].imag) + _fr(f_lo[i].imag)
            # error of a double-double evaluation: a small multiple of
            # 2^-104 times the sum of the term magnitudes
            bound = 64 * 2.0 ** -104 * scale[i]
            assert abs(float(got_re - exact[i][0])) <= bound
            assert abs(float(got_im - exact[i][1])) <= bound


def _univariate(coeffs):
    """p(x) = sum_k coeffs[k] x^k as a one-variable system."""
    d = len(coeffs) - 1
    return W.PolySystem(1, np.array([0, d + 1], np.int32),
                        np.array(coeffs[::-1], np.complex128),
                        np.array([[k] for k in range(d, -1, -1)], np.uint8))


def test_refine_gives_the_correctly_rounded_sqrt2(oracle_lib):
    s = _univariate([-2.0, 0.0, 1.0])  # x^2 - 2
    for x0 in (1.41421356, 1.4142135623731, math.sqrt(2) + 4 * math.ulp(math.sqrt(2))):
        out = oracle.refine_dd(s, np.array([x0 + 0j]), 3)
        assert out[0] == complex(math.sqrt(2), 0.0)  # IEEE sqrt rounds correctly
    # the residual there, exactly: |fl(sqrt 2)^2 - 2|
    r = math.sqrt(2)
    exact = abs(float(_fr(r) * _fr(r) - 2))
    assert oracle.residual_dd(s, np.array([r + 0j])) == exact


def test_refine_lands_on_a_representable_root_and_residual_is_zero(oracle_lib):
    # (x1 - 3/4)(x2 + 1/8 i) + x3 - 1/2, x2 - 2 x1 + 11/8 ... linear-times-linear,
    # root (3/4, -1/8 i + ..) chosen exactly representable
    rng = np.random.default_rng(7)
    root = np.array([0.75 - 0.5j, -0.125j + 1.0, 2.5 + 0.25j])
    n = 3
    # f_i = (l_i . (x - root)) * (1 + m_i . x): every root coordinate exact
    Ls = rng.integers(-3, 4, size=(n, n)) + 1j * rng.integers(-3, 4, size=(n, n))
    while abs(np.linalg.det(Ls)) < 1:
        Ls = rng.integers(-3, 4, size=(n, n)) + 1j * rng.integers(-3, 4, size=(n, n))
    eq_terms = []
    for i in range(n):
        lin = {(0,) * n: -complex(np.dot(Ls[i], root))}
        for j in range(n):
            e = [0] * n
            e[j] = 1
            lin[tuple(e)] = complex(Ls[i][j])
        m = {(0,) * n: 1.0}
        e = [0] * n
        e[(i + 1) % n] = 1
        m[tuple(e)] = 0.5j
        prod = {}
        for a, ca in lin.items():
            for b, cb in m.items():
                k = tuple(x + y for x, y in zip(a, b))
                prod[k] = prod.get(k, 0) + ca * cb
        eq_terms.append(prod)
    eq_ptr, coeff, exps = [0], [], []
    for prod in eq_terms:
        for k, c in prod.items():
            coeff.append(c)
            exps.append(k)
        eq_ptr.append(len(coeff))
    s = W.PolySystem(n, np.array(eq_ptr, np.int32), np.array(coeff, np.complex128),
                     np.array(exps, np.uint8))
    x0 = root * (1 + 1e-9) + 3e-10j
    out = oracle.refine_dd(s, x0, 2)
    assert np.array_equal(out, root)
    assert oracle.residual_dd(s, root) == 0.0


def test_refine_matches_mpmath_root_of_a_dense_system(oracle_lib):
    """Tracks a dense system's paths, then checks that every endpoint is the
    nearest complex double of the root mpmath finds at 50 digits from it."""
    rng = np.random.default_rng(109)
    s = W.dense_system(3, [2, 3, 2], rng)
    gamma = complex(W.unit_circle(rng))
    ends, st, _ = oracle.track_paths(s, gamma, n_paths=s.bezout())
    assert (st == 0).all()
    mpmath.mp.dps = 50
    xs = mpmath.matrix(3, 1)

    def F(*x):
        out = []
        for i in range(s.n):
            v = mpmath.mpc(0)
            for t in range(int(s.eq_ptr[i]), int(s.eq_ptr[i + 1])):
                c = complex(s.coeff[t])
                m = mpmath.mpc(c.real, c.imag)
                for j in range(s.n):
                    m *= x[j] ** int(s.exps[t, j])
                v += m
            out.append(v)
        return out

    for e in ends:
        r = mpmath.findroot(F, [mpmath.mpc(z.real, z.imag) for z in e])
        nearest = np.array([complex(float(r[j].real), float(r[j].imag)) for j in range(s.n)])
        assert np.array_equal(e, nearest)
    del xs


def test_residual_dd_against_rationals(oracle_lib):
    rng = np.random.default_rng(113)
    s = W.dense_system(4, [2, 3, 2, 2], rng)
    for _ in range(5):
        x = (rng.standard_normal(4) + 1j * rng.standard_normal(4)) * 2.0
        exact, _ = _exact_eval(s, x, np.zeros(4, np.complex128))
        mods = [abs(complex(float(re), float(im))) for re, im in exact]
        assert oracle.residual_dd(s, x) == pytest.approx(max(mods), rel=1e-15)
