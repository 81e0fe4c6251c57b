"""Seeded synthetic polynomial systems: the inputs both the CPU oracle and the
HIP path read.

This module only *builds* inputs (term tables, random coefficients, the
random gamma constant).  It performs none of the path tracker's arithmetic:
no evaluation, no start solutions, no linear algebra.

Representation of a square system f(x) = 0 in n unknowns (x_1..x_n):

* ``eq_ptr``  int32[n+1]      equation i owns terms eq_ptr[i]:eq_ptr[i+1]
* ``coeff``   complex128[T]   term coefficient
* ``exps``    uint8[T, n]     dense exponent vector of each term

Random numbers: every random complex constant is ``exp(2*pi*1j*u)`` with
``u`` drawn by ``numpy.random.default_rng(seed).random()``.  Draw order is
equation-major, terms in graded-lex order (total degree ascending, then
exponent vectors in descending lexicographic order, so x_1 > x_2 > ...),
and the homotopy constant gamma is drawn last.

Workloads follow the shapes of the paper's benchmark family (the cyclic
n-roots problems, Section 5), with random coefficients on the cyclic supports
standing in for the unit coefficients (which give positive-dimensional
solution sets for n = 8, 9, 12 by Backelin's Lemma, Section 1), plus random
dense systems.
"""
from __future__ import annotations

import dataclasses
import functools
import hashlib
import math

import numpy as np

MAX_N = 12


@dataclasses.dataclass
class PolySystem:
    n: int
    eq_ptr: np.ndarray  # int32[n+1]
    coeff: np.ndarray   # complex128[T]
    exps: np.ndarray    # uint8[T, n]
    name: str = ""

    @property
    def n_terms(self) -> int:
        return int(self.coeff.shape[0])

    def degrees(self) -> np.ndarray:
        """Total degree of each equation (largest term degree)."""
        out = np.zeros(self.n, dtype=np.int64)
        tdeg = self.exps.astype(np.int64).sum(axis=1)
        for i in range(self.n):
            a, b = int(self.eq_ptr[i]), int(self.eq_ptr[i + 1])
            out[i] = int(tdeg[a:b].max()) if b > a else 0
        return out

    def bezout(self) -> int:
        return int(np.prod(self.degrees()))

    def validate(self) -> None:
        assert self.eq_ptr.dtype == np.int32 and self.eq_ptr.shape == (self.n + 1,)
        assert self.coeff.dtype == np.complex128
        assert self.exps.dtype == np.uint8 and self.exps.shape == (self.n_terms, self.n)
        assert self.eq_ptr[0] == 0 and self.eq_ptr[-1] == self.n_terms
        assert np.all(np.diff(self.eq_ptr) >= 0)


def unit_circle(rng: np.random.Generator, size=None):
    """exp(2 pi i u), u ~ U[0,1): a random point on the unit circle."""
    u = rng.random(size)
    return np.exp(2j * np.pi * u)


def _assemble(n, eq_terms, name):
    """eq_terms: list over equations of lists of (coeff, exponent tuple)."""
    eq_ptr = [0]
    coeffs, exps = [], []
    for terms in eq_terms:
        for c, a in terms:
            coeffs.append(complex(c))
            exps.append(tuple(int(v) for v in a))
        eq_ptr.append(len(coeffs))
    s = PolySystem(
        n=n,
        eq_ptr=np.asarray(eq_ptr, dtype=np.int32),
        coeff=np.asarray(coeffs, dtype=np.complex128),
        exps=np.asarray(exps, dtype=np.uint8).reshape(len(coeffs), n),
        name=name,
    )
    s.validate()
    return s


def _compositions(n: int, deg: int):
    """Exponent vectors of n entries summing to deg, in descending
    lexicographic order."""
    if n == 1:
        return [(deg,)]
    out = []
    for a0 in range(deg, -1, -1):
        out.extend((a0,) + rest for rest in _compositions(n - 1, deg - a0))
    return out


@functools.lru_cache(maxsize=None)
def _graded_lex(n: int, d: int):
    out = []
    for deg in range(d + 1):
        out.extend(_compositions(n, deg))
    return tuple(out)


def graded_lex_monomials(n: int, d: int):
    """All exponent vectors of total degree <= d, degree ascending, then
    descending lexicographic order within a degree."""
    return list(_graded_lex(n, d))


def dense_system(n: int, degrees, rng: np.random.Generator, name="dense") -> PolySystem:
    """f_i = sum over all monomials x^a with |a| <= d_i of c_{i,a} x^a,
    c_{i,a} uniform on the unit circle."""
    eqs = []
    for i in range(n):
        mons = graded_lex_monomials(n, int(degrees[i]))
        cs = unit_circle(rng, len(mons))
        eqs.append(list(zip(cs, mons)))
    return _assemble(n, eqs, name)


def cyclic_system(n: int, rng: np.random.Generator, name=None) -> PolySystem:
    """Random coefficients on the supports of the cyclic n-roots problem.

    Equation k (k = 1..n-1) is sum_{i=1..n} c_{k,i} prod_{j=0..k-1} x_{(i-1+j mod n)+1};
    equation n is x_1 x_2 ... x_n - c.  Coefficients (and c) uniform on the
    unit circle; the leading monomial of equation n has coefficient exactly 1.
    The unit-coefficient instance of these supports is the cyclic n-roots
    system of the paper's Example 2.1 (n = 4) and Section 5.
    """
    eqs = []
    for k in range(1, n):
        terms = []
        cs = unit_circle(rng, n)
        for i in range(n):
            a = [0] * n
            for j in range(k):
                a[(i + j) % n] = 1
            terms.append((cs[i], tuple(a)))
        eqs.append(terms)
    c = unit_circle(rng)
    eqs.append([(1.0 + 0j, tuple([1] * n)), (-c, tuple([0] * n))])
    return _assemble(n, eqs, name or f"cyclic{n}")


def embedded_cyclic4(rng: np.random.Generator) -> PolySystem:
    """The embedded cyclic 4-roots system E_1(f(x), z_1) of Example 2.1:
    cyclic 4-roots (unit coefficients) with gamma_k z_1 added to equation k,
    plus the random hyperplane c_0 + c_1 x_1 + ... + c_4 x_4 + z_1 = 0.
    Unknowns are (x_1, x_2, x_3, x_4, z_1).  Draw order: gamma_1..gamma_4,
    then c_0..c_4."""
    n = 5
    g = unit_circle(rng, 4)
    c = unit_circle(rng, 5)
    z = (0, 0, 0, 0, 1)
    eqs = []
    for k in range(1, 4):
        terms = []
        for i in range(4):
            a = [0] * 5
            for j in range(k):
                a[(i + j) % 4] = 1
            terms.append((1.0, tuple(a)))
        terms.append((g[k - 1], z))
        eqs.append(terms)
    eqs.append([(1.0, (1, 1, 1, 1, 0)), (-1.0, (0, 0, 0, 0, 0)), (g[3], z)])
    eqs.append([(c[0], (0, 0, 0, 0, 0)), (c[1], (1, 0, 0, 0, 0)), (c[2], (0, 1, 0, 0, 0)),
                (c[3], (0, 0, 1, 0, 0)), (c[4], (0, 0, 0, 1, 0)), (1.0, z)])
    return _assemble(n, eqs, "embedded_cyclic4")


def univariate(d: int, rng: np.random.Generator) -> tuple[PolySystem, np.ndarray]:
    """One random polynomial sum_{k=0..d} c_k x^k.  Returns the system and the
    coefficient vector (highest degree first, numpy.roots order)."""
    cs = unit_circle(rng, d + 1)  # c_0..c_d
    s = _assemble(1, [[(cs[k], (k,)) for k in range(d + 1)]], f"univariate{d}")
    return s, cs[::-1].copy()


def decoupled(degrees, rng: np.random.Generator):
    """f_i = a_i x_i^{d_i} - b_i.  Returns the system and (a, b)."""
    n = len(degrees)
    a = unit_circle(rng, n)
    b = unit_circle(rng, n) * (0.5 + rng.random(n))
    eqs = []
    for i in range(n):
        e1 = [0] * n
        e1[i] = int(degrees[i])
        eqs.append([(a[i], tuple(e1)), (-b[i], tuple([0] * n))])
    return _assemble(n, eqs, "decoupled"), a, b


def _poly_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return out


def linear_products(n: int, degrees, rng: np.random.Generator):
    """f_i = prod_{k < d_i} (l_{ik} . x - beta_{ik}) with unit-circle l, beta,
    expanded into monomials (graded-lex order).  Returns the system and the
    factor data (L: list over i of complex[d_i, n], beta: list of complex[d_i])."""
    Ls, betas, eqs = [], [], []
    for i in range(n):
        d = int(degrees[i])
        L = unit_circle(rng, (d, n))
        beta = unit_circle(rng, d)
        poly = {tuple([0] * n): 1.0 + 0j}
        for k in range(d):
            lin = {tuple([0] * n): -beta[k]}
            for j in range(n):
                e = [0] * n
                e[j] = 1
                lin[tuple(e)] = L[k, j]
            poly = _poly_mul(poly, lin)
        order = graded_lex_monomials(n, d)
        eqs.append([(poly[a], a) for a in order if a in poly])
        Ls.append(L)
        betas.append(beta)
    return _assemble(n, eqs, "linear_products"), Ls, betas


def _expand(n, factors):
    """Product of polynomials given as dicts {exponent tuple: coefficient}."""
    poly = {tuple([0] * n): 1.0 + 0j}
    for q in factors:
        poly = _poly_mul(poly, q)
    return {a: c for a, c in poly.items() if c != 0}


def _lin(n, j, root):
    """x_j - root as a polynomial dict."""
    e = [0] * n
    e[j] = 1
    return {tuple(e): 1.0 + 0j, tuple([0] * n): -complex(root)}


def _var_pow(n, j, p):
    e = [0] * n
    e[j] = p
    return {tuple(e): 1.0 + 0j}


def membership_example() -> PolySystem:
    """The system of Example 4.1 (homotopy membership test), exact integer
    coefficients: (x1 - 1)(x1 - 2) = 0, (x1 - 1) x2^2 = 0: the line x1 = 1
    and the double point (2, 0)."""
    n = 2
    f1 = _expand(n, [_lin(n, 0, 1), _lin(n, 0, 2)])
    f2 = _expand(n, [_lin(n, 0, 1), _var_pow(n, 1, 2)])
    return _assemble(n, [sorted(((c, a) for a, c in f.items()), key=lambda t: (sum(t[1]), t[1]))
                         for f in (f1, f2)], "membership41")


def multistep_system() -> PolySystem:
    """The system of Example 3.1 (a 3-stage cascade), exact integer
    coefficients, expanded from its factored form:
    (x1-1)(x1-2)(x1-3)(x1-4), (x1-1)(x2-1)(x2-2)(x2-3),
    (x1-1)(x1-2)(x3-1)(x3-2), (x1-1)(x2-1)(x3-1)(x4-1)."""
    n = 4
    eqs = [
        _expand(n, [_lin(n, 0, 1), _lin(n, 0, 2), _lin(n, 0, 3), _lin(n, 0, 4)]),
        _expand(n, [_lin(n, 0, 1), _lin(n, 1, 1), _lin(n, 1, 2), _lin(n, 1, 3)]),
        _expand(n, [_lin(n, 0, 1), _lin(n, 0, 2), _lin(n, 2, 1), _lin(n, 2, 2)]),
        _expand(n, [_lin(n, 0, 1), _lin(n, 1, 1), _lin(n, 2, 1), _lin(n, 3, 1)]),
    ]
    return _assemble(n, [sorted(((c, a) for a, c in f.items()), key=lambda t: (sum(t[1]), t[1]))
                         for f in eqs], "multistep")


def embed(f: PolySystem, k: int, rng: np.random.Generator, name=None) -> PolySystem:
    """The embedding of Section 2.1 (Example 2.1 for k = 1): k slack
    variables z_1..z_k and k random hyperplanes.  Equation i of f becomes
    f_i + sum_j gamma_ij z_j; hyperplane j is c_j0 + sum_l c_jl x_l + z_j = 0.
    Unknowns (x_1..x_n, z_1..z_k).  Draw order: gamma_ij (i outer, j inner),
    then c_j0, c_j1, .., c_jn for j = 1..k, all uniform on the unit circle."""
    n = f.n
    m = n + k
    gam = unit_circle(rng, (n, k))
    cs = unit_circle(rng, (k, n + 1))
    eqs = []
    for i in range(n):
        terms = []
        for t in range(int(f.eq_ptr[i]), int(f.eq_ptr[i + 1])):
            terms.append((f.coeff[t], tuple(int(v) for v in f.exps[t]) + (0,) * k))
        for j in range(k):
            e = [0] * m
            e[n + j] = 1
            terms.append((gam[i, j], tuple(e)))
        eqs.append(terms)
    for j in range(k):
        terms = [(cs[j, 0], tuple([0] * m))]
        for l in range(n):
            e = [0] * m
            e[l] = 1
            terms.append((cs[j, l + 1], tuple(e)))
        e = [0] * m
        e[n + j] = 1
        terms.append((1.0, tuple(e)))
        eqs.append(terms)
    return _assemble(m, eqs, name or f"embedded_{f.name}_{k}")


# ---------------------------------------------------------------------------
# Named workloads (seeded)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    systems: list
    gammas: np.ndarray  # complex128[n_systems]

    @property
    def path_counts(self):
        return [s.bezout() for s in self.systems]

    @property
    def total_paths(self):
        return int(sum(self.path_counts))


def dense_small() -> Workload:
    """Dense random system, n = 5, five quadratics with all monomials of
    degree <= 2 (21 terms each); 32 total-degree paths.  Seed 1."""
    rng = np.random.default_rng(1)
    s = dense_system(5, [2] * 5, rng, name="dense5_d2")
    return Workload("dense5_d2", [s], np.asarray([unit_circle(rng)]))


def cyclic_workload(n: int, seed: int) -> Workload:
    rng = np.random.default_rng(seed)
    s = cyclic_system(n, rng)
    return Workload(f"cyclic{n}", [s], np.asarray([unit_circle(rng)]))


def cyclic8() -> Workload:
    """Random-coefficient cyclic-8 supports, 8! = 40320 paths.  Seed 2."""
    return cyclic_workload(8, 2)


def cyclic10() -> Workload:
    """Random-coefficient cyclic-10 supports, 10! = 3,628,800 paths.  Seed 5."""
    return cyclic_workload(10, 5)


def dense_batch(n_systems: int = 256, seed: int = 3) -> Workload:
    """n_systems dense random systems: n ~ U{3..10}, each equation degree
    ~ U{2,3} independently, one gamma per system.  Seed 3."""
    rng = np.random.default_rng(seed)
    systems, gammas = [], []
    for s in range(n_systems):
        n = int(rng.integers(3, 11))
        degs = rng.integers(2, 4, size=n)
        systems.append(dense_system(n, degs, rng, name=f"dense{s}_n{n}"))
        gammas.append(unit_circle(rng))
    return Workload("dense_batch", systems, np.asarray(gammas))


def embedded_cyclic4_workload() -> Workload:
    rng = np.random.default_rng(6)
    s = embedded_cyclic4(rng)
    return Workload("embedded_cyclic4", [s], np.asarray([unit_circle(rng)]))


def request_seed(base: int, request_id: int) -> int:
    h = hashlib.sha256(f"{base}:{request_id}".encode()).digest()
    return int.from_bytes(h[:8], "little")


def serving_request(request_id: int, base_seed: int = 4):
    """One solve request of the serving stream: with probability 1/2 a dense
    random system (n ~ U{4..12}, degrees ~ U{2,3}), otherwise a cyclic-support
    random system (n ~ U{5..9}).  Returns (system, gamma)."""
    rng = np.random.default_rng(request_seed(base_seed, request_id))
    if rng.random() < 0.5:
        n = int(rng.integers(4, 13))
        degs = rng.integers(2, 4, size=n)
        s = dense_system(n, degs, rng, name=f"req{request_id}_dense{n}")
    else:
        n = int(rng.integers(5, 10))
        s = cyclic_system(n, rng, name=f"req{request_id}_cyclic{n}")
    return s, complex(unit_circle(rng))


def poisson_arrivals(n_requests: int, rate: float, seed: int = 4) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream: exponential gaps at `rate`."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7919]))
    return np.cumsum(rng.exponential(1.0 / rate, size=n_requests))


def stride_sample(total: int, target: int) -> np.ndarray:
    """Deterministic stride sample of path ids 0..total-1 with about `target`
    entries (every k-th id)."""
    k = max(1, total // max(1, target))
    return np.arange(0, total, k, dtype=np.int64)


def n_terms_dense(n: int, d: int) -> int:
    return math.comb(n + d, d)
