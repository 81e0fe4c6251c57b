"""CPU oracle for the batched homotopy path tracker -- TEST INFRASTRUCTURE.

Plain, slow, fp64 C implementation (``oracle.c``) of the tracker reading the
project follows, wrapped with ctypes.  Only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg import this package.  It shares no code with
the HIP library and never imports it; inputs come from ``workloads``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CONVERGED, DIVERGED, FAILED_MINSTEP, FAILED_MAXSTEPS, FAILED_NEWTON_T1 = range(5)


def build() -> str:
    """Compile oracle.c into liboracle.so (gcc, no FMA contraction)."""
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
           os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class RefSystem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("eq_ptr", ctypes.c_void_p), ("coeff", ctypes.c_void_p),
                ("exps", ctypes.c_void_p)]


class RefTolerances(ctypes.Structure):
    _fields_ = [("tol_residual", ctypes.c_double), ("tol_corr", ctypes.c_double),
                ("tol_final", ctypes.c_double), ("div_radius", ctypes.c_double),
                ("h_init", ctypes.c_double), ("h_min", ctypes.c_double),
                ("h_max", ctypes.c_double), ("max_steps", ctypes.c_int32),
                ("max_newton", ctypes.c_int32), ("max_newton_final", ctypes.c_int32)]


STATS_DTYPE = np.dtype([("steps", np.int32), ("rejections", np.int32),
                        ("newton_iters", np.int32), ("evals", np.int32),
                        ("solves", np.int32), ("pad", np.int32),
                        ("t_final", np.float64), ("residual", np.float64)])


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build()
            L = ctypes.CDLL(_SO)
            vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
            L.ref_default_tolerances.argtypes = [ctypes.POINTER(RefTolerances)]
            L.ref_eval_system.argtypes = [ctypes.POINTER(RefSystem), vp, vp, vp]
            L.ref_lu_solve.argtypes = [ctypes.c_int, vp, vp, vp]
            L.ref_lu_solve.restype = ctypes.c_int
            L.ref_start_point.argtypes = [ctypes.c_int, vp, i64, vp]
            L.ref_rk4_predict.argtypes = [ctypes.POINTER(RefSystem), ctypes.POINTER(RefSystem),
                                          vp, vp, ctypes.c_double, ctypes.c_double, vp]
            L.ref_rk4_predict.restype = ctypes.c_int
            L.ref_track_paths.argtypes = [ctypes.POINTER(RefSystem), ctypes.POINTER(RefSystem),
                                          vp, vp, vp, i64, ctypes.POINTER(RefTolerances),
                                          vp, vp, vp, i32]
            L.ref_track_paths.restype = ctypes.c_int
            L.ref_eval_system_dd.argtypes = [ctypes.POINTER(RefSystem), vp, vp, vp, vp]
            L.ref_residual_dd.argtypes = [ctypes.POINTER(RefSystem), vp]
            L.ref_residual_dd.restype = ctypes.c_double
            L.ref_residuals_dd.argtypes = [ctypes.POINTER(RefSystem), i64, vp, vp]
            L.ref_refine_dd.argtypes = [ctypes.POINTER(RefSystem), vp, ctypes.c_int, vp]
            L.ref_dd_ops.argtypes = [ctypes.c_double] * 4 + [vp, vp]
            L.ref_track_paths_dd.argtypes = [ctypes.POINTER(RefSystem), ctypes.POINTER(RefSystem),
                                             vp, vp, vp, i64, ctypes.POINTER(RefTolerances),
                                             vp, vp, vp, vp, i32]
            L.ref_track_paths_dd.restype = ctypes.c_int
            L.ref_find_duplicates.argtypes = [ctypes.c_int, i64, vp, vp, ctypes.c_double, vp, i64]
            L.ref_find_duplicates.restype = i64
            _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


class _Sys:
    """Keeps the numpy buffers of a RefSystem alive."""

    def __init__(self, s):
        self.eq_ptr = np.ascontiguousarray(s.eq_ptr, dtype=np.int32)
        self.coeff = np.ascontiguousarray(s.coeff, dtype=np.complex128)
        self.exps = np.ascontiguousarray(s.exps, dtype=np.uint8)
        self.st = RefSystem(int(s.n), int(self.coeff.shape[0]), _ptr(self.eq_ptr).value,
                            _ptr(self.coeff).value, _ptr(self.exps).value)


def default_tolerances(**over) -> RefTolerances:
    t = RefTolerances()
    lib().ref_default_tolerances(ctypes.byref(t))
    for k, v in over.items():
        setattr(t, k, v)
    return t


def eval_system(s, x):
    """(f(x), J_f(x)) for one point x (complex[n])."""
    S = _Sys(s)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    fx = np.zeros(s.n, np.complex128)
    jac = np.zeros((s.n, s.n), np.complex128)
    lib().ref_eval_system(ctypes.byref(S.st), _ptr(x), _ptr(fx), _ptr(jac))
    return fx, jac


def eval_system_dd(s, x_hi, x_lo=None):
    """f at x_hi + x_lo in double-double: returns (f_hi, f_lo) complex[n]."""
    S = _Sys(s)
    xh = np.ascontiguousarray(x_hi, dtype=np.complex128)
    xl = np.ascontiguousarray(x_lo, dtype=np.complex128) if x_lo is not None else None
    fh = np.zeros(s.n, np.complex128)
    fl = np.zeros(s.n, np.complex128)
    lib().ref_eval_system_dd(ctypes.byref(S.st), _ptr(xh), _ptr(xl), _ptr(fh), _ptr(fl))
    return fh, fl


def residual_dd(s, x):
    """The end game's residual ||f(x)||_inf (f in double-double) at x."""
    S = _Sys(s)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    return float(lib().ref_residual_dd(ctypes.byref(S.st), _ptr(x)))


def residuals_dd(s, X):
    """residual_dd at every row of X (complex [m, n])."""
    S = _Sys(s)
    X = np.ascontiguousarray(X, dtype=np.complex128).reshape(-1, s.n)
    out = np.zeros(X.shape[0])
    lib().ref_residuals_dd(ctypes.byref(S.st), int(X.shape[0]), _ptr(X), _ptr(out))
    return out


def refine_dd(s, x, iters=2):
    """The end game's double-double Newton refinement of x; nearest double."""
    S = _Sys(s)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.zeros_like(x)
    lib().ref_refine_dd(ctypes.byref(S.st), _ptr(x), int(iters), _ptr(out))
    return out


def dd_ops(a_hi, a_lo, b_hi, b_lo):
    """Double-double (sum, product) of a and b, each as (hi, lo)."""
    s = np.zeros(2)
    p = np.zeros(2)
    lib().ref_dd_ops(float(a_hi), float(a_lo), float(b_hi), float(b_lo), _ptr(s), _ptr(p))
    return (float(s[0]), float(s[1])), (float(p[0]), float(p[1]))


def lu_solve(A, b):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    y = np.zeros_like(b)
    rc = lib().ref_lu_solve(int(A.shape[0]), _ptr(A), _ptr(b), _ptr(y))
    if rc != 0:
        raise ZeroDivisionError("zero pivot")
    return y


def start_point(degrees, path_id):
    d = np.ascontiguousarray(degrees, dtype=np.int32)
    x = np.zeros(d.shape[0], np.complex128)
    lib().ref_start_point(int(d.shape[0]), _ptr(d), int(path_id), _ptr(x))
    return x


def rk4_predict(f, gamma, x, t, h):
    """One RK4 predictor step of the total-degree homotopy from (x, t)."""
    F = _Sys(f)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    gam = np.asarray([complex(gamma).real, complex(gamma).imag], np.float64)
    out = np.zeros_like(x)
    rc = lib().ref_rk4_predict(ctypes.byref(F.st), None, _ptr(gam), _ptr(x), float(t), float(h),
                               _ptr(out))
    if rc != 0:
        raise ArithmeticError("predictor failed")
    return out


def track_paths(f, gamma, path_ids=None, n_paths=None, start=None, g=None,
                tol: RefTolerances | None = None, n_threads: int = 1):
    """Tracks total-degree paths (or paths from given start points of g).
    Returns (endpoints complex[P, n], status int32[P], stats STATS_DTYPE[P])."""
    F = _Sys(f)
    G = _Sys(g) if g is not None else None
    if path_ids is not None:
        path_ids = np.ascontiguousarray(path_ids, dtype=np.int64)
        P = int(path_ids.shape[0])
    elif start is not None:
        start = np.ascontiguousarray(start, dtype=np.complex128)
        P = int(start.shape[0])
    else:
        P = int(n_paths if n_paths is not None else f.bezout())
    if start is not None:
        start = np.ascontiguousarray(start, dtype=np.complex128)
    gam = np.asarray([complex(gamma).real, complex(gamma).imag], np.float64)
    ends = np.zeros((P, f.n), np.complex128)
    status = np.full(P, -1, np.int32)
    stats = np.zeros(P, STATS_DTYPE)
    tol = tol or default_tolerances()
    rc = lib().ref_track_paths(ctypes.byref(F.st), ctypes.byref(G.st) if G else None,
                               _ptr(gam), _ptr(start), _ptr(path_ids), P, ctypes.byref(tol),
                               _ptr(ends), _ptr(status), _ptr(stats), int(n_threads))
    if rc != 0:
        raise ValueError(f"ref_track_paths failed ({rc})")
    return ends, status, stats


def dd_tolerances(**over) -> RefTolerances:
    """The double-double tracker's defaults: the double tracker's, with the
    final Newton at t = 1 run to 1e-26 relative."""
    t = default_tolerances(tol_final=1e-26)
    for k, v in over.items():
        setattr(t, k, v)
    return t


def track_paths_dd(f, gamma, path_ids=None, n_paths=None, start=None, g=None,
                   tol: RefTolerances | None = None, n_threads: int = 1):
    """The double-double tracker.  Returns (endpoints_hi, endpoints_lo
    complex [P, n], status int32 [P], stats)."""
    F = _Sys(f)
    G = _Sys(g) if g is not None else None
    if path_ids is not None:
        path_ids = np.ascontiguousarray(path_ids, dtype=np.int64)
        P = int(path_ids.shape[0])
    elif start is not None:
        start = np.ascontiguousarray(start, dtype=np.complex128)
        P = int(start.shape[0])
    else:
        P = int(n_paths if n_paths is not None else f.bezout())
    gam = np.asarray([complex(gamma).real, complex(gamma).imag], np.float64)
    hi = np.zeros((P, f.n), np.complex128)
    lo = np.zeros((P, f.n), np.complex128)
    status = np.full(P, -1, np.int32)
    stats = np.zeros(P, STATS_DTYPE)
    tol = tol or dd_tolerances()
    rc = lib().ref_track_paths_dd(ctypes.byref(F.st), ctypes.byref(G.st) if G else None,
                                  _ptr(gam), _ptr(start), _ptr(path_ids), P, ctypes.byref(tol),
                                  _ptr(hi), _ptr(lo), _ptr(status), _ptr(stats), int(n_threads))
    if rc != 0:
        raise ValueError(f"ref_track_paths_dd failed ({rc})")
    return hi, lo, status, stats


def find_duplicates(endpoints, status, rel=1e-6, max_pairs=1 << 16):
    e = np.ascontiguousarray(endpoints, dtype=np.complex128)
    s = np.ascontiguousarray(status, dtype=np.int32)
    pairs = np.zeros((max_pairs, 2), np.int64)
    cnt = lib().ref_find_duplicates(int(e.shape[1]), int(e.shape[0]), _ptr(e), _ptr(s),
                                    float(rel), _ptr(pairs), int(max_pairs))
    return pairs[: min(cnt, max_pairs)].copy()


def solve(f, gamma, n_threads=1, path_ids=None, tol=None, retrack=True):
    """Tracks every total-degree path (or the given ids), then the post-pass:
    converged endpoints that coincide within 1e-6 relative are path jumps;
    both paths of each pair are tracked once more with h_max = 0.01 and
    tol_corr = 1e-10.  Returns (endpoints, status, stats, remaining pairs)."""
    tol = tol or default_tolerances()
    ends, status, stats = track_paths(f, gamma, path_ids=path_ids,
                                      n_paths=None if path_ids is not None else f.bezout(),
                                      tol=tol, n_threads=n_threads)
    pairs = find_duplicates(ends, status)
    if retrack and len(pairs):
        idx = np.unique(pairs.ravel())
        ids = path_ids[idx] if path_ids is not None else idx.astype(np.int64)
        t2 = default_tolerances(**{f: getattr(tol, f) for f, _ in RefTolerances._fields_})
        t2.h_max = 0.01
        t2.tol_corr = 1e-10
        e2, s2, st2 = track_paths(f, gamma, path_ids=ids, tol=t2, n_threads=n_threads)
        ends[idx], status[idx], stats[idx] = e2, s2, st2
        pairs = find_duplicates(ends, status)
    return ends, status, stats, pairs


def moved_hyperplanes(e_sys, n_hyper, y):
    """The target system of a homotopy membership test (Section 4.1,
    Example 4.1): e_sys with the constant term of each of its last n_hyper
    equations (linear: the hyperplanes of the embedding) replaced so that the
    equation vanishes at the test point y, c3 = -(sum of the other terms at y).
    A hyperplane without a constant term gets one."""
    import dataclasses
    y = np.asarray(y, np.complex128)
    n = e_sys.n
    eq_ptr, coeff, exps = [0], [], []
    for i in range(n):
        a, b = int(e_sys.eq_ptr[i]), int(e_sys.eq_ptr[i + 1])
        cs = list(e_sys.coeff[a:b])
        ex = [np.asarray(e_sys.exps[t]) for t in range(a, b)]
        if i >= n - n_hyper:
            if any(int(e.sum()) > 1 for e in ex):
                raise ValueError("the moved equations must be linear")
            rest = sum(c * np.prod(y ** e) for c, e in zip(cs, ex) if e.sum() > 0)
            const = [k for k, e in enumerate(ex) if e.sum() == 0]
            if const:
                cs[const[0]] = -rest
            else:
                cs.append(-rest)
                ex.append(np.zeros(n, np.uint8))
        coeff += cs
        exps += ex
        eq_ptr.append(len(coeff))
    return dataclasses.replace(e_sys, eq_ptr=np.asarray(eq_ptr, np.int32),
                               coeff=np.asarray(coeff, np.complex128),
                               exps=np.asarray(exps, np.uint8).reshape(len(coeff), n),
                               name=f"{e_sys.name}_moved")


def membership_test(e_sys, n_hyper, witness, tests, tol: RefTolerances | None = None,
                    rel=1e-6, n_threads=1):
    """Homotopy membership test (Section 4.1, Example 4.1): for each test
    point y, the witness points of a solution set (solutions of the embedded
    system e_sys on it) are tracked along (1 - t) g + t f, g = e_sys, f = the
    same system with its hyperplanes moved through y (gamma = 1: only the
    hyperplane constants move, from c0 to c3).  y lies on the set when an
    endpoint coincides with it, ||x - y||_inf <= rel max(1, ||y||_inf).
    Returns (endpoints [T, m, n], status [T, m], member bool [T])."""
    witness = np.ascontiguousarray(witness, np.complex128).reshape(-1, e_sys.n)
    tests = np.asarray(tests, np.complex128).reshape(-1, e_sys.n)
    E, S, M = [], [], []
    for y in tests:
        f = moved_hyperplanes(e_sys, n_hyper, y)
        ends, st, _ = track_paths(f, 1.0, start=witness, g=e_sys, tol=tol, n_threads=n_threads)
        hit = (st == CONVERGED) & (np.abs(ends - y).max(axis=1) <= rel * max(1.0, np.abs(y).max()))
        E.append(ends)
        S.append(st)
        M.append(bool(hit.any()))
    return np.asarray(E), np.asarray(S), np.asarray(M)


def cascade_stage_system(e_cur, k, d):
    """The target system of the cascade stage that removes slack variable
    z_d (Section 3.1, Example 3.1): in the current system e_cur (unknowns x,
    then z_1..z_k; its last k equations the hyperplanes, in slack order), the
    terms in z_d leave the first n - k equations and equation n - k + d - 1
    becomes z_d = 0."""
    import dataclasses
    n = e_cur.n
    nx = n - k
    zi = nx + d - 1
    eq_ptr, coeff, exps = [0], [], []
    for i in range(n):
        a, b = int(e_cur.eq_ptr[i]), int(e_cur.eq_ptr[i + 1])
        if i == zi:
            ex = np.zeros(n, np.uint8)
            ex[zi] = 1
            coeff.append(1.0 + 0j)
            exps.append(ex)
        else:
            for t in range(a, b):
                if i < nx and e_cur.exps[t][zi] > 0:
                    continue
                coeff.append(complex(e_cur.coeff[t]))
                exps.append(np.asarray(e_cur.exps[t]))
        eq_ptr.append(len(coeff))
    return dataclasses.replace(e_cur, eq_ptr=np.asarray(eq_ptr, np.int32),
                               coeff=np.asarray(coeff, np.complex128),
                               exps=np.asarray(exps, np.uint8).reshape(len(coeff), n),
                               name=f"{e_cur.name}_z{d}")


def cascade(e, k, gammas, tol: RefTolerances | None = None, slack_tol=1e-6, n_threads=1):
    """Cascade of homotopies (Section 3.1, Example 3.1, Figure 3) on the
    embedded system e (top dimension k).  Stage 0 solves e (all total-degree
    paths, then the duplicate post-pass) with gammas[0]; its converged
    endpoints with z_k = 0 are candidate generic points of dimension k, those
    with z_k != 0 start the next stage.  Stage s (dimension d = k - s) tracks
    them with gammas[s] from the current system to the one without z_{d+1}
    (cascade_stage_system); converged endpoints with z_d = 0 (|z_d| <=
    slack_tol) are candidates of dimension d, the others start stage s + 1;
    at dimension 0 every converged endpoint is a candidate isolated solution.
    Returns a list of k + 1 stage records (dict: dim, paths, status
    histogram, candidates complex [c, n], nonzero count)."""
    out = []
    ends, st, _, _ = solve(e, gammas[0], n_threads=n_threads, tol=tol)
    cur = e
    nx = e.n - k
    for s in range(k + 1):
        d = k - s
        conv = st == CONVERGED
        if d > 0:
            zero = conv & (np.abs(ends[:, nx + d - 1]) <= slack_tol)
        else:
            zero = conv
        nz = conv & ~zero
        out.append({"dim": d, "paths": len(st), "status": np.bincount(st, minlength=5),
                    "candidates": ends[zero], "nonzero": int(nz.sum())})
        if d == 0:
            break
        nxt = cascade_stage_system(cur, k, d)
        ends, st, _ = track_paths(nxt, gammas[s + 1], start=ends[nz], g=cur, tol=tol,
                                  n_threads=n_threads)
        cur = nxt
    return out
