"""Batched FP64 homotopy path tracking on AMD Instinct MI355X (gfx950).

Python binding of libhomotopy (include/homotopy.h): argument marshalling
only.  Host entry points take and return numpy arrays; device entry points
take torch tensors on the GPU (torch supplies device memory and streams).
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref

import numpy as np

from . import _lib
from ._lib import (CONVERGED, DIVERGED, FAILED_MAXSTEPS, FAILED_MINSTEP, FAILED_NEWTON_T1,
                   HP_BATCHED, HP_MAX_N, HP_PLAIN, STATS_DTYPE, HomotopyError, HpC64,
                   HpCascadeStage, HpSystem, HpTiming, HpTolerances, check, load)

__all__ = [
    "Context", "Plan", "Server", "default_tolerances", "path_count", "batch_layout",
    "find_duplicates", "spec_compile", "CONVERGED", "DIVERGED", "FAILED_MINSTEP", "FAILED_MAXSTEPS",
    "FAILED_NEWTON_T1", "HP_PLAIN", "HP_BATCHED", "STATS_DTYPE", "HomotopyError",
]

_MODES = {"plain": HP_PLAIN, "batched": HP_BATCHED, HP_PLAIN: HP_PLAIN, HP_BATCHED: HP_BATCHED}


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


class _SysView:
    """HpSystem over numpy buffers kept alive by this object."""

    def __init__(self, s):
        self.eq_ptr = np.ascontiguousarray(s.eq_ptr, dtype=np.int32)
        self.coeff = np.ascontiguousarray(s.coeff, dtype=np.complex128)
        self.exps = np.ascontiguousarray(s.exps, dtype=np.uint8)
        self.n = int(s.n)
        self.c = HpSystem(self.n, int(self.coeff.shape[0]), self.eq_ptr.ctypes.data,
                          self.coeff.ctypes.data, self.exps.ctypes.data)


def _stream(stream):
    """HIP stream handle of a torch stream (or an int), None for the default."""
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _c64(z):
    z = complex(z)
    return HpC64(z.real, z.imag)


def default_tolerances(**over) -> HpTolerances:
    t = HpTolerances()
    load().hp_default_tolerances(ctypes.byref(t))
    for k, v in over.items():
        setattr(t, k, v)
    return t


def default_tolerances_dd(**over) -> HpTolerances:
    """The double-double tracker's defaults (final Newton to 1e-26)."""
    t = HpTolerances()
    load().hp_default_tolerances_dd(ctypes.byref(t))
    for k, v in over.items():
        setattr(t, k, v)
    return t


def path_count(system) -> int:
    return int(load().hp_path_count(ctypes.byref(_SysView(system).c)))


def spec_compile(system, form=None) -> int:
    """Writes and compiles (hiprtc, gfx950) the kernel specialised to the
    system's support without a device; returns the code object's size.
    form None: the plans' and the server's forms; 0, 1, 2: the plans', the
    server's or the coefficient-parameter form alone."""
    out = ctypes.c_int64(0)
    if form is None:
        check(load().hp_spec_compile(ctypes.byref(_SysView(system).c), ctypes.byref(out)))
    else:
        check(load().hp_spec_compile_form(ctypes.byref(_SysView(system).c), int(form),
                                          ctypes.byref(out)))
    return int(out.value)


def batch_layout(systems):
    views = [_SysView(s) for s in systems]
    arr = (HpSystem * len(views))(*[v.c for v in views])
    po = np.zeros(len(views) + 1, np.int64)
    xo = np.zeros(len(views) + 1, np.int64)
    check(load().hp_batch_layout(arr, len(views), _ptr(po), _ptr(xo)))
    return po, xo


def find_duplicates(endpoints, status, rel=1e-6, max_pairs=1 << 16):
    e = np.ascontiguousarray(endpoints, dtype=np.complex128)
    s = np.ascontiguousarray(status, dtype=np.int32)
    pairs = np.zeros((max_pairs, 2), np.int64)
    cnt = load().hp_find_duplicates(int(e.shape[1]), int(e.shape[0]), _ptr(e), _ptr(s),
                                    float(rel), _ptr(pairs), int(max_pairs))
    if cnt < 0:
        check(-1)
    return pairs[: min(cnt, max_pairs)].copy()


# Live handles, closed at interpreter exit while the HIP runtime is still up
# (objects finalised later, during interpreter teardown, skip the C call).
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_LIVE):
        if not isinstance(obj, Context):
            obj.close()
    for obj in list(_LIVE):
        obj.close()


def _finalize(obj, _finalizing=sys.is_finalizing):
    """__del__ body: close unless the interpreter is shutting down (then the
    atexit hook above has closed every handle already)."""
    try:
        if not _finalizing():
            obj.close()
    except Exception:
        pass


class Context:
    """A libhomotopy context on one HIP device (its own stream)."""

    def __init__(self, device: int = 0):
        self._L = load()
        self.handle = None
        h = ctypes.c_void_p()
        check(self._L.hp_context_create(int(device), ctypes.byref(h)))
        self.handle = h
        self._children = weakref.WeakSet()  # plans and servers built on this context
        _LIVE.add(self)

    def close(self):
        """Destroys the plans and servers made from this context, then the
        context.  (The C library releases a context only after its children
        are gone, so any order of closing is safe.)"""
        if self.handle:
            for c in list(self._children):
                c.close()
            self._L.hp_context_destroy(self.handle)
            self.handle = None

    def __del__(self, _fin=_finalize):  # bound now: module globals are gone at teardown
        _fin(self)

    def last_timing(self) -> dict:
        t = HpTiming()
        check(self._L.hp_last_timing(self.handle, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in HpTiming._fields_}

    def track_paths(self, system, gamma, n_paths=None, tol=None, mode="batched", stats=True,
                    start=None, g=None):
        """Tracks paths of gamma(1-t) g + t f (host arrays in and out).
        start=None: total-degree paths 0..n_paths-1; otherwise one path per
        row of start (complex [P, n]), from the start system g (None: total
        degree).  Returns (endpoints complex[P, n], status int32[P], stats)."""
        v = _SysView(system)
        gv = _SysView(g) if g is not None else None
        if start is not None:
            start = np.ascontiguousarray(start, dtype=np.complex128).reshape(-1, v.n)
            P = int(start.shape[0])
        else:
            P = path_count(system) if n_paths is None else int(n_paths)
        ends = np.zeros((P, v.n), np.complex128)
        st = np.full(P, -1, np.int32)
        sts = np.zeros(P, STATS_DTYPE) if stats else None
        tol = tol or default_tolerances()
        check(self._L.hp_track_paths(self.handle, ctypes.byref(v.c),
                                     ctypes.byref(gv.c) if gv is not None else None,
                                     _ptr(start), P, _c64(gamma), ctypes.byref(tol), _ptr(ends),
                                     _ptr(st), _ptr(sts), _MODES[mode]))
        return ends, st, sts

    def track_paths_dd(self, system, gamma, n_paths=None, tol=None, stats=True, start=None):
        """The double-double tracker (hp_track_paths_dd).  Returns
        (endpoints_hi, endpoints_lo complex [P, n], status, stats)."""
        v = _SysView(system)
        if start is not None:
            start = np.ascontiguousarray(start, dtype=np.complex128).reshape(-1, v.n)
            P = int(start.shape[0])
        else:
            P = path_count(system) if n_paths is None else int(n_paths)
        hi = np.zeros((P, v.n), np.complex128)
        lo = np.zeros((P, v.n), np.complex128)
        st = np.full(P, -1, np.int32)
        sts = np.zeros(P, STATS_DTYPE) if stats else None
        tol = tol or default_tolerances_dd()
        check(self._L.hp_track_paths_dd(self.handle, ctypes.byref(v.c), _ptr(start), P, _c64(gamma),
                                        ctypes.byref(tol), _ptr(hi), _ptr(lo), _ptr(st), _ptr(sts)))
        return hi, lo, st, sts

    def track_batch(self, systems, gammas, tol=None, stats=True):
        """Many systems in one persistent launch.  Returns per-system lists of
        (endpoints, status, stats)."""
        views = [_SysView(s) for s in systems]
        arr = (HpSystem * len(views))(*[x.c for x in views])
        po, xo = batch_layout(systems)
        ends = np.zeros(int(xo[-1]), np.complex128)
        st = np.full(int(po[-1]), -1, np.int32)
        sts = np.zeros(int(po[-1]), STATS_DTYPE) if stats else None
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.complex128))
        tol = tol or default_tolerances()
        check(self._L.hp_track_batch(self.handle, arr, len(views), _ptr(g), ctypes.byref(tol),
                                     _ptr(ends), _ptr(st), _ptr(sts)))
        out = []
        for i, x in enumerate(views):
            p0, p1 = int(po[i]), int(po[i + 1])
            e = ends[int(xo[i]):int(xo[i + 1])].reshape(p1 - p0, x.n)
            out.append((e, st[p0:p1], sts[p0:p1] if stats else None))
        return out

    def tune_batch(self, systems, gammas, tol=None) -> dict:
        """Autotunes the launch of batches shaped like this one (hp_tune_batch);
        later track_batch calls on such batches use the choice."""
        views = [_SysView(s) for s in systems]
        arr = (HpSystem * len(views))(*[x.c for x in views])
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.complex128))
        tol = tol or default_tolerances()
        c = _lib.HpTuneChoice()
        check(self._L.hp_tune_batch(self.handle, arr, len(views), _ptr(g), ctypes.byref(tol),
                                    ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in c._fields_}

    def solve(self, system, gamma, tol=None):
        """All paths (batched), then the duplicate-endpoint re-track pass.
        Returns (endpoints, status, stats, remaining duplicate pairs)."""
        v = _SysView(system)
        P = path_count(system)
        ends = np.zeros((P, v.n), np.complex128)
        st = np.full(P, -1, np.int32)
        sts = np.zeros(P, STATS_DTYPE)
        rem = ctypes.c_int64(0)
        tol = tol or default_tolerances()
        check(self._L.hp_solve(self.handle, ctypes.byref(v.c), _c64(gamma), ctypes.byref(tol),
                               _ptr(ends), _ptr(st), _ptr(sts), ctypes.byref(rem)))
        return ends, st, sts, int(rem.value)

    def membership_test(self, e_sys, n_hyper, witness, tests, tol=None, rel=1e-6):
        """Homotopy membership test (hp_membership_test): the witness points
        of e_sys tracked as its last n_hyper hyperplanes move through each test
        point.  Returns (endpoints [T, m, n], status [T, m], member bool [T])."""
        v = _SysView(e_sys)
        w = np.ascontiguousarray(witness, np.complex128).reshape(-1, v.n)
        y = np.ascontiguousarray(tests, np.complex128).reshape(-1, v.n)
        T, m = y.shape[0], w.shape[0]
        ends = np.zeros((T, m, v.n), np.complex128)
        st = np.full((T, m), -1, np.int32)
        mem = np.zeros(T, np.int32)
        tol = tol or default_tolerances()
        check(self._L.hp_membership_test(self.handle, ctypes.byref(v.c), int(n_hyper), _ptr(w), m,
                                         _ptr(y), T, ctypes.byref(tol), float(rel), _ptr(ends),
                                         _ptr(st), _ptr(mem)))
        return ends, st, mem.astype(bool)

    def cascade(self, e_sys, k, gammas, tol=None, slack_tol=1e-6, cap=1 << 16):
        """Cascade of homotopies (hp_cascade) on an embedded system of top
        dimension k.  Returns (stages: list of dicts, candidates complex
        [c, n], their dimensions int [c])."""
        v = _SysView(e_sys)
        g = np.ascontiguousarray(np.asarray(gammas, np.complex128).reshape(-1))
        if g.shape[0] != k + 1:
            raise ValueError("need k + 1 gammas")
        stages = (HpCascadeStage * (k + 1))()
        wit = np.zeros((cap, v.n), np.complex128)
        dims = np.zeros(cap, np.int32)
        total = ctypes.c_int64(0)
        tol = tol or default_tolerances()
        check(self._L.hp_cascade(self.handle, ctypes.byref(v.c), int(k), _ptr(g), ctypes.byref(tol),
                                 float(slack_tol), stages, _ptr(wit), _ptr(dims), cap,
                                 ctypes.byref(total)))
        c = min(cap, int(total.value))
        recs = [{f: getattr(s, f) for f, _ in HpCascadeStage._fields_ if f != "pad"} for s in stages]
        return recs, wit[:c], dims[:c]

    def plan(self, system, gamma, tol=None, tune=False, g=None, start=None):
        return Plan(self, system, gamma, tol, tune, g=g, start=start)

    def find_duplicates_device(self, endpoints, status, rel=1e-6, max_pairs=1 << 16, stream=None):
        """Duplicate scan of device tensors (endpoints float64 [P, n, 2] or
        complex128 [P, n], status int32 [P]).  Returns (pairs int64 device
        tensor [min(found, max_pairs), 2], number found)."""
        import torch
        P, n = int(status.shape[0]), int(endpoints.shape[1])
        pairs = torch.zeros((max(1, max_pairs), 2), dtype=torch.int64, device=status.device)
        found = ctypes.c_int64(0)
        check(self._L.hp_find_duplicates_device(self.handle, n, P, _ptr(endpoints), _ptr(status),
                                                float(rel), _ptr(pairs), int(max_pairs),
                                                ctypes.byref(found), _stream(stream)))
        return pairs[: min(found.value, max_pairs)], int(found.value)

    def find_duplicates_device_static(self, endpoints, status, pairs, rel=1e-6, stream=None):
        """The same scan in the library's fixed per-GPU workspace (no device
        allocation; hp_find_duplicates_device_static) into the caller's int64
        device tensor pairs [max_pairs, 2]; returns the number found."""
        P, n = int(status.shape[0]), int(endpoints.shape[1])
        found = ctypes.c_int64(0)
        check(self._L.hp_find_duplicates_device_static(self.handle, n, P, _ptr(endpoints),
                                                       _ptr(status), float(rel), _ptr(pairs),
                                                       int(pairs.shape[0]), ctypes.byref(found),
                                                       _stream(stream)))
        return int(found.value)


class Plan:
    """A system resident on the device; tracks paths into torch tensors."""

    def __init__(self, ctx: Context, system, gamma, tol=None, tune=False, g=None, start=None):
        """start (complex [P, n]): a general plan (hp_plan_create_general) whose
        path k starts at start[k], from the start system g (None: total degree)."""
        self.ctx = ctx
        self._L = ctx._L
        self._view = _SysView(system)
        self.n = self._view.n
        self.tol = tol or default_tolerances()
        h = ctypes.c_void_p()
        self.handle = None
        if start is None:
            if g is not None:
                raise ValueError("a plan with a start system g needs its start points")
            self.paths = path_count(system)
            check(self._L.hp_plan_create(ctx.handle, ctypes.byref(self._view.c), _c64(gamma),
                                         ctypes.byref(self.tol), int(bool(tune)), ctypes.byref(h)))
        else:
            st = np.ascontiguousarray(np.asarray(start, dtype=np.complex128).reshape(-1, self.n))
            self.paths = len(st)
            self._gview = _SysView(g) if g is not None else None
            check(self._L.hp_plan_create_general(
                ctx.handle, ctypes.byref(self._view.c),
                ctypes.byref(self._gview.c) if self._gview is not None else None, _ptr(st), len(st),
                _c64(gamma), ctypes.byref(self.tol), int(bool(tune)), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)
        _LIVE.add(self)

    def close(self):
        if self.handle:
            self._L.hp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self, _fin=_finalize):  # bound now: module globals are gone at teardown
        _fin(self)

    def set_variant(self, variant: int):
        """Kernel variant code (see hp_plan_set_variant in homotopy.h)."""
        check(self._L.hp_plan_set_variant(self.handle, int(variant)))

    def set_launch(self, paths_per_wave: int = 0, waves_per_simd: int = 0):
        """Launch shape of the plan's variant (hp_plan_set_launch)."""
        check(self._L.hp_plan_set_launch(self.handle, int(paths_per_wave), int(waves_per_simd)))

    def tuning(self) -> dict:
        """The autotuner's record (hp_plan_tuning; zeros when not tuned)."""
        c = _lib.HpTuneChoice()
        check(self._L.hp_plan_tuning(self.handle, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in c._fields_}

    def outputs(self, n_paths, stats=True, device="cuda"):
        """Device tensors (endpoints as float64 [P, n, 2], status, stats bytes)."""
        import torch
        e = torch.empty((n_paths, self.n, 2), dtype=torch.float64, device=device)
        s = torch.empty((n_paths,), dtype=torch.int32, device=device)
        st = torch.empty((n_paths, STATS_DTYPE.itemsize), dtype=torch.uint8, device=device) \
            if stats else None
        return e, s, st

    def track_device(self, endpoints, status, stats=None, ids=None, n_paths=None,
                     mode="batched", stream=None):
        """Tracks into device tensors.  ids: optional int64 device tensor."""
        P = int(n_paths if n_paths is not None else status.shape[0])
        check(self._L.hp_plan_track_device(self.handle, _ptr(ids), P, _ptr(endpoints),
                                           _ptr(status), _ptr(stats), _MODES[mode],
                                           _stream(stream)))

    def solve_device(self, endpoints, status, stats=None, stream=None):
        """Every path, then the duplicate post-pass, into device tensors
        (hp_plan_solve_device).  Returns (pairs found, pairs left)."""
        found, left = ctypes.c_int64(0), ctypes.c_int64(0)
        check(self._L.hp_plan_solve_device(self.handle, _ptr(endpoints), _ptr(status), _ptr(stats),
                                           ctypes.byref(found), ctypes.byref(left),
                                           _stream(stream)))
        return int(found.value), int(left.value)

    @staticmethod
    def stats_to_numpy(stats_tensor):
        return stats_tensor.cpu().numpy().view(STATS_DTYPE).reshape(-1)

    @staticmethod
    def endpoints_to_numpy(e):
        a = e.cpu().numpy()
        return a[..., 0] + 1j * a[..., 1]


class Server:
    """Request loop with continuous batching (hp_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int):
        self.ctx = ctx
        self._L = ctx._L
        self.handle = None
        h = ctypes.c_void_p()
        check(self._L.hp_server_create(ctx.handle, int(hbm_budget_bytes), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)
        _LIVE.add(self)
        self._keep = {}

    def submit(self, system, gamma, tol=None) -> int:
        v = _SysView(system)
        tol = tol or default_tolerances()
        rid = ctypes.c_int64(-1)
        check(self._L.hp_server_submit(self.handle, ctypes.byref(v.c), _c64(gamma),
                                       ctypes.byref(tol), ctypes.byref(rid)))
        self._keep[int(rid.value)] = (v.n, path_count(system))
        return int(rid.value)

    def poll(self, rid) -> bool:
        d = ctypes.c_int32(0)
        check(self._L.hp_server_poll(self.handle, int(rid), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, rid, stats=False):
        n, P = self._keep.pop(int(rid))
        ends = np.zeros((P, n), np.complex128)
        st = np.full(P, -1, np.int32)
        sts = np.zeros(P, STATS_DTYPE) if stats else None
        lat = ctypes.c_double(0.0)
        check(self._L.hp_server_wait(self.handle, int(rid), _ptr(ends), _ptr(st), _ptr(sts),
                                     ctypes.byref(lat)))
        return ends, st, sts, float(lat.value)

    def peak_bytes(self) -> int:
        v = ctypes.c_size_t(0)
        check(self._L.hp_server_peak_bytes(self.handle, ctypes.byref(v)))
        return int(v.value)

    def set_slice(self, slice_ms: float, fixed_steps: int = 0) -> None:
        """Epoch kernel-time target (ms) of the sliced kernel families, or a
        fixed step budget per wavefront and epoch; 0, 0 runs queues to the end."""
        check(self._L.hp_server_set_slice(self.handle, float(slice_ms), int(fixed_steps)))

    def info(self) -> dict:
        v = _lib.HpServerInfo()
        check(self._L.hp_server_info_get(self.handle, ctypes.byref(v)))
        return {k: getattr(v, k) for k, _ in v._fields_ if k != "pad"}

    def close(self):
        if self.handle:
            self._L.hp_server_destroy(self.handle)
            self.handle = None

    def __del__(self, _fin=_finalize):  # bound now: module globals are gone at teardown
        _fin(self)
