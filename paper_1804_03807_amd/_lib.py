"""ctypes declarations of the libhomotopy C ABI (include/homotopy.h).

Argument marshalling only: every step of the path tracker runs in the HIP
library.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libhomotopy.so")

HP_OK, HP_E_INVALID_ARG, HP_E_UNSUPPORTED_N, HP_E_OOM, HP_E_DEVICE, HP_E_BUDGET = 0, -1, -2, -3, -4, -5
HP_PLAIN, HP_BATCHED = 0, 1
HP_MAX_N = 12

CONVERGED, DIVERGED, FAILED_MINSTEP, FAILED_MAXSTEPS, FAILED_NEWTON_T1 = range(5)

EXPORTED = [
    "hp_context_create", "hp_context_destroy", "hp_last_error", "hp_default_tolerances",
    "hp_last_timing", "hp_path_count", "hp_track_paths", "hp_plan_create", "hp_plan_destroy",
    "hp_plan_set_variant", "hp_plan_track_device", "hp_batch_layout", "hp_track_batch",
    "hp_find_duplicates", "hp_solve", "hp_server_create", "hp_server_submit", "hp_server_poll",
    "hp_server_wait", "hp_server_peak_bytes", "hp_server_destroy", "hp_spec_compile",
    "hp_find_duplicates_device", "hp_plan_solve_device", "hp_find_duplicates_device_static",
    "hp_membership_test", "hp_cascade", "hp_track_paths_dd", "hp_default_tolerances_dd",
    "hp_server_set_slice", "hp_server_info_get", "hp_plan_set_launch", "hp_plan_tuning",
    "hp_tune_batch", "hp_plan_create_general", "hp_spec_compile_form",
]


class HpC64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class HpSystem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_terms", ctypes.c_int32), ("eq_ptr", ctypes.c_void_p),
                ("coeff", ctypes.c_void_p), ("exps", ctypes.c_void_p)]


class HpTolerances(ctypes.Structure):
    _fields_ = [("tol_residual", ctypes.c_double), ("tol_corr", ctypes.c_double),
                ("tol_final", ctypes.c_double), ("div_radius", ctypes.c_double),
                ("h_init", ctypes.c_double), ("h_min", ctypes.c_double),
                ("h_max", ctypes.c_double), ("max_steps", ctypes.c_int32),
                ("max_newton", ctypes.c_int32), ("max_newton_final", ctypes.c_int32)]


class HpServerInfo(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int64), ("carried", ctypes.c_int64),
                ("epoch_ms_max", ctypes.c_double), ("epoch_ms_mean", ctypes.c_double),
                ("slice_ms", ctypes.c_double), ("fixed_steps", ctypes.c_int32),
                ("budget_min", ctypes.c_int32), ("budget_max", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("peak_bytes", ctypes.c_uint64)]


class HpCascadeStage(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad", ctypes.c_int32), ("paths", ctypes.c_int64),
                ("converged", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("nonzero", ctypes.c_int64), ("kernel_ms", ctypes.c_double)]


class HpTiming(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("endgame_ms", ctypes.c_double),
                ("post_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("launches", ctypes.c_int64), ("paths_per_wave", ctypes.c_int32),
                ("max_n", ctypes.c_int32), ("groups", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("lanes_per_path", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32)]


class HpTuneChoice(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("lanes_per_path", ctypes.c_int32),
                ("paths_per_wave", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("ms", ctypes.c_double), ("ms_default", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("cached", ctypes.c_int32)]


STATS_DTYPE = np.dtype([("steps", np.int32), ("rejections", np.int32),
                        ("newton_iters", np.int32), ("evals", np.int32),
                        ("solves", np.int32), ("pad", np.int32),
                        ("t_final", np.float64), ("residual", np.float64)])

_lock = threading.Lock()
_lib = None


class HomotopyError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhomotopy error {code}: {msg}")
        self.code = code


def load():
    """Loads libhomotopy.so; raises if it is not built (no fallback path)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(SO_PATH):
            raise ImportError(f"{SO_PATH} is not built; run paper_1804_03807_amd/build.py "
                              "(or __graft_entry__.build()) first")
        # torch ships its own HIP runtime whose soname (libamdhip64.so.7) is
        # the one libhomotopy needs; loading torch first makes the process use
        # a single runtime, so device pointers and streams from torch are valid
        # in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(SO_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        c64 = HpC64
        P = ctypes.POINTER
        sig = {
            "hp_context_create": (ctypes.c_int, [ctypes.c_int, P(vp)]),
            "hp_context_destroy": (None, [vp]),
            "hp_last_error": (ctypes.c_char_p, []),
            "hp_default_tolerances": (None, [P(HpTolerances)]),
            "hp_last_timing": (ctypes.c_int, [vp, P(HpTiming)]),
            "hp_path_count": (i64, [P(HpSystem)]),
            "hp_track_paths": (ctypes.c_int, [vp, P(HpSystem), P(HpSystem), vp, i64, c64,
                                              P(HpTolerances), vp, vp, vp, i32]),
            "hp_plan_create": (ctypes.c_int, [vp, P(HpSystem), c64, P(HpTolerances), i32, P(vp)]),
            "hp_plan_destroy": (None, [vp]),
            "hp_plan_set_variant": (ctypes.c_int, [vp, i32]),
            "hp_plan_track_device": (ctypes.c_int, [vp, vp, i64, vp, vp, vp, i32, vp]),
            "hp_batch_layout": (ctypes.c_int, [vp, i32, vp, vp]),
            "hp_track_batch": (ctypes.c_int, [vp, vp, i32, vp, P(HpTolerances), vp, vp, vp]),
            "hp_find_duplicates": (i64, [i32, i64, vp, vp, ctypes.c_double, vp, i64]),
            "hp_solve": (ctypes.c_int, [vp, P(HpSystem), c64, P(HpTolerances), vp, vp, vp, vp]),
            "hp_find_duplicates_device": (ctypes.c_int, [vp, i32, i64, vp, vp, ctypes.c_double,
                                                         vp, i64, P(i64), vp]),
            "hp_plan_solve_device": (ctypes.c_int, [vp, vp, vp, vp, P(i64), P(i64), vp]),
            "hp_membership_test": (ctypes.c_int, [vp, P(HpSystem), i32, vp, i64, vp, i32,
                                                  P(HpTolerances), ctypes.c_double, vp, vp, vp]),
            "hp_track_paths_dd": (ctypes.c_int, [vp, P(HpSystem), vp, i64, c64, P(HpTolerances),
                                                 vp, vp, vp, vp]),
            "hp_default_tolerances_dd": (None, [P(HpTolerances)]),
            "hp_cascade": (ctypes.c_int, [vp, P(HpSystem), i32, vp, P(HpTolerances),
                                          ctypes.c_double, P(HpCascadeStage), vp, vp, i64,
                                          P(i64)]),
            "hp_find_duplicates_device_static": (ctypes.c_int, [vp, i32, i64, vp, vp,
                                                                ctypes.c_double, vp, i64, P(i64),
                                                                vp]),
            "hp_server_create": (ctypes.c_int, [vp, ctypes.c_size_t, P(vp)]),
            "hp_server_submit": (ctypes.c_int, [vp, P(HpSystem), c64, P(HpTolerances), P(i64)]),
            "hp_server_poll": (ctypes.c_int, [vp, i64, P(i32)]),
            "hp_server_wait": (ctypes.c_int, [vp, i64, vp, vp, vp, P(ctypes.c_double)]),
            "hp_server_peak_bytes": (ctypes.c_int, [vp, P(ctypes.c_size_t)]),
            "hp_server_destroy": (None, [vp]),
            "hp_server_set_slice": (ctypes.c_int, [vp, ctypes.c_double, i32]),
            "hp_plan_set_launch": (ctypes.c_int, [vp, i32, i32]),
            "hp_spec_compile_form": (ctypes.c_int, [P(HpSystem), i32, P(i64)]),
            "hp_plan_create_general": (ctypes.c_int, [vp, P(HpSystem), P(HpSystem), vp, i64, c64,
                                                      P(HpTolerances), i32, P(vp)]),
            "hp_plan_tuning": (ctypes.c_int, [vp, P(HpTuneChoice)]),
            "hp_tune_batch": (ctypes.c_int, [vp, vp, i32, vp, P(HpTolerances), P(HpTuneChoice)]),
            "hp_server_info_get": (ctypes.c_int, [vp, P(HpServerInfo)]),
            "hp_spec_compile": (ctypes.c_int, [P(HpSystem), P(i64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return L


def check(rc):
    if rc != HP_OK:
        msg = load().hp_last_error().decode(errors="replace")
        raise HomotopyError(rc, msg)
    return rc
