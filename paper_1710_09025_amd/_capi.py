"""ctypes declarations of the C ABI in include/pamc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpamc.so")

OK = 0
ERR_INVALID = -1
ERR_NOMEM = -2
ERR_CAPACITY = -3
ERR_EXTINCT = -4
ERR_DEVICE = -5
ERR_STATE = -6
ERR_BUSY = -7
ERR_REJECTED = -8

SPINS_INT8 = 0
SPINS_PACKED = 1

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [
        ("spin_format", ctypes.c_int),
        ("capacity", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_user", ctypes.c_void_p),
        ("overlap_steps", ctypes.POINTER(ctypes.c_int32)),
        ("n_overlap_steps", ctypes.c_int),
        ("fuse_gather", ctypes.c_int),
        ("device", ctypes.c_int),
        ("tile_rows", ctypes.c_int),
        ("graphs", ctypes.c_int),
        ("timing", ctypes.c_int),
        ("group_replicas", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("pop_schedule", ctypes.POINTER(ctypes.c_int64)),
        ("real_couplings", ctypes.c_int),
        ("icm_rounds", ctypes.c_int),
        ("icm_beta_min", ctypes.c_double),
        ("dim", ctypes.c_int),
    ]


class StepObs(ctypes.Structure):
    _fields_ = [
        ("beta", ctypes.c_double),
        ("R", ctypes.c_int64),
        ("sum_E", ctypes.c_int64),
        ("sum_E2", ctypes.c_int64),
        ("sum_E2_hi", ctypes.c_int64),
        ("E_min", ctypes.c_int64),
        ("E_max", ctypes.c_int64),
        ("mean_E", ctypes.c_double),
        ("e", ctypes.c_double),
        ("C_V", ctypes.c_double),
        ("lnQ", ctypes.c_double),
        ("lnZ", ctypes.c_double),
        ("betaF", ctypes.c_double),
        ("f", ctypes.c_double),
        ("S_f", ctypes.c_double),
        ("rho_s", ctypes.c_double),
        ("q_abs", ctypes.c_double),
        ("q2", ctypes.c_double),
        ("q4", ctypes.c_double),
        ("g_SG", ctypes.c_double),
        ("measured", ctypes.c_int32),
    ]


class State(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int),
        ("R", ctypes.c_int64),
        ("lnZ", ctypes.c_double),
        ("spins", ctypes.c_void_p),
        ("E", ctypes.c_void_p),
        ("family", ctypes.c_void_p),
        ("E_fixed", ctypes.c_void_p),
    ]


class Instance(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int),
        ("couplings", ctypes.c_void_p),
        ("R", ctypes.c_int64),
        ("beta", ctypes.c_void_p),
        ("n_temps", ctypes.c_int),
        ("sweeps", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("pop_schedule", ctypes.c_void_p),
        ("real_couplings", ctypes.c_void_p),
    ]


class ServerOptions(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int), ("device", ctypes.c_int), ("autotune", ctypes.c_int),
                ("spin_format", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("n_temps", ctypes.c_int),
        ("obs", ctypes.POINTER(StepObs)),
        ("submit_time_s", ctypes.c_double),
        ("admit_time_s", ctypes.c_double),
        ("finish_time_s", ctypes.c_double),
    ]


# name -> (restype, argtypes)
P = ctypes.c_void_p
SIGNATURES = {
    "pamc_default_options": (None, [ctypes.POINTER(Options)]),
    "pamc_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(Options),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double)]),
    "pamc_create": (ctypes.c_int, [ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_uint64, ctypes.POINTER(Options), ctypes.POINTER(P)]),
    "pamc_create_real": (ctypes.c_int, [ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint64, ctypes.POINTER(Options), ctypes.POINTER(P)]),
    "pamc_anneal": (ctypes.c_int, [P, ctypes.c_int]),
    "pamc_anneal_async": (ctypes.c_int, [P, ctypes.c_int]),
    "pamc_sync": (ctypes.c_int, [P]),
    "pamc_observables": (ctypes.c_int, [P, ctypes.POINTER(StepObs), ctypes.c_int]),
    "pamc_overlap_hist": (ctypes.c_int, [P, ctypes.c_int, P]),
    "pamc_step_sums": (ctypes.c_int, [P, P, P, ctypes.c_int]),
    "pamc_get_shape": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]),
    "pamc_sweep_shape": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "pamc_get_state": (ctypes.c_int, [P, ctypes.POINTER(State)]),
    "pamc_set_state": (ctypes.c_int, [P, ctypes.POINTER(State)]),
    "pamc_thresholds": (ctypes.c_int, [P, P, P]),
    "pamc_phase_times": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "pamc_footprint": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(Options)]),
    "pamc_make_pm_j": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, P]),
    "pamc_calibrate": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pamc_rho_f": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P, P, P, P]),
    "pamc_destroy": (None, [P]),
    "pamc_anneal_static": (ctypes.c_int, [ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_uint64, P, ctypes.POINTER(StepObs), ctypes.POINTER(State)]),
    "pamc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pamc_last_error": (ctypes.c_char_p, []),
    "pamc_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Instance), ctypes.POINTER(Options),
                                         ctypes.POINTER(P)]),
    "pamc_batch_anneal": (ctypes.c_int, [P]),
    "pamc_batch_observables": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(StepObs), ctypes.c_int]),
    "pamc_batch_get_state": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(State)]),
    "pamc_batch_shape": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "pamc_batch_destroy": (None, [P]),
    "pamc_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]),
    "pamc_server_submit": (ctypes.c_int, [P, ctypes.POINTER(Instance), ctypes.POINTER(ctypes.c_uint64)]),
    "pamc_server_poll": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "pamc_server_cancel": (ctypes.c_int, [P, ctypes.c_uint64]),
    "pamc_server_stats": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "pamc_server_usage": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pamc_server_destroy": (None, [P]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Loads the in-tree libpamc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch-ROCm bundles its own HIP runtime under the same soname;
        # load it first so that the library binds to that single runtime
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is missing: build it with `python -m paper_1710_09025_amd.build` "
                "(there is no fallback implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
