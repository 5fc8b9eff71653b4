"""ctypes declarations of libpso.so (include/pso.h).  Loading fails loudly if
the library has not been built: there is no other implementation."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpso.so")

PSO_OK, PSO_EINVAL, PSO_ENOMEM, PSO_EDEVICE, PSO_EAGAIN, PSO_ESTATE = 0, -1, -2, -3, -4, -5
PSO_ECANCELED, PSO_ETIMEDOUT = -6, -7
PSO_SPHERE, PSO_RASTRIGIN, PSO_ROSENBROCK, PSO_ACKLEY, PSO_CUBIC = 0, 1, 2, 3, 4
PSO_SYNC, PSO_ASYNC, PSO_REDUCE, PSO_REDUCE_UNROLLED, PSO_PERSISTENT = 0, 1, 2, 3, 4

c_int, c_i32, c_i64, c_u64, c_f, c_size, c_vp = (ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                                   ctypes.c_float, ctypes.c_size_t, ctypes.c_void_p)
P = ctypes.POINTER
c_f64 = ctypes.c_double


class PsoDesc(ctypes.Structure):
    """struct pso_desc of include/pso.h."""
    _fields_ = [("fitness_id", ctypes.c_int32), ("D", ctypes.c_int32), ("N", ctypes.c_int64),
                ("bounds", ctypes.c_float * 2), ("w", ctypes.c_float), ("c1", ctypes.c_float),
                ("c2", ctypes.c_float), ("vmax", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("shift", ctypes.c_void_p), ("max_iter", ctypes.c_int64), ("tol", ctypes.c_float),
                ("f_star", ctypes.c_float)]


class PsoBatchShape(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("grid", ctypes.c_int32), ("part_work", ctypes.c_int64),
                ("stage_kib", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PsoResult(ctypes.Structure):
    """struct pso_result of include/pso.h."""
    _fields_ = [("gbest_value", ctypes.c_float), ("status", ctypes.c_int32), ("gbest_iter", ctypes.c_int64),
                ("iters", ctypes.c_int64), ("gbest_pos", ctypes.c_void_p)]


class PsoServerCounters(ctypes.Structure):
    """struct pso_server_counters of include/pso.h."""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("launches", ctypes.c_uint64), ("mem_budget", ctypes.c_size_t),
                ("mem_used", ctypes.c_size_t), ("mem_peak", ctypes.c_size_t), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("cancelled", ctypes.c_uint64),
                ("timed_out", ctypes.c_uint64)]


# name -> (restype, argtypes), in the order of include/pso.h
SIGNATURES = {
    "pso_last_error": (ctypes.c_char_p, []),
    "pso_workspace_bytes": (c_size, [c_i64, c_i32]),
    "pso_create": (c_int, [c_int, c_i64, c_i32, P(c_f), c_f, c_f, c_f, c_f, c_u64, P(c_vp)]),
    "pso_create_in": (c_int, [c_int, c_i64, c_i32, P(c_f), c_f, c_f, c_f, c_f, c_u64, c_vp, c_size, c_vp, P(c_vp)]),
    "pso_set_shift": (c_int, [c_vp, P(c_f)]),
    "pso_set_variant": (c_int, [c_vp, c_int]),
    "pso_reset": (c_int, [c_vp]),
    "pso_step": (c_int, [c_vp]),
    "pso_run": (c_int, [c_vp, c_i64, c_f, c_f, P(c_f), P(c_f), P(c_i64), P(c_i64)]),
    "pso_get_best": (c_int, [c_vp, P(c_f), P(c_f), P(c_i64), P(c_i64)]),
    "pso_get_history": (c_int, [c_vp, c_i64, c_i64, P(c_u64)]),
    "pso_get_state": (c_int, [c_vp, P(c_f), P(c_f), P(c_f), P(c_f), P(c_u64), P(c_f), P(c_i64), P(c_i64)]),
    "pso_set_state": (c_int, [c_vp, P(c_f), P(c_f), P(c_f), P(c_f), c_u64, P(c_f), c_i64, c_i64]),
    "pso_get_counters": (c_int, [c_vp, P(c_u64)]),
    "pso_get_async_counters": (c_int, [c_vp, P(c_u64), P(c_u64)]),
    "pso_sync": (c_int, [c_vp]),
    "pso_destroy": (c_int, [c_vp]),
    "pso_batch_create": (c_int, [P(PsoDesc), c_i64, c_vp, P(c_vp)]),
    "pso_batch_launch": (c_int, [c_vp]),
    "pso_batch_results": (c_int, [c_vp, P(PsoResult)]),
    "pso_batch_destroy": (c_int, [c_vp]),
    "pso_batch_run": (c_int, [P(PsoDesc), c_i64, P(PsoResult)]),
    "pso_batch_run_static": (c_int, [P(PsoDesc), c_i64, P(PsoResult), c_vp]),
    "pso64_create": (c_int, [c_int, c_i64, c_i32, P(c_f), c_f, c_f, c_f, c_f, c_u64, P(c_vp)]),
    "pso64_set_shift": (c_int, [c_vp, P(c_f)]),
    "pso64_reset": (c_int, [c_vp]),
    "pso64_step": (c_int, [c_vp]),
    "pso64_run": (c_int, [c_vp, c_i64, c_f64, c_f64, P(c_f64), P(c_f64), P(c_i64), P(c_i64)]),
    "pso64_get_state": (c_int, [c_vp, P(c_f64), P(c_f64), P(c_f64), P(c_f64), P(c_i64), P(c_i64)]),
    "pso64_eval": (c_int, [c_vp, P(c_f64), c_i64, P(c_f64)]),
    "pso64_destroy": (c_int, [c_vp]),
    "pso_set_max_lead": (c_int, [c_vp, c_i64]),
    "pso_batch_get_shape": (c_int, [c_vp, P(PsoBatchShape)]),
    "pso_batch_set_shape": (c_int, [c_vp, P(PsoBatchShape)]),
    "pso_batch_autotune": (c_int, [c_vp, c_i64, P(PsoBatchShape)]),
    "pso_server_create": (c_int, [c_size, c_i64, P(c_vp)]),
    "pso_server_submit": (c_int, [c_vp, P(PsoDesc), P(c_u64)]),
    "pso_server_poll": (c_int, [c_vp, c_u64, P(PsoResult), P(ctypes.c_double)]),
    "pso_server_cancel": (c_int, [c_vp, c_u64]),
    "pso_server_set_deadline": (c_int, [c_vp, c_u64, ctypes.c_double]),
    "pso_server_stats": (c_int, [c_vp, P(PsoServerCounters)]),
    "pso_server_destroy": (c_int, [c_vp]),
}

_lib = None


def _single_hip_runtime():
    """PyTorch ships its own HIP runtime, which it loads under a file name
    different from the system one.  Importing torch before libpso.so makes
    libpso bind to that same runtime, so a process never holds two (two
    runtimes cannot share device pointers or streams)."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load(path: str = LIB_PATH):
    """Load libpso.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is None:
        _single_hip_runtime()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run paper_2205_01313_amd/build.py (hipcc, gfx950)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
