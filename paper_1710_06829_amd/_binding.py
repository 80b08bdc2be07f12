"""ctypes binding of libxfdtd (argument marshalling only).

Every numerical step runs in the HIP library; this module converts torch
tensors into device pointers and a HIP stream, and raises on error codes.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# XFDTD_LIB names another build of the same library (e.g. one whose host code
# is built with sanitizers); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("XFDTD_LIB") or os.path.join(HERE, "libxfdtd.so")

XFDTD_F32 = 1
XFDTD_F64 = 2
STATUS = {0: "XFDTD_OK", -1: "XFDTD_EINVAL", -2: "XFDTD_EUNSTABLE", -3: "XFDTD_ENONFINITE",
          -4: "XFDTD_EHIP", -5: "XFDTD_ESTATE"}
WARN_ALPHA = 1


class XfdtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


class StencilProblem(ctypes.Structure):
    """xfdtd_stencil_problem."""
    _fields_ = [("nparam", ctypes.c_int32), ("alpha_rule", ctypes.c_int32), ("dt_mode", ctypes.c_int32),
                ("dt_param", ctypes.c_int32), ("base", ctypes.c_double * 13), ("map", ctypes.c_double * (13 * 8)),
                ("lo", ctypes.c_double * 8), ("hi", ctypes.c_double * 8), ("dims", ctypes.c_int32),
                ("weight", ctypes.c_int32), ("width", ctypes.c_double), ("n", ctypes.c_int64),
                ("starts", ctypes.c_int32), ("max_iter", ctypes.c_int32)]


class Stats(ctypes.Structure):
    """xfdtd_stats."""
    _fields_ = [(n, ctypes.c_int64) for n in ("run_calls", "steps", "in_place_steps", "fused_launches",
                                               "two_step_launches", "graph_replays", "graph_captures", "tunes",
                                               "grad_forward_steps", "adjoint_steps", "recomputed_steps")] + \
               [(n, ctypes.c_double) for n in ("model_bytes", "elapsed_ms", "gcells_per_s")]


XFDTD_WEIGHT_UNIT = 0
XFDTD_WEIGHT_AXIS = 1

_lib = None

# name -> (argtypes, restype); every symbol include/xfdtd.h declares
_vp, _dp, _i64, _int = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int
_GP = ctypes.POINTER(Grid)
SIGNATURES = {
    "xfdtd_abi_version": ([], _int),
    "xfdtd_last_error": ([], ctypes.c_char_p),
    "xfdtd_cfl_limit": ([_GP, _dp, _dp, _dp, _dp], _int),
    "xfdtd_consistent_alpha": ([_dp], _int),
    "xfdtd_create": ([_GP, ctypes.c_double, _dp, _int, _int, ctypes.POINTER(_vp)], _int),
    "xfdtd_destroy": ([_vp], None),
    "xfdtd_flags": ([_vp], _int),
    "xfdtd_bind": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp], _int),
    "xfdtd_step_faraday": ([_vp], _int),
    "xfdtd_step_ampere": ([_vp], _int),
    "xfdtd_step_ampere_current": ([_vp, ctypes.POINTER(_vp)], _int),
    "xfdtd_run": ([_vp, _i64], _int),
    "xfdtd_get_weights": ([_vp, _dp, ctypes.POINTER(_int)], _int),
    "xfdtd_tune": ([_vp, _int, _dp], _int),
    "xfdtd_launch_config": ([_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                             ctypes.POINTER(_int)], _int),
    "xfdtd_set_steps_per_pass": ([_vp, _int], _int),
    "xfdtd_launch_config2": ([_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                              ctypes.POINTER(_int), ctypes.POINTER(_int)], _int),
    "xfdtd_dispersion": ([_GP, ctypes.c_double, _dp, _vp, _i64, _vp, _vp, _vp, _vp], _int),
    "xfdtd_dispersion_norm": ([_GP, ctypes.c_double, _dp, _int, _i64, _int, ctypes.c_double, _dp, _dp, _vp],
                              _int),
    "xfdtd_optimize_stencil": ([_GP, ctypes.POINTER(StencilProblem), _dp, _dp, _dp, _dp, ctypes.POINTER(_int),
                                _vp], _int),
    "xfdtd_divergence": ([_vp, _vp, _vp], _int),
    "xfdtd_divergence_max": ([_vp, _vp, _vp, _dp], _int),
    "xfdtd_adjoint_step": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp], _int),
    "xfdtd_get_stats": ([_vp, ctypes.POINTER(Stats)], _int),
    "xfdtd_run_checked": ([_vp, _i64, _i64, ctypes.POINTER(_i64)], _int),
    "xfdtd_reset_stats": ([_vp, _int], _int),
    "xfdtd_adjoint_step_noalloc": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp],
                                   _int),
    "xfdtd_grad_workspace": ([_vp, _i64, _i64, ctypes.POINTER(ctypes.c_uint64)], _int),
    "xfdtd_grad_forward": ([_vp, _i64, _i64, _vp, ctypes.c_uint64], _int),
    "xfdtd_grad_backward": ([_vp, _i64, _i64, _vp, ctypes.c_uint64, ctypes.POINTER(_vp), _dp], _int),
    "xfdtd_batch_create": ([_GP, _dp, _dp, _i64, _int, _int, ctypes.POINTER(_vp)], _int),
    "xfdtd_batch_destroy": ([_vp], None),
    "xfdtd_batch_bind": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp], _int),
    "xfdtd_batch_tune": ([_vp, _int, _dp], _int),
    "xfdtd_batch_set_config": ([_vp, _int, _int, _int, _int], _int),
    "xfdtd_batch_get_config": ([_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                                ctypes.POINTER(_int), ctypes.POINTER(_int)], _int),
    "xfdtd_batch_run": ([_vp, _i64], _int),
    "xfdtd_batch_set_steps_per_pass": ([_vp, _int], _int),
    "xfdtd_batch_get_steps_per_pass": ([_vp, ctypes.POINTER(_int)], _int),
    "xfdtd_batch_get_adjoint_config": ([_vp] + [ctypes.POINTER(_int)] * 4, _int),
    "xfdtd_batch_run_eager": ([_vp, _i64], _int),
    "xfdtd_batch_grad_workspace": ([_vp, _i64, _i64, ctypes.POINTER(ctypes.c_uint64)], _int),
    "xfdtd_batch_grad_forward": ([_vp, _i64, _i64, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint64)], _int),
    "xfdtd_batch_grad_backward": ([_vp, _i64, _i64, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(_vp), _dp], _int),
}


def lib():
    """The loaded libxfdtd (raises ImportError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"libxfdtd.so not found at {LIB_PATH}: build it with "
                "`python -m paper_1710_06829_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int):
    if rc != 0:
        msg = lib().xfdtd_last_error()
        raise XfdtdError(rc, msg.decode() if msg else "")
    return rc


def dbl_array(values, n=None):
    vals = [float(v) for v in values]
    if n is not None and len(vals) != n:
        raise ValueError(f"expected {n} values, got {len(vals)}")
    return (ctypes.c_double * len(vals))(*vals)


def make_grid(shape, spacing=(1.0, 1.0, 1.0)) -> Grid:
    """Grid from a field shape (nz, ny, nx) and spacings (dx, dy, dz)."""
    nz, ny, nx = (int(v) for v in shape)
    dx, dy, dz = (float(v) for v in spacing)
    return Grid(nx, ny, nz, dx, dy, dz)
