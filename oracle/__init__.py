"""Test-only FP64 oracle (see ``oracle.fdtd``) plus a ctypes loader for the
plain-C oracle ``fdtd_oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
the CPU-baseline leg of bench.py.  The HIP library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import fdtd  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# XFDTD_ORACLE_LIB names another build of the C oracle (e.g. a sanitized one)
LIB_PATH = os.environ.get("XFDTD_ORACLE_LIB") or os.path.join(_HERE, "libfdtd_oracle.so")
SRC_PATH = os.path.join(_HERE, "fdtd_oracle.c")
_lib = None


def build_c_oracle(verbose: bool = False, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the plain-C oracle (gcc, OpenMP, no FMA contraction) to `out`
    (default: the in-tree library).  sanitize=True builds it with ROCm's clang
    under AddressSanitizer and UBSan instead, for a process that preloads that
    clang's ASan runtime (the sanitized host build of libxfdtd uses the same
    one)."""
    out = out or LIB_PATH
    if sanitize:
        cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan",
               "-fno-omit-frame-pointer", SRC_PATH, "-o", out + ".tmp", "-lm"]
    else:
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               SRC_PATH, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def c_oracle():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_c_oracle()
        lib = ctypes.CDLL(LIB_PATH)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        lib.oracle_run.argtypes = [i64, i64, i64, dp, ctypes.c_double, dp,
                                   ctypes.POINTER(dp), i64]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_step_at.argtypes = [i64, i64, i64, dp, ctypes.c_double, dp,
                                       ctypes.POINTER(dp), ctypes.POINTER(i64), i64, dp]
        lib.oracle_step_at.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def c_run(fields, n, coeffs, dt, d=(1.0, 1.0, 1.0)):
    """n steps of the C oracle; returns six new float64 arrays."""
    lib = c_oracle()
    f = [np.ascontiguousarray(np.array(x, dtype=np.float64, copy=True)) for x in fields]
    nz, ny, nx = f[0].shape
    dd = np.asarray(d, dtype=np.float64)
    cc = np.asarray(coeffs, dtype=np.float64)
    arr = (ctypes.POINTER(ctypes.c_double) * 6)(*[_dptr(x) for x in f])
    rc = lib.oracle_run(nx, ny, nz, _dptr(dd), float(dt), _dptr(cc), arr, int(n))
    if rc != 0:
        raise RuntimeError("oracle_run failed")
    return f


def c_step_at(fields, idx, coeffs, dt, d=(1.0, 1.0, 1.0)):
    """One step evaluated only at flat site indices ``idx``; returns (m, 6)."""
    lib = c_oracle()
    f = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) for x in fields]
    nz, ny, nx = f[0].shape
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.zeros((idx.size, 6))
    dd = np.asarray(d, dtype=np.float64)
    cc = np.asarray(coeffs, dtype=np.float64)
    arr = (ctypes.POINTER(ctypes.c_double) * 6)(*[_dptr(x) for x in f])
    rc = lib.oracle_step_at(nx, ny, nz, _dptr(dd), float(dt), _dptr(cc), arr,
                            idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            idx.size, _dptr(out))
    if rc != 0:
        raise RuntimeError("oracle_step_at failed")
    return out
