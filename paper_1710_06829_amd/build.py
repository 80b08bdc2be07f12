"""Build libxfdtd.so (HIP, gfx950) in place.  Run: python -m paper_1710_06829_amd.build"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libxfdtd.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["host.cpp", "batch.cpp", "norm.cpp", "kernels_step.hip", "kernels_diag.hip", "kernels_adjoint.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off: some of their forms have given
    # wrong results, without error, on this GPU family
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only inside one source expression, so every
    # tiling and kernel variant rounds a cell's update the same way
    "-ffp-contract=on",
    "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-result",
]


# roctx ranges around run, tune and the gradient phases (ROCm's roctx library)
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *LIBS, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


# Host-side sanitizers for the build variant below: each -fsanitize= applies
# to the host compilation only (device code is built as in build()).
HOST_SOURCES = ["host.cpp", "batch.cpp", "norm.cpp"]
SAN_FLAGS = [
    "-O1", "-g", "-Wno-unused-value",
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
]


def build_host_sanitized(out_dir: str, verbose: bool = False) -> str:
    """libxfdtd with its host code (argument validation, work lists, tuning,
    checkpoint schedules, the C ABI) built under AddressSanitizer and UBSan,
    linked with the device objects of build() (compiled here if that build
    has not run).  The result is loaded by a process that preloads ROCm
    clang's ASan runtime and names it in XFDTD_LIB."""
    os.makedirs(out_dir, exist_ok=True)

    def host_obj(src: str) -> str:
        obj = os.path.join(out_dir, src + ".san.o")
        cmd = [HIPCC, *FLAGS, *SAN_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    def device_obj(src: str) -> str:
        obj = os.path.join(BUILD, src + ".o")
        return obj if os.path.exists(obj) else _compile(src)

    os.makedirs(BUILD, exist_ok=True)
    kernels = [s for s in SOURCES if s not in HOST_SOURCES]
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(host_obj, HOST_SOURCES)) + list(ex.map(device_obj, kernels))
    out = os.path.join(out_dir, "libxfdtd_hostsan.so")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", *objs, *LIBS, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
