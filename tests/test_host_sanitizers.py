"""The host logic under AddressSanitizer and UBSan (CPU only, no GPU calls).

Builds libxfdtd with its host code sanitized (device code as usual) and the C
oracle with the same clang sanitizers, then runs the host-side tests
(tests/test_abi.py: argument validation, error paths, work-list and workspace
arithmetic, the exported symbols; the C-oracle tests of
tests/test_oracle_step.py) in a child process that preloads clang's ASan
runtime.  Any ASan or UBSan report fails the run.

One test is left out there: test_host_allocation_failure_is_an_error_code_not_
an_exception caps the child's address space so that operator new fails, and
ASan's allocator reports such a failure and aborts instead of throwing
std::bad_alloc; the plain CPU suite runs it.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.skipif(not shutil.which("/opt/rocm/bin/hipcc") or _asan_runtime() is None,
                    reason="needs hipcc and ROCm clang's ASan runtime")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    import oracle
    from paper_1710_06829_amd import build

    lib = build.build_host_sanitized(str(tmp_path))
    orc = oracle.build_c_oracle(out=str(tmp_path / "liboracle_hostsan.so"), sanitize=True)
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": _asan_runtime(),
        # leaks: the interpreter's own allocations at exit are not ours
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "XFDTD_LIB": lib,
        "XFDTD_ORACLE_LIB": orc,
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
           "-k", "not allocation_failure",
           os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_oracle_step.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out and "failed" not in out, out[-3000:]
