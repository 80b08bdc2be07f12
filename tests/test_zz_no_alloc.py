"""The allocation-free adjoint step (xfdtd_adjoint_step_noalloc), called
through the C interface: on two calls in a row, the second on a smaller grid,
its adjoint fields and coefficient gradient equal those of
xfdtd_adjoint_step bitwise (same kernels, same summation order), in FP64 and
FP32; oversized launches are rejected before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import fdtd as O
import paper_1710_06829_amd as pkg
from paper_1710_06829_amd import _binding as B
from tests._gpu import DEV, to_dev

pytestmark = pytest.mark.gpu


def _arr(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def _call(fn, solver, lam_in, lam_out, e_n, grad):
    solver._bind()
    return fn(solver._h, _arr(lam_in), _arr(lam_out), _arr(e_n), ctypes.c_void_p(grad.data_ptr()))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_adjoint_step_equals_adjoint_step(dtype):
    L = B.lib()
    beta, delta = S.distinct_beta_delta(1701)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c)
    for shape, seed in [((40, 33, 130), 1702), ((9, 7, 20), 1703)]:  # second call: a smaller grid
        f0 = to_dev(S.uniform_fields(shape, seed), dtype)
        s = pkg.Solver(f0, dt, c, scratch=False)
        lam = to_dev(S.uniform_fields(shape, seed + 10), dtype)
        out_ref = [torch.empty_like(t) for t in lam]
        out_na = [torch.full_like(t, float("nan")) for t in lam]
        g_ref = torch.zeros(12, dtype=torch.float64, device=DEV)
        g_na = torch.zeros(12, dtype=torch.float64, device=DEV)
        assert _call(L.xfdtd_adjoint_step, s, lam, out_ref, f0[:3], g_ref) == 0
        assert _call(L.xfdtd_adjoint_step_noalloc, s, lam, out_na, f0[:3], g_na) == 0, L.xfdtd_last_error()
        torch.cuda.synchronize()
        for a, b in zip(out_na, out_ref):
            assert torch.equal(a, b), shape
        assert torch.equal(g_na, g_ref), (shape, g_na, g_ref)
        assert torch.count_nonzero(g_ref) == 12
        # and the sums accumulate into grad like the allocating step
        assert _call(L.xfdtd_adjoint_step_noalloc, s, lam, out_na, f0[:3], g_na) == 0
        torch.cuda.synchronize()
        assert torch.allclose(g_na, 2 * g_ref, rtol=1e-14, atol=0)


def test_noalloc_adjoint_step_rejects_oversized_launches_before_device_work():
    # a 1 x 16384 x 16384 plane needs far more than 16384 adjoint workgroups
    L = B.lib()
    c = O.yee_coeffs()
    dt = 0.5 * O.cfl_dt(c)
    g = B.make_grid((1, 16384, 16384))
    h = ctypes.c_void_p()
    assert L.xfdtd_create(ctypes.byref(g), dt, B.dbl_array(c, 12), B.XFDTD_F32, 0, ctypes.byref(h)) == 0
    try:
        t = torch.empty(6, 1, 16384, 16384, dtype=torch.float32, device=DEV)
        assert L.xfdtd_bind(h, _arr(list(t)), None, None) == 0
        grad = torch.zeros(12, dtype=torch.float64, device=DEV)
        u = torch.empty(6, 1, 16384, 16384, dtype=torch.float32, device=DEV)
        v = torch.empty(6, 1, 16384, 16384, dtype=torch.float32, device=DEV)
        rc = L.xfdtd_adjoint_step_noalloc(h, _arr(list(u)), _arr(list(v)), _arr(list(t[:3])),
                                          ctypes.c_void_p(grad.data_ptr()))
        assert rc == -1 and b"workgroups" in L.xfdtd_last_error(), L.xfdtd_last_error()
        torch.cuda.synchronize()
        assert torch.count_nonzero(grad) == 0
    finally:
        L.xfdtd_destroy(h)
