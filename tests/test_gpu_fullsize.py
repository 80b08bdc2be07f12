"""Parity at the full 512x256x256 size, in the launch configuration the
benchmark times (fused kernel, tiling chosen by the autotuner):

* 1000 steps of the Gaussian-pulse workload against sampled outputs of the
  FP64 oracle (stored by tests/golden/make_c2_samples.py): FP64 to 1e-12,
  FP32 to 1e-5 relative L2 both against the oracle run with the FP32 weights
  (FP32 convention of tests/_fp32.py) and against the plain-coefficient
  oracle from FP64 inputs;
* the same 1000 steps on the FP64 two-step kernel (FP64's non-default
  kernel), sampled, to 1e-12;
* 3 steps, full field, against the C oracle;
* 1000 steps of an exact discrete eigenmode against its closed form;
* the 1024x256x256 pulse of the sustained run: 100 steps against sampled
  outputs of the FP64 oracle (tests/golden/make_c5a_samples.py), same bars;
* the largest plane the library accepts (16384 x 16384 = 2^28 cells, where
  the kernels' 32-bit lane byte offsets come closest to their limit): an
  exact eigenmode after 20 steps against its closed form at sampled sites.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from oracle import fdtd as O
import paper_1710_06829_amd as pkg
from tests import _fp32
from tests import workloads as W
from tests._gpu import DEV, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sampled(tensors, idx):
    torch.cuda.synchronize()
    ii = torch.from_numpy(idx).to(DEV)
    return np.stack([t.reshape(-1)[ii].double().cpu().numpy() for t in tensors], axis=1)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype,variant,tol", [(torch.float64, "exact", 1e-12),
                                               (torch.float32, "fp32", 1e-5),
                                               # FP32 against the plain-coefficient FP64
                                               # oracle from FP64 inputs: the literal bar
                                               (torch.float32, "exact", 1e-5)],
                         ids=["fp64-vs-oracle", "fp32-vs-fp32-weight-oracle", "fp32-vs-plain-oracle"])
def test_c2_pulse_1000_steps_vs_oracle_samples(dtype, variant, tol):
    path = os.path.join(GOLD, f"c2_pulse_{variant}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    ref = np.load(path)
    f0, c, dt, sp = W.c2_inputs()
    assert np.array_equal(ref["coeffs"], c) and float(ref["dt"]) == dt
    t = to_dev(f0, dtype)
    del f0
    s = pkg.Solver(t, dt, c, spacing=sp)
    lc = s.tune()  # the launch configuration the benchmark times
    s.run(int(ref["steps"]))
    got = _sampled(t, ref["idx"])
    err = _rel(got, ref["vals"])
    print(f"c2 {dtype} vs {variant} oracle: sampled rel L2 = {err:.3e} ({lc})")
    assert err < tol


def test_c2_pulse_1000_steps_fp64_two_step_kernel_vs_oracle_samples():
    """The FP64 two-step kernel (24x8 tiles, not FP64's default) over the
    1000 steps of the pulse workload: 500 launches, sampled outputs against
    the FP64 oracle to 1e-12."""
    path = os.path.join(GOLD, "c2_pulse_exact.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    ref = np.load(path)
    f0, c, dt, sp = W.c2_inputs()
    t = to_dev(f0, torch.float64)
    del f0
    s = pkg.Solver(t, dt, c, spacing=sp)
    s.set_steps_per_pass(2)
    s.reset_stats()
    s.run(int(ref["steps"]))
    assert s.stats()["two_step_launches"] == int(ref["steps"]) // 2
    err = _rel(_sampled(t, ref["idx"]), ref["vals"])
    print(f"c2 FP64 two-step kernel vs oracle: sampled rel L2 = {err:.3e} ({s.launch_config()['two_step']})")
    assert err < 1e-12


@pytest.mark.parametrize("dtype,variant,tol", [(torch.float64, "exact", 1e-12),
                                               (torch.float32, "fp32", 1e-5)])
def test_c5a_pulse_100_steps_vs_oracle_samples(dtype, variant, tol):
    path = os.path.join(GOLD, f"c5a_pulse_{variant}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    ref = np.load(path)
    f0, c, dt, sp = W.c5a_inputs()
    assert np.array_equal(ref["coeffs"], c) and float(ref["dt"]) == dt
    t = to_dev(f0, dtype)
    del f0
    s = pkg.Solver(t, dt, c, spacing=sp)
    s.run(int(ref["steps"]))
    got = _sampled(t, ref["idx"])
    err = _rel(got, ref["vals"])
    print(f"c5a {variant}: sampled rel L2 = {err:.3e}")
    assert err < tol


def test_c2_three_steps_full_field_fp32():
    f0, c, dt, sp = W.c2_inputs()
    t = to_dev(f0, torch.float32)
    pkg.Solver(t, dt, c, spacing=sp).run(3)
    got = to_host(t)
    ce, spe = _fp32.effective(c, dt, sp)
    exp = oracle.c_run(_fp32.round_fields(f0), 3, ce, dt, spe)
    err = rel_l2(got, exp)
    print(f"c2 3 steps fp32 full field rel L2 = {err:.3e}")
    assert err < 1e-6


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
def test_c2_eigenmode_1000_steps(dtype, tol):
    shape = W.C2_SHAPE
    f0_, c, dt, sp = W.c2_inputs((4, 4, 4))  # coefficients and dt of the workload
    if dtype == torch.float32:
        ce, spe = _fp32.effective(c, dt, sp)
    else:
        ce, spe = c, sp
    modes = (32, 5, 3)  # wavelength 16 cells along x, oblique
    f0, *_ = O.plane_wave(shape, modes, dt, ce, spe)
    if dtype == torch.float32:
        f0 = _fp32.round_fields(f0)
    t = to_dev(f0, dtype)
    del f0
    pkg.Solver(t, dt, c, spacing=sp).run(1000)
    exp = O.plane_wave_at(shape, modes, dt, ce, 1000, spe)
    got = to_host(t)
    err = rel_l2(got, exp)
    print(f"eigenmode {dtype}: rel L2 = {err:.3e}")
    assert err < tol


def _mode_on_device(shape, params, dt, d, dtype):
    """The eigenmode of the oracle's plane_wave_params at t = 0 (E) and
    t = -dt/2 (B), evaluated on the device in float64 and cast once."""
    w, Eh, Bh, k = params
    nz, ny, nx = shape
    ar = lambda n, o, h: (torch.arange(n, dtype=torch.float64, device=DEV) + o) * h
    out = []
    for c in range(6):
        ox, oy, oz = O.STAGGER[c]
        phase = (k[0] * ar(nx, ox, d[0]))[None, None, :] + (k[1] * ar(ny, oy, d[1]))[None, :, None] \
            + (k[2] * ar(nz, oz, d[2]))[:, None, None]
        amp, shift = (Eh[c], 0.0) if c < 3 else (Bh[c - 3], 0.5 * w * dt)
        out.append((float(amp) * torch.cos(phase + shift)).to(dtype).contiguous())
        del phase
    return out


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
def test_largest_plane_eigenmode(dtype, tol):
    shape = (1, 16384, 16384)
    _, c, dt, sp = W.c2_inputs((4, 4, 4))  # the c2 coefficients and dt
    if dtype == torch.float32:
        ce, spe = _fp32.effective(c, dt, sp)
    else:
        ce, spe = c, sp
    params = O.plane_wave_params(shape, (640, 1000, 0), dt, ce, spe)
    t = _mode_on_device(shape, params, dt, spe, dtype)
    s = pkg.Solver(t, dt, c, spacing=sp)
    assert s.launch_config()["workgroups"] > 0
    n = 20
    s.run(n)
    idx = S.rng(2026).choice(shape[1] * shape[2], size=4096, replace=False)
    got = _sampled(t, idx)
    exp = np.stack([O.plane_wave_sample(shape, params, comp, idx, n, dt, spe) for comp in range(6)], axis=1)
    err = _rel(got, exp)
    print(f"largest plane {dtype}: sampled rel L2 = {err:.3e}")
    assert err < tol
