"""GPU checks of the handle's instrumentation (xfdtd_get_stats): the step and
launch counters follow the launches xfdtd_run makes (one-step, two-step,
in-place, graph replays), the bytes model is 12 values per cell per forward
step and 15 per adjoint step, device timing reports a positive span, and the
gradient passes count their forward, adjoint and recomputed steps."""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle import fdtd as O
import paper_1710_06829_amd as pkg
from tests._gpu import to_dev

pytestmark = pytest.mark.gpu


def _solver(shape, dtype=torch.float32, seed=880):
    beta, delta = S.extended_beta_delta(seed)
    c = O.coeffs_from(beta, delta)
    dt = 0.9 * O.cfl_dt(c)
    return pkg.Solver(to_dev(S.uniform_fields(shape, seed + 1), dtype), dt, c), dt, c


@pytest.mark.parametrize("spp", [1, 2])
def test_run_counters_follow_the_launches(spp):
    shape = (40, 36, 70)  # (nz, ny, nx)
    cells = shape[0] * shape[1] * shape[2]
    s, _, _ = _solver(shape)
    s.set_steps_per_pass(spp)
    s.reset_stats()
    total = 0
    for n in (0, 1, 5, 32, 70, 4):
        s.run(n)
        total += n
    torch.cuda.synchronize()
    st = s.stats()
    print(f"stats spp={spp}: {st}")
    assert st["run_calls"] == 6 and st["steps"] == total
    assert st["in_place_steps"] + st["fused_launches"] + 2 * st["two_step_launches"] == total
    assert st["graph_replays"] == 32 // 32 + 70 // 32
    if spp == 1:
        assert st["two_step_launches"] == 0
    else:
        assert st["two_step_launches"] > 0
    assert st["model_bytes"] == pytest.approx(48.0 * cells * total, rel=1e-12)
    assert st["elapsed_ms"] == -1.0 and st["gcells_per_s"] == -1.0


def test_timing_reports_the_run_span():
    shape = (64, 64, 64)
    cells = shape[0] * shape[1] * shape[2]
    s, _, _ = _solver(shape)
    s.reset_stats(timing=True)
    s.run(40)
    s.run(24)
    st = s.stats()
    assert st["steps"] == 64 and st["elapsed_ms"] > 0
    assert st["gcells_per_s"] == pytest.approx(64 * cells / (st["elapsed_ms"] * 1e-3) / 1e9, rel=1e-9)
    s.reset_stats(timing=False)
    assert s.stats()["steps"] == 0 and s.stats()["elapsed_ms"] == -1.0


def test_gradient_counters():
    """13 steps in segments of 3: 5 segments; the forward pass keeps the E of
    the last two, so the backward recomputes segments 0-2 (2 steps each)."""
    shape = (10, 9, 12)
    cells = shape[0] * shape[1] * shape[2]
    s, _, _ = _solver(shape, torch.float64, seed=890)
    n, seg = 13, 3
    ws = torch.empty(s.grad_workspace_bytes(n, seg), dtype=torch.uint8, device="cuda")
    s.reset_stats()
    s.grad_forward(n, ws, seg)
    lam = to_dev(S.uniform_fields(shape, 893), torch.float64)
    s.grad_backward(n, ws, lam, seg)
    st = s.stats()
    assert st["grad_forward_steps"] == n and st["adjoint_steps"] == n and st["recomputed_steps"] == 6
    assert st["model_bytes"] == pytest.approx(8.0 * cells * (12 * (n + 6) + 15 * n), rel=1e-12)
    # a single adjoint step counts as well
    e = [torch.zeros_like(x) for x in lam[:3]]
    out = [torch.empty_like(x) for x in lam]
    g = torch.zeros(12, dtype=torch.float64, device="cuda")
    s.adjoint_step(lam, out, e, g)
    assert s.stats()["adjoint_steps"] == n + 1
    assert np.isfinite(g.cpu().numpy()).all()


def test_checked_run_stops_at_the_first_non_finite_block():
    """An unstable time step (1.3x the bound, allowed on purpose) blows the
    fields up: the checked run stops after the first block of 25 steps that
    leaves a non-finite value; a stable run completes every step."""
    shape = (24, 20, 36)
    beta, delta = S.extended_beta_delta(895)
    c = O.coeffs_from(beta, delta)
    f = to_dev(S.uniform_fields(shape, 896), torch.float32)
    s = pkg.Solver(f, 1.3 * O.cfl_dt(c), c, allow_unstable=True)
    with pytest.raises(pkg.XfdtdError) as err:
        s.run(4000, check_every=25)
    assert err.value.code == -3  # XFDTD_ENONFINITE
    assert 0 < s.steps_done < 4000 and s.steps_done % 25 == 0
    assert not all(torch.isfinite(x).all() for x in f)
    g = to_dev(S.uniform_fields(shape, 897), torch.float32)
    s2 = pkg.Solver(g, 0.9 * O.cfl_dt(c), c)
    s2.run(120, check_every=50)
    assert s2.steps_done == 120
    assert all(torch.isfinite(x).all() for x in g)
