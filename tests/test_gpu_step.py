"""GPU parity of the time step (Faraday, Ampere, fused z-march) against the
FP64 oracle, on sizes that span several tiles with ragged tails, degenerate
axes, both tile heights and several z-chunk depths."""
import os

import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from oracle import fdtd as O
import paper_1710_06829_amd as pkg
from tests import _fp32
from tests._gpu import max_rel, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


def _coeffs(seed):
    beta, delta = S.distinct_beta_delta(seed)
    return O.coeffs_from(beta, delta)


@pytest.fixture
def env(monkeypatch):
    def set_(**kw):
        for k, v in kw.items():
            monkeypatch.setenv(k, str(v))
    return set_


SHAPES = [(20, 18, 70), (7, 9, 130), (33, 17, 64), (5, 4, 3), (1, 1, 5), (1, 3, 1), (2, 1, 1),
          (9, 1, 66), (3, 26, 1)]


@pytest.mark.parametrize("shape", SHAPES)
def test_faraday_and_ampere_unfused_fp64(shape):
    c = _coeffs(401)
    sp = (1.0, 0.8, 1.2)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 402)
    t = to_dev(f0)
    s = pkg.Solver(t, dt, c, spacing=sp, scratch=False)
    s.step_faraday()
    got = to_host(t)
    Bn = O.faraday(f0[:3], f0[3:], c, dt, sp)
    assert max_rel(got[3:], Bn) < 1e-13
    assert max_rel(got[:3], f0[:3]) == 0.0
    s.step_ampere()
    got = to_host(t)
    En = O.ampere(f0[:3], Bn, dt, sp)
    assert max_rel(got[:3], En) < 1e-13


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("n", [1, 2, 5])
def test_run_fused_fp64(shape, n):
    c = _coeffs(411)
    sp = (1.0, 1.1, 0.9)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 412)
    t = to_dev(f0)
    pkg.Solver(t, dt, c, spacing=sp).run(n)
    got = to_host(t)
    exp = oracle.c_run(f0, n, c, dt, sp)
    assert rel_l2(got, exp) < 1e-13


@pytest.mark.parametrize("tile_x", [64, 32])
@pytest.mark.parametrize("tile_y", [4, 8])
@pytest.mark.parametrize("zchunk", [1, 3, 8, 64])
def test_fused_launch_shapes_fp64(env, tile_x, tile_y, zchunk):
    env(XFDTD_TILE_X=tile_x, XFDTD_TILE_Y=tile_y, XFDTD_ZCHUNK=zchunk)
    shape = (19, 21, 131)
    c = _coeffs(421)
    dt = 0.95 * O.cfl_dt(c)
    f0 = S.uniform_fields(shape, 422)
    t = to_dev(f0)
    pkg.Solver(t, dt, c).run(4)
    exp = oracle.c_run(f0, 4, c, dt)
    assert rel_l2(to_host(t), exp) < 1e-13


def test_fused_matches_unfused_fp64():
    shape = (24, 20, 100)
    c = _coeffs(431)
    dt = 0.95 * O.cfl_dt(c)
    f0 = S.uniform_fields(shape, 432)
    a, b = to_dev(f0), to_dev(f0)
    pkg.Solver(a, dt, c, scratch=True).run(10)
    pkg.Solver(b, dt, c, scratch=False).run(10)
    assert rel_l2(to_host(a), to_host(b)) < 1e-13


def test_run_zero_steps_is_identity():
    f0 = S.uniform_fields((6, 7, 8), 441)
    t = to_dev(f0)
    pkg.Solver(t, 0.3, O.yee_coeffs()).run(0)
    assert max_rel(to_host(t), f0) == 0.0


@pytest.mark.parametrize("shape", [(20, 18, 70), (5, 9, 200), (1, 1, 7)])
@pytest.mark.parametrize("scratch", [True, False])
def test_fp32_against_fp64_oracle(shape, scratch):
    c = _coeffs(451)
    sp = (1.0, 0.9, 1.1)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 452)
    t = to_dev(f0, torch.float32)
    pkg.Solver(t, dt, c, spacing=sp, scratch=scratch).run(20)
    ce, spe = _fp32.effective(c, dt, sp)
    exp = oracle.c_run(_fp32.round_fields(f0), 20, ce, dt, spe)
    assert rel_l2(to_host(t), exp) < 2e-6


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_plane_kernel_equals_z_march_and_oracle(dtype):
    """A box one plane deep (nz = 1) runs the plane kernel: several tiles with
    ragged tails in x and y, bitwise equal to the z-marching kernels (the
    two-step kernel and a one-box batch, which march the periodic plane) and
    to the oracle within its bar."""
    shape = (1, 45, 150)
    c = _coeffs(455)
    sp = (1.0, 0.8, 1.3)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 456)
    n = 7
    a = to_dev(f0, dtype)
    sa = pkg.Solver(a, dt, c, spacing=sp)
    assert sa.launch_config()["steps_per_pass"] == 1
    sa.run(n)
    b = to_dev(f0, dtype)
    sb = pkg.Solver(b, dt, c, spacing=sp)
    sb.set_steps_per_pass(2)
    sb.run(n - 1)
    assert sb.stats()["two_step_launches"] > 0
    sb.set_steps_per_pass(1)
    sb.run(1)
    bt_f = to_dev(f0, dtype)
    bt = pkg.Batch([(bt_f, dt, c, sp)], tune=False)
    bt.run(n)
    torch.cuda.synchronize()
    for x, y, z in zip(a, b, bt_f):
        assert torch.equal(x, y) and torch.equal(x, z)
    if dtype == torch.float64:
        assert rel_l2(to_host(a), oracle.c_run(f0, n, c, dt, sp)) < 1e-13
    else:
        ce, spe = _fp32.effective(c, dt, sp)
        assert rel_l2(to_host(a), oracle.c_run(_fp32.round_fields(f0), n, ce, dt, spe)) < 2e-6


@pytest.mark.parametrize("kind", ["yee", "extended"])
def test_config1_plane_wave(kind):
    """32^3 FP64, 100 steps: equal to the oracle and to the exact eigenmode."""
    shape = (32, 32, 32)
    if kind == "yee":
        c = O.yee_coeffs()
    else:
        beta, delta = S.extended_beta_delta(101)
        c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c)
    modes = S.mode_numbers(102)
    f0, *_ = O.plane_wave(shape, modes, dt, c)
    t = to_dev(f0)
    pkg.Solver(t, dt, c).run(100)
    got = to_host(t)
    assert rel_l2(got, oracle.c_run(f0, 100, c, dt)) < 1e-12
    assert rel_l2(got, O.plane_wave_at(shape, modes, dt, c, 100)) < 1e-12


@pytest.mark.parametrize("kind", ["yee", "extended"])
def test_config1_random_projected(kind):
    shape = (32, 32, 32)
    if kind == "yee":
        c = O.yee_coeffs()
    else:
        beta, delta = S.extended_beta_delta(101)
        c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c)
    f = S.uniform_fields(shape, 103)
    f0 = f[:3] + O.project_div_star_free(f[3:], c)
    t = to_dev(f0)
    s = pkg.Solver(t, dt, c)
    db0, de0 = s.divergence()
    s.run(100)
    got = to_host(t)
    assert rel_l2(got, oracle.c_run(f0, 100, c, dt)) < 1e-12
    mb, me, bad = s.divergence_max(db0, de0)
    assert bad == 0
    assert mb < 1e-12 and me < 1e-12
    mb0, _, _ = s.divergence_max(None, None)
    assert mb0 < 1e-12  # D*.B stays at rounding level (it starts at ~0)


def test_divergence_fields_match_oracle():
    shape = (9, 10, 70)
    c = _coeffs(461)
    sp = (1.0, 0.7, 1.4)
    f0 = S.uniform_fields(shape, 462)
    t = to_dev(f0)
    s = pkg.Solver(t, 0.1, c, spacing=sp)
    db, de = s.divergence()
    db, de = to_host([db, de])
    assert np.abs(db - O.div_star_B(f0[3:], c, sp)).max() < 1e-12
    assert np.abs(de - O.div_E(f0[:3], sp)).max() < 1e-12


@pytest.mark.parametrize("shape", [(70000, 1, 2), (1, 270000, 1)])
def test_long_boxes_beyond_65535_grid_blocks_fp64(shape):
    """Boxes whose z extent, or y extent in 4-row blocks, exceeds 65535: the
    unfused updates (step_faraday / step_ampere, the odd first step of run)
    and the divergence loop over their capped grids; the fused step has a
    one-dimensional grid."""
    c = _coeffs(481)
    dt = 0.9 * O.cfl_dt(c)
    f0 = S.uniform_fields(shape, 482)
    t = to_dev(f0)
    s = pkg.Solver(t, dt, c)
    s.step_faraday()
    s.step_ampere()
    s.run(3)  # one unfused step, then a fused pair
    assert rel_l2(to_host(t), oracle.c_run(f0, 4, c, dt)) < 1e-13
    f1 = to_host(t)
    db, de = to_host(list(s.divergence()))
    sp = (1.0, 1.0, 1.0)
    assert np.abs(db - O.div_star_B(f1[3:], c, sp)).max() < 1e-12
    assert np.abs(de - O.div_E(f1[:3], sp)).max() < 1e-12


def test_divergence_max_reports_nonfinite():
    f0 = S.uniform_fields((4, 5, 6), 471)
    f0[2][1, 2, 3] = np.nan
    t = to_dev(f0)
    s = pkg.Solver(t, 0.3, O.yee_coeffs())
    _, _, bad = s.divergence_max(raise_nonfinite=False)
    assert bad == 1
    with pytest.raises(pkg.XfdtdError):
        s.divergence_max()


def test_dispersion_matches_oracle():
    c = _coeffs(481)
    sp = (1.0, 0.6, 1.3)
    dt = 0.95 * O.cfl_dt(c, sp)
    k = S.rng(482).uniform(0.0, 1.0, (5000, 3)) * np.pi / np.asarray(sp)
    k[0] = 0.0
    w, vph, vg = pkg.dispersion(torch.from_numpy(k).cuda(), dt, c, sp)
    ow, ovph, ovg = O.dispersion(k, dt, c, sp)
    w, vph, vg = to_host([w, vph, vg])
    assert np.abs(w - ow).max() < 1e-13
    assert np.allclose(vph[1:], ovph[1:], rtol=1e-13, atol=0)
    assert np.abs(vg[1:] - ovg[1:]).max() < 1e-11


def test_dispersion_flags_unstable_wave_vectors():
    c = O.yee_coeffs()
    dt = 1.2 * O.cfl_dt(c)
    k = torch.tensor([[0.1, 0.0, 0.0], [np.pi, np.pi, np.pi]], dtype=torch.float64).cuda()
    with pytest.raises(pkg.XfdtdError):
        pkg.dispersion(k, dt, c)
    w, _, _ = pkg.dispersion(k, dt, c, allow_unstable=True)
    w = w.cpu().numpy()
    assert np.isfinite(w[0]) and np.isnan(w[1])


@pytest.mark.parametrize("shape", [(37, 45, 150), (16, 33, 64), (3, 17, 5)])
def test_fp32_tilings_agree_bitwise_and_match_oracle(env, shape):
    """Every FP32 tiling (64 and 32 columns; 4, 8 and 16 rows, the 16-row one
    with two rows per lane) and z-chunking evaluates the same arithmetic per
    cell: results are bitwise equal and match the oracle under the FP32
    convention."""
    c = _coeffs(491)
    sp = (1.0, 0.9, 1.1)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 492)
    outs = []
    for tx in (64, 32):
        for ty in (4, 8, 16):
            for zc in (2, 7, 64):
                env(XFDTD_TILE_X=tx, XFDTD_TILE_Y=ty, XFDTD_ZCHUNK=zc, XFDTD_STEPS_PER_PASS=1)
                t = to_dev(f0, torch.float32)
                s = pkg.Solver(t, dt, c, spacing=sp)
                assert s.launch_config()["tile_x"] == tx
                s.run(6)
                outs.append(to_host(t))
    for o in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(o, outs[0]))
    ce, spe = _fp32.effective(c, dt, sp)
    exp = oracle.c_run(_fp32.round_fields(f0), 6, ce, dt, spe)
    assert rel_l2(outs[0], exp) < 1e-6


TWO_STEP_SHAPES = [(37, 45, 150), (16, 33, 64), (3, 17, 5), (1, 1, 5), (2, 40, 33), (9, 1, 70), (1, 8, 1),
                   (5, 16, 32), (64, 7, 2)]


@pytest.mark.parametrize("shape", TWO_STEP_SHAPES)
def test_two_step_kernel_bitwise_equals_one_step(env, shape):
    """Two steps per launch (FP32): every tile height and z-chunking, and run
    lengths that take each of the paths that keep the result in the bound
    fields (odd and even counts of two-step launches, odd n), give bitwise
    the result of one fused step per launch; that result matches the oracle
    under the FP32 convention."""
    c = _coeffs(481)
    sp = (1.0, 0.9, 1.1)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 482)
    for n in (1, 2, 3, 4, 7, 8):
        env(XFDTD_STEPS_PER_PASS=1)
        ref = to_dev(f0, torch.float32)
        s1 = pkg.Solver(ref, dt, c, spacing=sp)
        assert s1.launch_config()["steps_per_pass"] == 1
        s1.run(n)
        ref = to_host(ref)
        env(XFDTD_STEPS_PER_PASS=2)
        for ty in (8, 16):
            for zc in (1, 3, 7, 64) if n in (4, 7) else (64,):
                env(XFDTD_BLK_TILE_Y=ty, XFDTD_BLK_ZCHUNK=zc)
                t = to_dev(f0, torch.float32)
                s = pkg.Solver(t, dt, c, spacing=sp)
                lc = s.launch_config()
                assert lc["steps_per_pass"] == 2 and lc["two_step"]["tile_y"] == ty
                assert lc["two_step"]["zchunk"] == zc
                s.run(n)
                got = to_host(t)
                assert all(np.array_equal(a, b) for a, b in zip(got, ref)), (n, ty, zc)
        if n == 8:
            ce, spe = _fp32.effective(c, dt, sp)
            exp = oracle.c_run(_fp32.round_fields(f0), n, ce, dt, spe)
            assert rel_l2(got, exp) < 1e-6


@pytest.mark.parametrize("shape", TWO_STEP_SHAPES)
def test_two_step_kernel_fp64_equals_one_step_and_oracle(env, shape):
    """FP64 two steps per launch (24 x 8 tiles): bitwise the one-step
    launches for run lengths that take each path and several z-chunkings,
    and within 1e-13 of the FP64 oracle."""
    c = _coeffs(487)
    sp = (1.0, 0.9, 1.1)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 488)
    for n in (1, 2, 3, 4, 7, 8):
        env(XFDTD_STEPS_PER_PASS=1)
        ref = to_dev(f0)
        pkg.Solver(ref, dt, c, spacing=sp).run(n)
        ref = to_host(ref)
        env(XFDTD_STEPS_PER_PASS=2)
        for zc in (1, 3, 7, 64) if n in (4, 7) else (64,):
            env(XFDTD_BLK_ZCHUNK=zc)
            t = to_dev(f0)
            s = pkg.Solver(t, dt, c, spacing=sp)
            lc = s.launch_config()
            assert lc["steps_per_pass"] == 2 and lc["two_step"]["tile_x"] == 24 and lc["two_step"]["zchunk"] == zc
            s.run(n)
            got = to_host(t)
            assert all(np.array_equal(a, b) for a, b in zip(got, ref)), (n, zc)
        if n == 8:
            exp = oracle.c_run(f0, n, c, dt, sp)
            assert rel_l2(got, exp) < 1e-13


@pytest.mark.parametrize("dtype,shape,spp", [(torch.float32, (33, 17, 64), 1), (torch.float32, (37, 45, 150), 2),
                                             (torch.float64, (20, 18, 70), 1), (torch.float64, (21, 19, 50), 2)])
def test_run_graph_replay_is_bitwise_the_direct_launches(env, dtype, shape, spp):
    """xfdtd_run replays a captured graph of 32 steps and launches the rest
    directly: bitwise the same as direct launches only, for step counts below,
    at and above one replay, across rebinding to other arrays (which captures
    a new graph) and after retuning."""
    c = _coeffs(471)
    dt = 0.95 * O.cfl_dt(c)
    f0 = S.uniform_fields(shape, 472)
    for n in (5, 32, 70, 131):
        env(XFDTD_GRAPH=0, XFDTD_STEPS_PER_PASS=spp)
        a = to_dev(f0, dtype)
        pkg.Solver(a, dt, c).run(n)
        env(XFDTD_GRAPH=1)
        b = to_dev(f0, dtype)
        sb = pkg.Solver(b, dt, c)
        sb.run(n // 2)
        sb.run(n - n // 2)
        assert all(torch.equal(x, y) for x, y in zip(a, b)), n
        # other arrays on the same handle: the old graph must not be replayed
        b2 = to_dev(f0, dtype)
        sb.fields = b2
        sb.run(n)
        assert all(torch.equal(x, y) for x, y in zip(a, b2)), n


def test_two_step_kernel_rejects_bad_counts():
    shape = (6, 5, 7)
    c = _coeffs(485)
    dt = 0.9 * O.cfl_dt(c)
    s = pkg.Solver(to_dev(S.uniform_fields(shape, 486)), dt, c)
    assert s.launch_config()["steps_per_pass"] == 1
    s.set_steps_per_pass(2)  # FP64: the 24 x 8 two-step tile
    lc = s.launch_config()
    assert lc["steps_per_pass"] == 2 and (lc["two_step"]["tile_x"], lc["two_step"]["tile_y"]) == (24, 8)
    s32 = pkg.Solver(to_dev(S.uniform_fields(shape, 486), torch.float32), dt, c)
    for bad in (0, 3, -1):
        with pytest.raises(pkg.XfdtdError):
            s32.set_steps_per_pass(bad)
    s32.set_steps_per_pass(1)
    assert s32.launch_config()["steps_per_pass"] == 1


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_tuner_keeps_state_and_result(dtype):
    """Tuning reads the state and writes only the scratch arrays and its own
    temporary copy of the state; the tuned tiling gives bitwise the same steps
    as the default one, and a second handle of the same shape takes the
    cached choice."""
    shape = (40, 37, 96)
    c = _coeffs(495)
    dt = 0.95 * O.cfl_dt(c)
    f0 = S.uniform_fields(shape, 496)
    a, b = to_dev(f0, dtype), to_dev(f0, dtype)
    sa = pkg.Solver(a, dt, c)
    cfg = sa.tune(force=True)
    assert sa.tuned_ms > 0
    assert cfg["tile_x"] in (32, 64) and cfg["zchunk"] >= 1 and cfg["workgroups"] > 0
    assert all(np.array_equal(x, y) for x, y in zip(to_host(a), to_host(b)))
    sb = pkg.Solver(b, dt, c)
    assert sb.tune() == cfg and sb.tuned_ms == -1.0
    sa.run(6)
    pkg.Solver(b, dt, c).run(6)
    assert all(np.array_equal(x, y) for x, y in zip(to_host(a), to_host(b)))
    with pytest.raises(ValueError):
        pkg.Solver(b, dt, c, scratch=False).tune()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_box_anisotropic_spacing(dtype):
    """The 2D variant (nz = 1: k_z = 0 only) on a grid with d_y = 10 d_x
    (Sec. 5.3), against the oracle; FP32 under the documented convention."""
    shape = (1, 48, 200)
    sp = (1.0, 10.0, 1.0)
    c = _coeffs(431)
    dt = 0.95 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 432)
    n = 40
    t = to_dev(f0, dtype)
    pkg.Solver(t, dt, c, spacing=sp).run(n)
    got = to_host(t)
    if dtype == torch.float64:
        assert rel_l2(got, oracle.c_run(f0, n, c, dt, sp)) < 1e-13
    else:
        ce, spe = _fp32.effective(c, dt, sp)
        assert rel_l2(got, oracle.c_run(_fp32.round_fields(f0), n, ce, dt, spe)) < 2e-6


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ampere_with_current_matches_oracle(dtype):
    """The current-source hook (App. A eq. update4-6 with mu_0 J): a Faraday
    step then the Ampere step with J, against the oracle; the GPU divergence
    diagnostic sees the discrete continuity D.E^{n+1} - D.E^n = -dt D.J."""
    shape = (9, 20, 70)
    c = _coeffs(441)
    sp = (1.0, 0.9, 1.1)
    dt = 0.9 * O.cfl_dt(c, sp)
    f0 = S.uniform_fields(shape, 442)
    J = S.uniform_fields(shape, 443)[:3]
    t = to_dev(f0, dtype)
    s = pkg.Solver(t, dt, c, spacing=sp, scratch=False)
    _, de0 = s.divergence()
    s.step_faraday()
    s.step_ampere(J=to_dev(J, dtype))
    got = to_host(t)
    if dtype == torch.float64:
        Bn = O.faraday(f0[:3], f0[3:], c, dt, sp)
        exp = O.ampere_current(f0[:3], Bn, J, dt, sp) + Bn
        assert rel_l2(got, exp) < 1e-14
        tol = 1e-11
    else:
        ce, spe = _fp32.effective(c, dt, sp)
        f32 = _fp32.round_fields(f0)
        dt32 = float(np.float32(dt))
        Bn = O.faraday(f32[:3], f32[3:], ce, dt, spe)
        exp = O.ampere_current(f32[:3], Bn, _fp32.round_fields(J), dt32, spe) + Bn
        assert rel_l2(got, exp) < 1e-6
        tol = 1e-4
    _, de1 = s.divergence()
    ddj = O.div_E(J, sp)
    err = (de1 - de0).cpu().double().numpy() + dt * ddj
    assert np.abs(err).max() <= tol * np.abs(dt * ddj).max()
