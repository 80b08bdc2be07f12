"""GPU parity of the batched checkpointed gradient: every box against the
oracle's adjoint, against the single-box schedule, and the 16 x 96^3
coefficient-tuning workload against FP64 finite differences of the oracle."""
import os

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import fdtd as O
import paper_1710_06829_amd as pkg
from tests import workloads as W
from tests._gpu import DEV, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

SHAPES = [(5, 4, 3), (12, 10, 70), (1, 1, 5), (9, 33, 130), (7, 1, 64)]


def _boxes(seed):
    out = []
    for b, shape in enumerate(SHAPES):
        beta, delta = S.distinct_beta_delta(seed + b)
        c = O.coeffs_from(beta, delta)
        sp = (1.0, 1.0 + 0.1 * b, 1.0 - 0.05 * b)
        dt = 0.95 * O.cfl_dt(c, sp)
        out.append((shape, S.uniform_fields(shape, seed + 40 + b), c, dt, sp,
                    S.uniform_fields(shape, seed + 80 + b)))
    return out


@pytest.mark.parametrize("n,seg", [(7, 0), (7, 3), (10, 2), (5, 1), (9, 9), (1, 0), (0, 0), (13, 1), (13, 2)])
@pytest.mark.parametrize("cfg", [(8, 1, 0), (4, 2, 3), (4, 1, 0, 32), (8, 0, 0)])
def test_batch_grad_matches_oracle_fp64(n, seg, cfg):
    boxes = _boxes(900)
    t = [to_dev(f) for (_, f, _, _, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp, _) in enumerate(boxes)], tune=False)
    bt.set_config(*cfg)
    ws = bt.grad_workspaces(n, seg)
    bt.grad_forward(n, ws, seg)
    lams = [to_dev(lamN) for (*_, lamN) in boxes]
    g = bt.grad_backward(n, ws, lams, seg)
    for i, (shape, f0, c, dt, sp, lamN) in enumerate(boxes):
        fN, g0, gc = O.run_with_adjoint(f0, n, c, dt, sp, lambda f, l=lamN: l)
        assert rel_l2(to_host(t[i]), fN) < 1e-13, (i, shape)
        assert rel_l2(to_host(lams[i]), g0) < 1e-12, (i, shape)
        if n:
            assert np.abs(np.asarray(g[i]) - gc).max() <= 1e-11 * np.abs(gc).max(), (i, shape)
        else:
            assert np.all(np.asarray(g[i]) == 0)


@pytest.mark.parametrize("shapes", [[(32, 40, 96), (24, 24, 64), (48, 17, 70)],
                                    # 16 boxes of 96^3: the model picks the 32x12 adjoint tile
                                    [(96, 96, 96)] * 16])
def test_batch_grad_equals_single_box_fp32(shapes):
    """Final states and adjoint fields bitwise equal to the single-box
    schedule whatever the batched tilings (the per-cell arithmetic is the
    same); coefficient gradients equal up to the order of the FP64
    workgroup sums."""
    n = 23
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.extended_beta_delta(910 + b)
        c = O.coeffs_from(beta, delta)
        boxes.append((shape, S.uniform_fields(shape, 920 + b), c, 0.95 * O.cfl_dt(c),
                      S.uniform_fields(shape, 930 + b)))
    tb = [to_dev(f, torch.float32) for (_, f, _, _, _) in boxes]
    bt = pkg.Batch([(tb[i], dt, c) for i, (_, _, c, dt, _) in enumerate(boxes)], tune=False)
    bt.set_config(8, 1, 0)
    ws = bt.grad_workspaces(n)
    bt.grad_forward(n, ws)
    lb = [to_dev(l, torch.float32) for (*_, l) in boxes]
    gb = bt.grad_backward(n, ws, lb)
    acfg = bt.adjoint_config()
    print(f"batched adjoint configuration: {acfg}")
    if len(shapes) > 3:
        assert acfg["tile_x"] == 32 and acfg["tile_y"] == 12, acfg
    for i, (shape, f0, c, dt, lamN) in enumerate(boxes):
        ts = to_dev(f0, torch.float32)
        s = pkg.Solver(ts, dt, c, scratch=False)
        w1 = torch.empty(s.grad_workspace_bytes(n), dtype=torch.uint8, device=DEV)
        s.grad_forward(n, w1)
        ls = to_dev(lamN, torch.float32)
        gs = s.grad_backward(n, w1, ls)
        torch.cuda.synchronize()
        for a, b in zip(tb[i], ts):
            assert torch.equal(a, b), (i, shape)
        for a, b in zip(lb[i], ls):
            assert torch.equal(a, b), (i, shape)
        gs = np.asarray(gs)
        assert np.abs(np.asarray(gb[i]) - gs).max() <= 1e-12 * np.abs(gs).max(), (i, shape)


@pytest.mark.parametrize("dtype,shapes", [
    (torch.float32, [(30, 40, 96), (24, 24, 64), (40, 17, 70), (16, 20, 33)]),
    (torch.float64, [(30, 40, 96), (24, 24, 64), (40, 17, 70), (16, 20, 33)]),
    # degenerate boxes: one-cell planes and columns, a 3-wide box, a ragged 130-wide one
    (torch.float32, [(5, 4, 3), (1, 1, 5), (7, 1, 64), (9, 33, 130)]),
    (torch.float64, [(5, 4, 3), (1, 1, 5), (7, 1, 64), (9, 33, 130)])])
def test_batch_grad_timed_adjoint_tiling_equals_single_boxes(dtype, shapes):
    """xfdtd_batch_tune also times the batched adjoint's tilings; the timed
    choice changes the launch only: states and adjoint fields bitwise equal
    to the single-box schedule, gradients up to the order of the FP64
    workgroup sums."""
    n = 11
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.extended_beta_delta(1810 + b)
        c = O.coeffs_from(beta, delta)
        boxes.append((shape, S.uniform_fields(shape, 1820 + b), c, 0.95 * O.cfl_dt(c),
                      S.uniform_fields(shape, 1830 + b)))
    tb = [to_dev(f, dtype) for (_, f, _, _, _) in boxes]
    bt = pkg.Batch([(tb[i], dt, c) for i, (_, _, c, dt, _) in enumerate(boxes)], tune=True)
    acfg = bt.adjoint_config()
    print(f"forward {bt.config()}, timed adjoint tiling {acfg}")
    assert acfg["tile_y"] in (4, 8, 12) and 1 <= acfg["zsplit"] <= 1024 and acfg["slots"] > 0
    ws = bt.grad_workspaces(n)
    bt.grad_forward(n, ws)
    lb = [to_dev(l, dtype) for (*_, l) in boxes]
    gb = bt.grad_backward(n, ws, lb)
    assert bt.adjoint_config() == acfg
    for i, (shape, f0, c, dt, lamN) in enumerate(boxes):
        ts = to_dev(f0, dtype)
        s = pkg.Solver(ts, dt, c, scratch=False)
        w1 = torch.empty(s.grad_workspace_bytes(n), dtype=torch.uint8, device=DEV)
        s.grad_forward(n, w1)
        ls = to_dev(lamN, dtype)
        gs = np.asarray(s.grad_backward(n, w1, ls))
        torch.cuda.synchronize()
        for a, b in zip(tb[i], ts):
            assert torch.equal(a, b), (i, shape)
        for a, b in zip(lb[i], ls):
            assert torch.equal(a, b), (i, shape)
        assert np.abs(np.asarray(gb[i]) - gs).max() <= 1e-12 * np.abs(gs).max(), (i, shape)


def test_batch_grad_rejects_bad_workspaces():
    boxes = _boxes(950)[:2]
    t = [to_dev(f) for (_, f, _, _, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp, _) in enumerate(boxes)], tune=False)
    ws = bt.grad_workspaces(5)
    small = [ws[0], ws[1][:128]]
    with pytest.raises(RuntimeError):
        bt.grad_forward(5, small)
    with pytest.raises(RuntimeError):
        bt.grad_forward(5, [ws[0], ws[1][1:]])  # misaligned


def test_config5_16_boxes_96cube_300_steps_vs_finite_differences():
    """16 coefficient sets on 96^3 FP32 boxes, 300 steps, forward and adjoint
    batched: each box's gradient along two seeded directions in coefficient
    space, and all 12 coefficients of four boxes, within 1e-4 of FP64 central
    differences of the oracle (stored by tests/golden/make_c5_fd.py)."""
    path = os.path.join(GOLD, "c5_fd.npz")
    if not os.path.exists(path):
        pytest.skip("c5_fd.npz not generated")
    ref = np.load(path)
    n = int(ref["steps"])
    boxes = W.c5_boxes(steps=n)
    t = [to_dev(f, torch.float32) for (f, *_) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, c, dt, sp, _, _) in enumerate(boxes)], tune=True)
    ws = bt.grad_workspaces(n)
    bt.grad_forward(n, ws)
    lams = []
    for i, (f0, c, dt, sp, xp, tgt) in enumerate(boxes):
        assert np.array_equal(ref["coeffs"][i], c) and ref["dt"][i] == dt
        lam = [torch.zeros_like(x) for x in t[i]]
        for a in range(3):
            lam[a][:, :, xp] = t[i][a][:, :, xp] - torch.from_numpy(tgt[a]).to(DEV, torch.float32)
        lams.append(lam)
    g = bt.grad_backward(n, ws, lams)
    # Directional derivatives along two seeded unit directions per box.  A
    # projection can cancel far below the size of the gradient, so the bar is
    # 1e-4 relative to max(|fd|, 1e-3 |g|_2) (the per-entry floor of the
    # gradient checks, applied to the projection's natural scale |g|_2).
    worst = 0.0
    for key_v, key_d in (("dirs", "dir_deriv"), ("dirs2", "dir_deriv2")):
        if key_d not in ref:
            continue
        for i in range(len(boxes)):
            gi = np.asarray(g[i])
            got = float(np.dot(gi, ref[key_v][i]))
            fd = float(ref[key_d][i])
            rel = abs(got - fd) / max(abs(fd), 1e-3 * np.linalg.norm(gi))
            worst = max(worst, rel)
            assert rel < 1e-4, (key_d, i, got, fd, rel)
    # every coefficient of four boxes, per entry against
    # max(|fd|, 1e-3 max |fd|) of that box
    if "full_grad" in ref:
        for row, i in enumerate(ref["full_boxes"]):
            fd = ref["full_grad"][row]
            rel = np.abs(np.asarray(g[int(i)]) - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
            worst = max(worst, float(rel.max()))
            assert rel.max() < 1e-4, (int(i), rel, np.asarray(g[int(i)]), fd)
    print(f"c5 batched gradients: worst relative error {worst:.2e}")


def test_batch_grad_rejects_aliased_lambda():
    """Two boxes handed the same adjoint arrays: an argument error found before
    device work; distinct arrays then go through."""
    shape = (6, 5, 7)
    boxes = []
    for b in range(2):
        beta, delta = S.distinct_beta_delta(961 + b)
        c = O.coeffs_from(beta, delta)
        boxes.append((to_dev(S.uniform_fields(shape, 963 + b)), 0.9 * O.cfl_dt(c), c))
    bt = pkg.Batch(boxes, tune=False)
    n = 3
    ws = bt.grad_workspaces(n)
    bt.grad_forward(n, ws)
    lam = to_dev(S.uniform_fields(shape, 965))
    with pytest.raises(pkg.XfdtdError):
        bt.grad_backward(n, ws, [lam, lam])
    bt.grad_backward(n, ws, [lam, [t.clone() for t in lam]])


def test_batch_grad_backward_consumes_the_forward():
    """As for one box: the backward pass needs a forward pass of the same n
    and seg into the same workspaces before it."""
    shape = (6, 5, 7)
    boxes = []
    for b in range(2):
        beta, delta = S.distinct_beta_delta(971 + b)
        c = O.coeffs_from(beta, delta)
        boxes.append((to_dev(S.uniform_fields(shape, 973 + b)), 0.9 * O.cfl_dt(c), c))
    f0 = [[t.clone() for t in f] for (f, _, _) in boxes]
    bt = pkg.Batch(boxes, tune=False)
    n, seg = 9, 2
    ws = bt.grad_workspaces(n, seg)
    lamN = [to_dev(S.uniform_fields(shape, 975 + b)) for b in range(2)]
    fresh = lambda: [[t.clone() for t in l] for l in lamN]
    with pytest.raises(pkg.XfdtdError):
        bt.grad_backward(n, ws, fresh(), seg)
    bt.grad_forward(n, ws, seg)
    with pytest.raises(pkg.XfdtdError):
        bt.grad_backward(n, ws[::-1], fresh(), seg)  # workspaces of other boxes
    with pytest.raises(pkg.XfdtdError):
        bt.grad_backward(n - 1, ws, fresh(), seg)
    l1 = fresh()
    g1 = bt.grad_backward(n, ws, l1, seg)
    with pytest.raises(pkg.XfdtdError):
        bt.grad_backward(n, ws, fresh(), seg)
    for b, (f, _, _) in enumerate(boxes):
        for a in range(6):
            f[a].copy_(f0[b][a])
    bt.grad_forward(n, ws, seg)
    l2 = fresh()
    g2 = bt.grad_backward(n, ws, l2, seg)
    assert [list(g) for g in g1] == [list(g) for g in g2]
    for b in range(2):
        for a in range(6):
            assert torch.equal(l1[b][a], l2[b][a]), (b, a)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_grad_of_plane_boxes(dtype):
    """A batch of boxes one plane deep (forward and recompute on the plane
    kernel; adjoint work items of several tiles once the batch has at least
    two per workgroup of every CU: on 256 CUs with 64-wide tiles, 2 in FP32
    and 4 in FP64, the 17x64 box then in groups of 2 and 1, or 4 and 1):
    FP64 against the oracle's adjoint; FP32 bitwise
    (states, adjoint fields) against single-box gradient runs, coefficient
    gradients up to the order of the FP64 sums."""
    shapes = [(1, 45, 150), (1, 17, 64), (1, 1, 5), (1, 520, 1000)]
    n, seg = 9, 3
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.distinct_beta_delta(1870 + b)
        c = O.coeffs_from(beta, delta)
        sp = (1.0, 1.0 + 0.1 * b, 1.0)
        boxes.append((shape, S.uniform_fields(shape, 1880 + b), c, 0.95 * O.cfl_dt(c, sp), sp,
                      S.uniform_fields(shape, 1890 + b)))
    t = [to_dev(f, dtype) for (_, f, _, _, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp, _) in enumerate(boxes)], tune=False)
    assert bt.config()["tile_x"] == 64
    ws = bt.grad_workspaces(n, seg)
    bt.grad_forward(n, ws, seg)
    lams = [to_dev(lamN, dtype) for (*_, lamN) in boxes]
    g = bt.grad_backward(n, ws, lams, seg)
    torch.cuda.synchronize()
    for i, (shape, f0, c, dt, sp, lamN) in enumerate(boxes):
        if dtype == torch.float64:
            fN, g0, gc = O.run_with_adjoint(f0, n, c, dt, sp, lambda f, l=lamN: l)
            assert rel_l2(to_host(t[i]), fN) < 1e-13, (i, shape)
            assert rel_l2(to_host(lams[i]), g0) < 1e-12, (i, shape)
            assert np.abs(np.asarray(g[i]) - gc).max() <= 1e-11 * np.abs(gc).max(), (i, shape)
        else:
            ts = to_dev(f0, dtype)
            s = pkg.Solver(ts, dt, c, spacing=sp, scratch=False)
            w1 = torch.empty(s.grad_workspace_bytes(n, seg), dtype=torch.uint8, device=DEV)
            s.grad_forward(n, w1, seg)
            ls = to_dev(lamN, dtype)
            gs = np.asarray(s.grad_backward(n, w1, ls, seg))
            torch.cuda.synchronize()
            for a, b in zip(t[i], ts):
                assert torch.equal(a, b), (i, shape)
            for a, b in zip(lams[i], ls):
                assert torch.equal(a, b), (i, shape)
            assert np.abs(np.asarray(g[i]) - gs).max() <= 1e-12 * np.abs(gs).max(), (i, shape)


@pytest.mark.parametrize("plane", [(1, 45, 150), (1, 1090, 900)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_one_plane_adjoint_pass_equals_the_z_march(dtype, plane):
    """A single box one plane deep takes the adjoint's one-plane pass (on 256
    CUs the 1090x900 plane has 2055 tiles of 64x8 in FP32, 4 per workgroup
    and 3 in the last, and 4095 of 64x4 in FP64, 7 per workgroup); the same
    box in a batch with a deeper box is marched.  States and adjoint fields bitwise equal, coefficient gradients
    up to the order of the FP64 sums; FP64 also against the oracle's
    adjoint."""
    shapes = [plane, (12, 20, 40)]
    n, seg = 7, 3
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.distinct_beta_delta(1900 + b)
        c = O.coeffs_from(beta, delta)
        sp = (1.0, 0.9, 1.2)
        boxes.append((shape, S.uniform_fields(shape, 1910 + b), c, 0.95 * O.cfl_dt(c, sp), sp,
                      S.uniform_fields(shape, 1920 + b)))
    t = [to_dev(f, dtype) for (_, f, _, _, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp, _) in enumerate(boxes)], tune=False)
    ws = bt.grad_workspaces(n, seg)
    bt.grad_forward(n, ws, seg)
    lams = [to_dev(lamN, dtype) for (*_, lamN) in boxes]
    gb = bt.grad_backward(n, ws, lams, seg)
    shape, f0, c, dt, sp, lamN = boxes[0]
    ts = to_dev(f0, dtype)
    s = pkg.Solver(ts, dt, c, spacing=sp, scratch=False)
    w1 = torch.empty(s.grad_workspace_bytes(n, seg), dtype=torch.uint8, device=DEV)
    s.grad_forward(n, w1, seg)
    ls = to_dev(lamN, dtype)
    gs = np.asarray(s.grad_backward(n, w1, ls, seg))
    torch.cuda.synchronize()
    for a, b in zip(t[0], ts):
        assert torch.equal(a, b)
    for a, b in zip(lams[0], ls):
        assert torch.equal(a, b)
    assert np.abs(np.asarray(gb[0]) - gs).max() <= 1e-12 * np.abs(gs).max()
    if dtype == torch.float64:
        fN, g0, gc = O.run_with_adjoint(f0, n, c, dt, sp, lambda f, l=lamN: l)
        assert rel_l2(to_host(ls), g0) < 1e-12
        assert np.abs(gs - gc).max() <= 1e-11 * np.abs(gc).max()
