"""GPU parity of the batched, graph-captured multi-box step: against the
oracle per box, against sequential single-box runs, across launch
configurations, and the 64-box workload after 500 steps."""
import os

import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from oracle import fdtd as O
import paper_1710_06829_amd as pkg
from tests import workloads as W
from tests._gpu import DEV, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

SMALL = [(5, 4, 3), (20, 18, 70), (1, 1, 5), (9, 33, 130), (7, 1, 64), (33, 17, 31)]


def _small_batch(dtype, seed=700):
    boxes = []
    for b, shape in enumerate(SMALL):
        beta, delta = S.distinct_beta_delta(seed + b)
        c = O.coeffs_from(beta, delta)
        sp = (1.0, 1.0 + 0.1 * b, 1.0 - 0.05 * b)
        dt = 0.95 * O.cfl_dt(c, sp)
        boxes.append((shape, S.uniform_fields(shape, seed + 50 + b), c, dt, sp))
    return boxes


@pytest.mark.parametrize("cfg", [(8, 1, 0), (4, 2, 0), (8, 4, 3), (4, 1, 1), (8, 2, 512), (4, 1, 0, 32),
                                 (8, 2, 3, 32), (8, 0, 0), (4, 0, 5, 32)])
@pytest.mark.parametrize("n", [6, 5])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_oracle_fp64(cfg, n, graph):
    boxes = _small_batch(torch.float64)
    t = [to_dev(f) for (_, f, _, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp) in enumerate(boxes)], tune=False)
    bt.set_config(*cfg)
    bt.run(n, graph=graph)
    for i, (shape, f0, c, dt, sp) in enumerate(boxes):
        exp = oracle.c_run(f0, n, c, dt, sp)
        assert rel_l2(to_host(t[i]), exp) < 1e-13, (i, shape)


def test_batch_graph_replays_and_tuner_keeps_state_fp32():
    boxes = _small_batch(torch.float32, seed=720)
    t = [to_dev(f, torch.float32) for (_, f, _, _, _) in boxes]
    ref = [to_dev(f, torch.float32) for (_, f, _, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp) in enumerate(boxes)], tune=True)
    cfg = bt.config()
    assert cfg["tile_x"] in (32, 64) and cfg["tile_y"] in (4, 8, 16) and cfg["items"] > 0
    for i in range(len(boxes)):  # tuning leaves the state untouched
        assert all(torch.equal(a, b) for a, b in zip(t[i], ref[i]))
    # the same graph replayed three times with host synchronisations in between
    for _ in range(3):
        bt.run(4)
        torch.cuda.synchronize()
    for i, (shape, f0, c, dt, sp) in enumerate(boxes):
        s = pkg.Solver(ref[i], dt, c, spacing=sp)
        for _ in range(3):
            s.run(4)
        torch.cuda.synchronize()
        # identical arithmetic per cell whatever the tiling: bitwise equal
        for a, b in zip(t[i], ref[i]):
            assert torch.equal(a, b), (i, shape)


@pytest.mark.parametrize("cfg", [(8, 1, 0), (16, 2, 0), (8, 4, 3), (16, 1, 256), (16, 0, 0), (8, 0, 7)])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_two_steps_per_launch_equals_single_runs_fp32(cfg, graph):
    """Two steps per launch (FP32, 32-column tiles): every tile height,
    z-split and grid, and step counts that take each path that keeps the
    result in the state arrays (odd n, odd and even numbers of pairs), give
    bitwise the results of single-box runs."""
    boxes = _small_batch(torch.float32, seed=740)
    for n in (3, 4, 6, 9):
        t = [to_dev(f, torch.float32) for (_, f, _, _, _) in boxes]
        bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp) in enumerate(boxes)], tune=False)
        bt.set_config(cfg[0], cfg[1], cfg[2], tile_x=32)
        bt.set_steps_per_pass(2)
        assert bt.config()["steps_per_pass"] == 2
        bt.run(n, graph=graph)
        for i, (shape, f0, c, dt, sp) in enumerate(boxes):
            ref = to_dev(f0, torch.float32)
            pkg.Solver(ref, dt, c, spacing=sp).run(n)
            torch.cuda.synchronize()
            for a, b in zip(t[i], ref):
                assert torch.equal(a, b), (n, i, shape)
    with pytest.raises(pkg.XfdtdError):  # 64-column tilings have no two-step kernel
        bt.set_config(8, 1, 0, tile_x=64)
        bt.set_steps_per_pass(2)


def test_config3_64_boxes_500_steps():
    path = os.path.join(GOLD, "c3_boxes_fp32.npz")
    boxes = W.c3_boxes()
    t = [to_dev(f, torch.float32) for (_, f, _, _) in boxes]
    seq = [to_dev(f, torch.float32) for (_, f, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c) for i, (_, _, c, dt) in enumerate(boxes)], tune=True)
    bt.run(500)
    print(f"c3 batch configuration: {bt.config()}")
    for i, (shape, f0, c, dt) in enumerate(boxes):
        pkg.Solver(seq[i], dt, c).run(500)
    torch.cuda.synchronize()
    for i in range(len(boxes)):
        for a, b in zip(t[i], seq[i]):
            assert torch.equal(a, b), i
    if not os.path.exists(path):
        pytest.skip("c3_boxes_fp32.npz not generated (batched == sequential checked)")
    ref = np.load(path)
    worst = 0.0
    for i in range(len(boxes)):
        ii = torch.from_numpy(ref["idx"][i]).to(DEV)
        got = np.stack([x.reshape(-1)[ii].double().cpu().numpy() for x in t[i]], axis=1)
        e = float(np.linalg.norm(got - ref["vals"][i]) / np.linalg.norm(ref["vals"][i]))
        worst = max(worst, e)
    print(f"c3 worst sampled rel L2 over 64 boxes: {worst:.3e}")
    assert worst < 1e-5


def test_batch_with_largest_plane_box_equals_single_runs_fp32():
    """A batch holding a box on the largest accepted plane (16384 x 16384
    cells) next to a tiny box gives bitwise the results of single-box runs
    (every tiling evaluates the same arithmetic per cell)."""
    shapes = [(1, 16384, 16384), (5, 4, 3)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(731)
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.distinct_beta_delta(732 + b)
        c = O.coeffs_from(beta, delta)
        dt = 0.95 * O.cfl_dt(c)
        f = [torch.rand(shape, device="cuda", generator=gen) * 2 - 1 for _ in range(6)]
        boxes.append((f, dt, c))
    single = []
    for f, dt, c in boxes:
        t = [u.clone() for u in f]
        pkg.Solver(t, dt, c).run(4)
        single.append(t)
    bt = pkg.Batch([(f, dt, c) for f, dt, c in boxes], tune=False)
    bt.run(4)
    torch.cuda.synchronize()
    for (f, _, _), t in zip(boxes, single):
        assert all(torch.equal(a, b) for a, b in zip(f, t))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("tune", [False, True])
def test_batch_of_plane_boxes_equals_single_runs(dtype, tune):
    """Every box one plane deep (the 2D variant): the batch runs the plane
    kernel (tiles of 64 columns, no z-march), bitwise equal to single-box
    runs of the same boxes, and in FP64 equal to the oracle; 7 steps (an odd
    count: one in-place step) and 12."""
    shapes = [(1, 45, 150), (1, 17, 64), (1, 1, 5), (1, 33, 33)]
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.extended_beta_delta(1850 + b)
        c = O.coeffs_from(beta, delta)
        sp = (1.0, 0.9 + 0.1 * b, 1.0)
        boxes.append((shape, S.uniform_fields(shape, 1860 + b), c, 0.95 * O.cfl_dt(c, sp), sp))
    t = [to_dev(f, dtype) for (_, f, _, _, _) in boxes]
    bt = pkg.Batch([(t[i], dt, c, sp) for i, (_, _, c, dt, sp) in enumerate(boxes)], tune=tune)
    cfg = bt.config()
    assert cfg["tile_x"] == 64 and cfg["steps_per_pass"] == 1, cfg
    for n in (7, 12):
        bt.run(n)
        torch.cuda.synchronize()
    for i, (shape, f0, c, dt, sp) in enumerate(boxes):
        ref = to_dev(f0, dtype)
        s = pkg.Solver(ref, dt, c, spacing=sp)
        s.run(7)
        s.run(12)
        torch.cuda.synchronize()
        for a, b in zip(t[i], ref):
            assert torch.equal(a, b), (i, shape)
        if dtype == torch.float64:
            assert rel_l2(to_host(t[i]), oracle.c_run(f0, 19, c, dt, sp)) < 1e-13, (i, shape)
