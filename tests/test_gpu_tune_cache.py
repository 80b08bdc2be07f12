"""GPU checks of the tuning file (XFDTD_TUNE_CACHE): a timed tuning is
appended, a stored line for a grid not tuned in this process is taken
without timing, lines a handle cannot launch and malformed lines are
ignored, and batches do the same with their shape keys."""
import numpy as np
import pytest
import torch

import synthetic as S
from oracle import fdtd as O
import paper_1710_06829_amd as pkg
from tests._gpu import to_dev

pytestmark = pytest.mark.gpu


def _solver(shape, seed, dtype=torch.float32):
    beta, delta = S.extended_beta_delta(seed)
    c = O.coeffs_from(beta, delta)
    return pkg.Solver(to_dev(S.uniform_fields(shape, seed + 1), dtype), 0.9 * O.cfl_dt(c), c)


def test_tuning_file_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("XFDTD_TUNE_CACHE", str(path))
    # shapes (nz, ny, nx) that no other test tunes in this process
    s = _solver((40, 44, 96), 1700)
    lc = s.tune()
    assert s.tuned_ms > 0
    text = path.read_text()
    lines = [ln.split() for ln in text.splitlines()]
    mine = [ln for ln in lines if ln[1] == "single:f32:96x44x40"]
    assert len(mine) == 1, text
    got = [int(x) for x in mine[0][2:]]
    tl = lc["two_step"] if lc["steps_per_pass"] == 2 else lc
    assert got == [lc["steps_per_pass"], tl["tile_x"], tl["tile_y"], tl["zchunk"]]
    dev = mine[0][0]
    # a stored choice is taken as it is (best_ms -1: nothing timed); a
    # malformed line and a line for another device are skipped
    path.write_text(text + "not a tuning line\n" + f"gfx000/1 single:f32:80x52x36 1 64 4 6\n"
                    + f"{dev} single:f32:80x52x36 1 32 8 12\n")
    s2 = _solver((36, 52, 80), 1710)
    lc2 = s2.tune()
    assert s2.tuned_ms == -1.0
    assert (lc2["steps_per_pass"], lc2["tile_x"], lc2["tile_y"], lc2["zchunk"]) == (1, 32, 8, 12)
    # a stored two-step choice with 64-column tiles cannot be launched: timed instead
    path.write_text(text + f"{dev} single:f32:72x20x28 2 64 8 12\n")
    s3 = _solver((28, 20, 72), 1720)
    s3.tune()
    assert s3.tuned_ms > 0
    # FP64: the two-step kernel's 24x8 tiles are taken, its 32x8 FP32 tiles are not
    path.write_text(text + f"{dev} single:f64:60x26x30 2 24 8 10\n" + f"{dev} single:f64:44x22x18 2 32 8 6\n")
    s4 = _solver((30, 26, 60), 1730, torch.float64)
    lc4 = s4.tune()
    assert s4.tuned_ms == -1.0
    assert lc4["steps_per_pass"] == 2 and (lc4["two_step"]["tile_x"], lc4["two_step"]["tile_y"],
                                           lc4["two_step"]["zchunk"]) == (24, 8, 10)
    s5 = _solver((18, 22, 44), 1740, torch.float64)
    s5.tune()
    assert s5.tuned_ms > 0


def test_batch_tuning_file_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("XFDTD_TUNE_CACHE", str(path))
    shapes = [(30, 20, 50), (18, 26, 44)]
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.extended_beta_delta(1730 + b)
        c = O.coeffs_from(beta, delta)
        boxes.append((to_dev(S.uniform_fields(shape, 1740 + b), torch.float32), 0.9 * O.cfl_dt(c), c))
    bt = pkg.Batch(boxes, tune=True)
    cfg = bt.config()
    line = [ln.split() for ln in path.read_text().splitlines() if ln.split()[1] == "batch:f32:50x20x30:44x26x18"]
    assert len(line) == 1
    stored = [int(x) for x in line[0][2:]]
    # the file keeps the configured grid; config() reports the launched one
    # (0 or a grid above the slot count launch one workgroup per slot)
    launched = cfg["items"] if stored[3] == 0 or stored[3] > cfg["items"] else stored[3]
    assert stored[:3] + stored[4:] == [cfg["tile_x"], cfg["tile_y"], cfg["zsplit"], cfg["steps_per_pass"]]
    assert launched == cfg["grid"]
    # the batched adjoint's timed tiling: tile width, height, z-split, whole-box runs
    aline = [ln.split() for ln in path.read_text().splitlines()
             if ln.split()[1] == "batchadj:f32:50x20x30:44x26x18"]
    assert len(aline) == 1
    acfg = bt.adjoint_config()
    astored = [int(x) for x in aline[0][2:]]
    assert astored[:3] == [acfg["tile_x"], acfg["tile_y"], acfg["zsplit"]] and astored[3] in (0, 1)
    dev = line[0][0]
    # another set of shapes, stored: taken without timing, the adjoint's tiling too
    path.write_text(path.read_text() + f"{dev} batch:f32:40x24x16:36x36x20 32 8 2 0 1\n"
                    + f"{dev} batchadj:f32:40x24x16:36x36x20 32 12 3 1\n")
    boxes2 = []
    for b, shape in enumerate([(16, 24, 40), (20, 36, 36)]):
        beta, delta = S.extended_beta_delta(1750 + b)
        c = O.coeffs_from(beta, delta)
        boxes2.append((to_dev(S.uniform_fields(shape, 1760 + b), torch.float32), 0.9 * O.cfl_dt(c), c))
    bt2 = pkg.Batch(boxes2, tune=True)
    c2 = bt2.config()
    assert bt2.tuned_ms == -1.0
    assert (c2["tile_x"], c2["tile_y"], c2["zsplit"], c2["steps_per_pass"]) == (32, 8, 2, 1)
    assert c2["grid"] == c2["items"]  # grid 0: one workgroup per slot
    bt2.run(4)
    ws = bt2.grad_workspaces(5)
    bt2.grad_forward(5, ws)
    bt2.grad_backward(5, ws, [[torch.ones_like(x) for x in f] for (f, _, _) in boxes2])
    a2 = bt2.adjoint_config()
    assert (a2["tile_x"], a2["tile_y"], a2["zsplit"]) == (32, 12, 3)
    torch.cuda.synchronize()


def test_batch_adjoint_line_the_batch_cannot_launch_is_ignored(tmp_path, monkeypatch):
    """A stored adjoint tiling with a tile FP64 lacks (32x12) is not taken:
    the model's tiling runs, and the gradient pass completes."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("XFDTD_TUNE_CACHE", str(path))
    shapes = [(14, 18, 40), (10, 22, 36)]
    boxes = []
    for b, shape in enumerate(shapes):
        beta, delta = S.extended_beta_delta(1770 + b)
        c = O.coeffs_from(beta, delta)
        boxes.append((to_dev(S.uniform_fields(shape, 1780 + b), torch.float64), 0.9 * O.cfl_dt(c), c))
    # learn this device's tag from a timed tuning of another shape set
    probe = pkg.Batch([(to_dev(S.uniform_fields((8, 8, 16), 1790), torch.float64), boxes[0][1], boxes[0][2])],
                      tune=True)
    dev = path.read_text().split()[0]
    del probe
    key = "f64:40x18x14:36x22x10"
    path.write_text(f"{dev} batch:{key} 32 8 1 0 1\n{dev} batchadj:{key} 32 12 2 0\n")
    bt = pkg.Batch(boxes, tune=True)
    assert bt.tuned_ms == -1.0 and bt.config()["tile_x"] == 32
    ws = bt.grad_workspaces(4)
    bt.grad_forward(4, ws)
    g = bt.grad_backward(4, ws, [[torch.ones_like(x) for x in f] for (f, _, _) in boxes])
    a = bt.adjoint_config()
    assert a["tile_x"] == 32 and a["tile_y"] in (4, 8), a
    assert all(np.isfinite(np.asarray(gi)).all() for gi in g)
