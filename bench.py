"""Benchmark of the extended-stencil FDTD time step on one MI355X.

Workload (one step = Faraday + Ampere over the whole box, the fused
out-of-place kernel): 512 x 256 x 256 periodic box, FP32, seed-drawn extended
coefficient set, Gaussian pulse along x (wavelength 16, waist 32, duration 40
cells) plus 1e-3 uniform noise; dt = 0.95 x the stability bound.  Inputs are
synthetic and resident in HBM before timing starts.

Prints one JSON line: Gcell-updates/s, the roofline object of the fused kernel
(algorithmic 48 B per cell-update against 8 TB/s), and the FP64 CPU oracle
timed on the host cores on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--no-cpu] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SHAPE = (256, 256, 512)  # (nz, ny, nx)
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1710_06829_amd", "csrc", "kernels_step.hip")
PROFILES = {1: os.path.join(ROOT, "profiles", "fused_step_512x256x256_fp32.md"),
            2: os.path.join(ROOT, "profiles", "two_step_512x256x256_fp32.md")}
TILE_NAMES = {(64, 4): "TileCfg<1,8,64>", (64, 8): "TileCfg<1,12,64>", (64, 16): "TileCfg<2,10,64>",
              (32, 4): "TileCfg<1,4,32>", (32, 8): "TileCfg<1,6,32>", (32, 16): "TileCfg<2,5,32>"}
# Batches replay a captured graph and single boxes replay graphs of 32 steps;
# --no-graph launches everything directly (rocprofv3 counter passes).
USE_GRAPH = True
BLK_NAMES = {(32, 16): "Blk2Cfg<32,16,1,15>", (32, 8): "Blk2Cfg<32,8,1,10>"}


def measured_traffic(steps_per_pass=1):
    """HBM bytes per launch of the timed kernel (one-step or two-step) from the
    committed rocprofv3 summary (FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy), or None when the kernel source has changed since those counters
    were taken."""
    import hashlib
    import re
    try:
        txt = open(PROFILES[steps_per_pass]).read()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    m_sha = re.search(r"kernel_sha256:\s*([0-9a-f]{64})", txt)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))
METRIC = "Gcell-updates/s & %HBM roofline (fwd), fwd+adjoint time/step vs plain fwd"


def make_inputs(shape, dtype):
    """Seeded pulse workload; coefficients and dt from the library itself."""
    import numpy as np
    import torch

    import synthetic as S
    import paper_1710_06829_amd as pkg

    beta, delta = S.extended_beta_delta(201)
    raw = [0.0] * 12
    for a in range(3):
        raw[4 * a + 1], raw[4 * a + 2], raw[4 * a + 3] = beta[a, 0], beta[a, 1], delta[a]
    coeffs = pkg.consistent_alpha(raw)
    dt_max, _, _ = pkg.cfl_limit(shape, coeffs)
    dt = 0.95 * dt_max
    f = S.gaussian_pulse(shape, dt, wavelength=16.0, waist=32.0, duration=40.0)
    f = S.add_noise(f, 1e-3, 202)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(np.ascontiguousarray(x)).to(device=dev, dtype=dtype) for x in f]
    return t, coeffs, dt, f


def cpu_model():
    """The host CPU's model name and logical CPU count, from /proc/cpuinfo."""
    try:
        names = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")]
    except OSError:
        return "unknown"
    return f"{names[0]} ({len(names)} logical CPUs visible)" if names else "unknown"


def cpu_baseline(f64_fields, coeffs, dt, steps):
    """The FP64 C oracle, as it stands, on the full grid for `steps` steps."""
    import oracle

    cells = f64_fields[0].size
    t0 = time.perf_counter()
    oracle.c_run(f64_fields, steps, coeffs, dt)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {
        "value": cells * steps / el / 1e9,
        "unit": "Gcell-updates/s",
        "cores": threads,
        "cpu": cpu_model(),
        "kind": "oracle",
        "sample": f"{steps} FP64 steps of the full 512x256x256 pulse workload "
                  f"(plain C oracle, OpenMP, {el:.1f} s)",
    }


def adjoint_step_rate(steps=40):
    """One adjoint step (the transposed update with its 12 coefficient-gradient
    partials) on the 512x256x256 FP32 workload with nothing else running:
    time per step and HBM rate at 60 B per cell (the 6 adjoint components
    read and written once, the 3 primal E components read once)."""
    import torch

    import paper_1710_06829_amd as pkg

    fields, coeffs, dt, _ = make_inputs(SHAPE, torch.float32)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    la = [torch.rand(SHAPE, device="cuda", generator=g) * 2 - 1 for _ in range(6)]
    lb = [torch.empty_like(x) for x in la]
    s = pkg.Solver(fields, dt, coeffs, scratch=False)
    gr = torch.zeros(12, dtype=torch.float64, device="cuda")
    steps = max(2, steps + (steps & 1))
    for i in range(4):
        s.adjoint_step(la, lb, fields[:3], gr) if i % 2 == 0 else s.adjoint_step(lb, la, fields[:3], gr)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    best = float("inf")
    for rep in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            s.adjoint_step(la, lb, fields[:3], gr) if i % 2 == 0 else s.adjoint_step(lb, la, fields[:3], gr)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / steps)
    cells = SHAPE[0] * SHAPE[1] * SHAPE[2]
    gbs = 60.0 * cells / (best * 1e-3) / 1e9
    del s, fields, la, lb
    return {"workload": "512x256x256 FP32 adjoint step (transposed update + 12 coefficient-gradient partials)",
            "us_per_step": round(best * 1e3, 2), "bytes_per_cell": 60,
            "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "kernel": "adjoint_step_kernel"}


def fwd_adj_ratio(steps=200):
    """Time of the checkpointed forward + adjoint over the plain forward, on the
    128^3 FP32 differentiation workload (Gaussian pulse, wavelength 12, probe
    plane loss), sqrt(N) checkpoints (segments of ceil(sqrt(2N)) steps)."""
    import math

    import numpy as np
    import torch

    import synthetic as S
    import paper_1710_06829_amd as pkg

    shape = (128, 128, 128)
    beta, delta = S.extended_beta_delta(501)
    raw = [0.0] * 12
    for a in range(3):
        raw[4 * a + 1], raw[4 * a + 2], raw[4 * a + 3] = beta[a, 0], beta[a, 1], delta[a]
    coeffs = pkg.consistent_alpha(raw)
    dt = 0.95 * pkg.cfl_limit(shape, coeffs)[0]
    f = S.add_noise(S.gaussian_pulse(shape, dt, 12.0, 24.0, 30.0), 1e-3, 502)
    dev = torch.device("cuda:0")
    f32 = [torch.from_numpy(np.ascontiguousarray(x)).to(device=dev, dtype=torch.float32) for x in f]
    ev = lambda: torch.cuda.Event(enable_timing=True)

    plain = [x.clone() for x in f32]
    sp = pkg.Solver(plain, dt, coeffs)
    sp.run(10)
    fwd_times = []
    for rep in range(3):  # the same protocol as the fwd+adj timing below: min of 3
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        sp.run(steps)
        e1.record()
        torch.cuda.synchronize()
        fwd_times.append(e0.elapsed_time(e1))
    t_fwd = min(fwd_times)

    seg = int(math.ceil(math.sqrt(2 * steps)))  # the library's default segment
    work = [x.clone() for x in f32]
    sg = pkg.Solver(work, dt, coeffs, scratch=False)
    ws = torch.empty(sg.grad_workspace_bytes(steps, seg), dtype=torch.uint8, device=dev)
    lam = [torch.zeros_like(x) for x in work]
    xp = int(round(0.25 * shape[2] + steps * dt)) % shape[2]
    times = []
    for rep in range(3):
        for a in range(6):
            work[a].copy_(f32[a])
        torch.cuda.synchronize()
        e0, em, e1 = ev(), ev(), ev()
        e0.record()
        sg.grad_forward(steps, ws, seg)
        em.record()
        for a in range(6):
            lam[a].zero_()
        for a in range(3):
            lam[a][:, :, xp] = work[a][:, :, xp]
        sg.grad_backward(steps, ws, lam, seg)
        e1.record()
        torch.cuda.synchronize()
        times.append((e0.elapsed_time(e1), e0.elapsed_time(em)))
    t_fa, t_gf = min(times)
    # every E kept (one segment of n steps: no recompute), for comparison
    ws2 = torch.empty(sg.grad_workspace_bytes(steps, steps), dtype=torch.uint8, device=dev)
    for a in range(6):
        work[a].copy_(f32[a])
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    sg.grad_forward(steps, ws2, steps)
    for a in range(6):
        lam[a].zero_()
    for a in range(3):
        lam[a][:, :, xp] = work[a][:, :, xp]
    sg.grad_backward(steps, ws2, lam, steps)
    e1.record()
    torch.cuda.synchronize()
    t_all = e0.elapsed_time(e1)
    return {"ratio": round(t_fa / t_fwd, 3), "fwd_ms": round(t_fwd, 3), "fwd_adj_ms": round(t_fa, 3),
            "grad_forward_ms": round(t_gf, 3), "grad_backward_ms": round(t_fa - t_gf, 3),
            "steps": steps, "segment": seg,
            "ratio_all_E_kept": round(t_all / t_fwd, 3),
            "workload": "128^3 FP32 Gaussian pulse (wavelength 12), "
            "probe-plane misfit loss, gradients w.r.t. 12 coefficients and initial fields"}


def plane_2d(steps=200, edge=2048):
    """A box one plane deep (edge x edge x 1 FP32, the pulse workload):
    forward rate on the plane kernel, the one-plane adjoint step against 60 B
    per cell, and the checkpointed forward + backward over the forward with
    sqrt(N) segments (adjoint seeds drawn uniformly)."""
    import math

    import torch

    import paper_1710_06829_amd as pkg

    shape = (1, edge, edge)
    f, coeffs, dt, _ = make_inputs(shape, torch.float32)
    cells = edge * edge
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    sp = pkg.Solver([x.clone() for x in f], dt, coeffs)
    sp.run(10)
    t_fwd = min(timed(lambda: sp.run(steps)) for _ in range(3))
    seg = int(math.ceil(math.sqrt(2 * steps)))
    work = [x.clone() for x in f]
    sg = pkg.Solver(work, dt, coeffs, scratch=False)
    ws = torch.empty(sg.grad_workspace_bytes(steps, seg), dtype=torch.uint8, device=f[0].device)
    gen = torch.Generator(device=f[0].device)
    gen.manual_seed(560)
    lam0 = [torch.rand(x.shape, device=x.device, generator=gen) * 2 - 1 for x in work]
    lam = [x.clone() for x in lam0]
    best = None
    for rep in range(3):
        for a in range(6):
            work[a].copy_(f[a])
            lam[a].copy_(lam0[a])
        tf = timed(lambda: sg.grad_forward(steps, ws, seg))
        tb = timed(lambda: sg.grad_backward(steps, ws, lam, seg))
        if best is None or tf + tb < sum(best):
            best = (tf, tb)
    g = torch.zeros(12, dtype=torch.float64, device=f[0].device)
    lb = [torch.empty_like(x) for x in lam0]
    sg.adjoint_step(lam0, lb, f[:3], g)
    n_adj = 50
    t_adj = min(timed(lambda: [sg.adjoint_step(lam0, lb, f[:3], g) for _ in range(n_adj)]) for _ in range(3)) / n_adj
    return {"workload": f"{edge}x{edge}x1 FP32 pulse box (one plane deep), {steps} steps",
            "forward_us_per_step": round(t_fwd / steps * 1e3, 2),
            "Gcell_updates_per_s": round(cells * steps / (t_fwd * 1e-3) / 1e9, 2),
            "hbm_frac_48B": round(48.0 * cells / (t_fwd / steps * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "adjoint_us_per_step": round(t_adj * 1e3, 2),
            "adjoint_frac_60B": round(60.0 * cells / (t_adj * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "grad_forward_ms": round(best[0], 3), "grad_backward_ms": round(best[1], 3), "segment": seg,
            "ratio_to_forward": round(sum(best) / t_fwd, 3)}


def fp64_step(steps=200):
    """The 512x256x256 pulse workload in FP64 (tuned launch): rate and the
    fraction of 8 TB/s at 96 algorithmic bytes per cell-update."""
    import torch

    import paper_1710_06829_amd as pkg

    fields, coeffs, dt, _ = make_inputs(SHAPE, torch.float64)
    s = pkg.Solver(fields, dt, coeffs)
    lc = s.tune()
    s.run(10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s.run(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = SHAPE[0] * SHAPE[1] * SHAPE[2]
    gc = cells * steps / (ms * 1e-3) / 1e9
    return {"workload": "512x256x256 FP64 pulse workload, fused step", "steps": steps,
            "ms_per_step": round(ms / steps, 4), "Gcell_updates_per_s": round(gc, 2),
            "hbm_roofline_pct": round(100.0 * gc * 96.0 / HBM_PEAK_GBS, 2), "launch": lc}


def sustained_large(steps=5000):
    """1024x256x256 FP32 box, 5000 steps of a Gaussian pulse (wavelength 20,
    waist 40, duration 50 cells; extended set seed 601): sustained rate."""
    import numpy as np
    import torch

    import synthetic as S
    import paper_1710_06829_amd as pkg

    shape = (256, 256, 1024)
    beta, delta = S.extended_beta_delta(601)
    raw = [0.0] * 12
    for a in range(3):
        raw[4 * a + 1], raw[4 * a + 2], raw[4 * a + 3] = beta[a, 0], beta[a, 1], delta[a]
    coeffs = pkg.consistent_alpha(raw)
    dt = 0.95 * pkg.cfl_limit(shape, coeffs)[0]
    f = S.gaussian_pulse(shape, dt, 20.0, 40.0, 50.0)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(np.ascontiguousarray(x)).to(device=dev, dtype=torch.float32) for x in f]
    del f
    s = pkg.Solver(t, dt, coeffs)
    s.run(10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s.run(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = shape[0] * shape[1] * shape[2]
    _, _, bad = s.divergence_max(raise_nonfinite=False)
    return {"workload": "1024x256x256 FP32 Gaussian pulse (wavelength 20), 5000 steps",
            "steps": steps, "seconds": round(ms / 1e3, 3),
            "Gcell_updates_per_s": round(cells * steps / (ms * 1e-3) / 1e9, 2),
            "launch": s.launch_config(), "nonfinite": bad}


def batched_boxes(steps=500):
    """64 periodic boxes (edges iid in {32, 48, 64, 96, 128}, own coefficient
    sets and random FP32 fields): one graph-captured batched run vs 64
    sequential single-box runs."""
    import numpy as np
    import torch

    import synthetic as S
    import paper_1710_06829_amd as pkg

    dev = torch.device("cuda:0")
    boxes, seq = [], []
    cells = 0
    for b, (nx, ny, nz) in enumerate(S.box_edges(64, 301)):
        beta, delta = S.extended_beta_delta(302 + b)
        raw = [0.0] * 12
        for a in range(3):
            raw[4 * a + 1], raw[4 * a + 2], raw[4 * a + 3] = beta[a, 0], beta[a, 1], delta[a]
        c = pkg.consistent_alpha(raw)
        shape = (nz, ny, nx)
        dt = 0.95 * pkg.cfl_limit(shape, c)[0]
        f = [torch.from_numpy(x).to(device=dev, dtype=torch.float32) for x in S.uniform_fields(shape, 400 + b)]
        boxes.append(([x.clone() for x in f], dt, c))
        seq.append((f, dt, c))
        cells += nx * ny * nz
    bt = pkg.Batch(boxes, tune=True)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    bt.run(steps, graph=USE_GRAPH)  # captures the graph (first call)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    bt.run(steps, graph=USE_GRAPH)
    e1.record()
    torch.cuda.synchronize()
    t_b = e0.elapsed_time(e1)
    solvers = [pkg.Solver(f, dt, c) for (f, dt, c) in seq]
    for s in solvers:  # the sequential baseline gets its own per-box tuning
        s.tune()
        s.run(2)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for s in solvers:
        s.run(steps)
    e1.record()
    torch.cuda.synchronize()
    t_s = e0.elapsed_time(e1)
    return {"workload": "64 boxes, edges in {32,48,64,96,128}, FP32, 500 steps", "cells": cells,
            "batched_ms": round(t_b, 3), "sequential_ms": round(t_s, 3),
            "batched_Gcell_updates_per_s": round(cells * steps / (t_b * 1e-3) / 1e9, 2),
            # the metric's 48 B per cell-update over the batch / 8 TB/s
            "hbm_roofline_frac": round(cells * steps / (t_b * 1e-3) * 48.0 / (HBM_PEAK_GBS * 1e9), 4),
            "sequential_Gcell_updates_per_s": round(cells * steps / (t_s * 1e-3) / 1e9, 2),
            "speedup": round(t_s / t_b, 3), "config": bt.config()}


def batched_grads(steps=300, count=16, edge=96):
    """16 extended coefficient sets on 96^3 FP32 pulse boxes, 300 steps:
    batched checkpointed forward + adjoint vs the batched forward alone and
    vs 16 sequential single-box gradient runs."""
    import torch

    import synthetic as S
    import paper_1710_06829_amd as pkg

    dev = torch.device("cuda:0")
    shape = (edge, edge, edge)
    boxes = []
    for b in range(count):
        beta, delta = S.extended_beta_delta(520 + 10 * b)
        raw = [0.0] * 12
        for a in range(3):
            raw[4 * a + 1], raw[4 * a + 2], raw[4 * a + 3] = beta[a, 0], beta[a, 1], delta[a]
        c = pkg.consistent_alpha(raw)
        dt = 0.95 * pkg.cfl_limit(shape, c)[0]
        f = S.add_noise(S.gaussian_pulse(shape, dt, wavelength=12.0, waist=16.0, duration=16.0,
                                         x0=0.5 * edge), 1e-3, 521)
        boxes.append(([torch.from_numpy(x).to(device=dev, dtype=torch.float32) for x in f], dt, c))
    lam0 = [torch.from_numpy(x).to(device=dev, dtype=torch.float32) for x in S.uniform_fields(shape, 540)]
    init = [[x.clone() for x in f] for (f, _, _) in boxes]
    bt = pkg.Batch(boxes, tune=True)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def reset():
        for (f, _, _), f0 in zip(boxes, init):
            for a, b in zip(f, f0):
                a.copy_(b)

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    bt.run(steps, graph=USE_GRAPH)  # graph capture
    reset()
    t_fwd = timed(lambda: bt.run(steps, graph=USE_GRAPH))
    ws = bt.grad_workspaces(steps)
    lams = [[x.clone() for x in lam0] for _ in range(count)]
    reset()
    bt.grad_forward(steps, ws)
    bt.grad_backward(steps, ws, lams)  # warm-up (descriptor uploads, buffers)
    reset()
    lams = [[x.clone() for x in lam0] for _ in range(count)]
    t_f = timed(lambda: bt.grad_forward(steps, ws))
    t_b = timed(lambda: bt.grad_backward(steps, ws, lams))
    del ws
    torch.cuda.empty_cache()
    reset()
    solvers = [pkg.Solver(f, dt, c, scratch=False) for (f, dt, c) in boxes]
    w1 = torch.empty(solvers[0].grad_workspace_bytes(steps), dtype=torch.uint8, device=dev)
    lam1 = [x.clone() for x in lam0]

    def seq():
        for s in solvers:
            s.grad_forward(steps, w1)
            s.grad_backward(steps, w1, lam1)

    seq()
    reset()
    t_s = timed(seq)
    cells = count * edge ** 3
    return {"workload": f"{count} extended sets x {edge}^3 FP32 pulse boxes, {steps} steps, forward+adjoint",
            "forward_ms": round(t_fwd, 3), "grad_forward_ms": round(t_f, 3), "grad_backward_ms": round(t_b, 3),
            "fwd_adj_ms": round(t_f + t_b, 3), "ratio_to_forward": round((t_f + t_b) / t_fwd, 3),
            "sequential_fwd_adj_ms": round(t_s, 3), "speedup_vs_sequential": round(t_s / (t_f + t_b), 3),
            "Gcell_updates_per_s_fwd_adj": round(cells * steps / ((t_f + t_b) * 1e-3) / 1e9, 2),
            "config": bt.config(), "adjoint_config": bt.adjoint_config()}


def norm_bench():
    """Dispersion norm f_w with its gradient (3D n = 256 and 2D n = 1000
    midpoint grids) and the minimisation of Table 1's min.1 family."""
    import time

    import numpy as np
    import torch

    import paper_1710_06829_amd as pkg

    beta, delta = 0.110, -0.125
    c = [1 - 2 * beta - 3 * delta, beta, 0.0, delta, 1 - 2 * beta - 3 * delta, beta, 0.0, delta,
         1.0, 0.0, 0.0, 0.0]
    out = {}
    for dims, n, dt in ((3, 256, 0.5), (2, 1000, 0.686)):
        pkg.dispersion_norm(dt, c, dims=dims, n=n)
        ts = []
        for _ in range(10):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f, _ = pkg.dispersion_norm(dt, c, dims=dims, n=n)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        out[f"{dims}d_n{n}"] = {"samples": n ** dims, "ms": round(t * 1e3, 3),
                                "Gsamples_per_s": round(n ** dims / t / 1e9, 3), "f": f}
    fam = (pkg.Family().param(-0.125, 0.25, beta_xy=1, beta_yx=1)
           .param(-0.125, 0.125, delta_x=1, delta_y=1).dt_fraction(0.1, 1.0))
    t0 = time.perf_counter()
    r = pkg.optimize_stencil(fam, dims=2, n=1000, starts=3)
    out["minimise_table1_min1"] = {"seconds": round(time.perf_counter() - t0, 3), "evaluations": r["evals"],
                                   "beta": round(r["x"][0], 5), "delta": round(r["x"][1], 5),
                                   "dt": round(r["dt"], 5), "f": r["f"]}
    return out


def calib_copy(gib=1.0, reps=5):
    """A plain device copy of known size (for scaling rocprofv3 byte counters);
    returns its size and achieved bandwidth (read + write bytes per second)."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes": n * 4, "copy_GBps": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-adj", action="store_true")
    ap.add_argument("--calib", action="store_true", help="also run a 1 GiB plain copy")
    ap.add_argument("--adj-only", action="store_true", help="only the fwd+adjoint measurement")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the 512x256x256 adjoint step (--steps adjoint steps)")
    ap.add_argument("--grad-batch-only", action="store_true", help="only the batched gradient measurement")
    ap.add_argument("--norm-only", action="store_true", help="only the dispersion-norm measurement")
    ap.add_argument("--fp64-only", action="store_true", help="only the FP64 512x256x256 measurement")
    ap.add_argument("--batch-only", action="store_true", help="only the 64-box batched measurement")
    ap.add_argument("--plane-only", action="store_true", help="only the 2048^2 one-plane measurement")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch kernels directly instead of replaying captured graphs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 1024x256x256 sustained run and the 64-box batch")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.no_graph:
        global USE_GRAPH
        USE_GRAPH = False
        os.environ["XFDTD_GRAPH"] = "0"  # read when a solver is created
    import torch

    import paper_1710_06829_amd as pkg

    if args.adj_only:
        print(json.dumps({"fwd_adj": fwd_adj_ratio()}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint_512x256x256": adjoint_step_rate(args.steps)}), flush=True)
        return
    if args.norm_only:
        print(json.dumps({"dispersion_norm": norm_bench()}), flush=True)
        return
    if args.grad_batch_only:
        print(json.dumps({"batched_grads_16x96cube": batched_grads()}), flush=True)
        return
    if args.fp64_only:
        print(json.dumps({"fp64_512x256x256": fp64_step()}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batched_64_boxes": batched_boxes()}), flush=True)
        return
    if args.plane_only:
        print(json.dumps({"plane_2048x2048": plane_2d()}), flush=True)
        return
    fields, coeffs, dt, f64 = make_inputs(SHAPE, torch.float32)
    solver = pkg.Solver(fields, dt, coeffs)
    lc = solver.tune()
    spp = lc["steps_per_pass"]
    cells = SHAPE[0] * SHAPE[1] * SHAPE[2]
    # run() keeps the result in the bound fields with an even number of
    # launches: a multiple of 2 steps (one-step kernel) or of 4 (two-step
    # kernel) makes every timed launch the tuned kernel
    q = 2 * spp
    steps = (args.steps + q - 1) // q * q

    solver.run(args.warmup + (args.warmup & 1))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    solver.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_step = ms / steps
    gcells = cells * steps / (ms * 1e-3) / 1e9
    # every launch in the timed region is the tuned kernel, which advances
    # every cell spp steps; its algorithmic bytes are 48 B per cell-update
    # (each of the 6 FP32 components read once and written once per step)
    # times the spp x cells cell-updates of a launch.  The kernel itself
    # reads and writes the state once per launch (48 B per cell), which for
    # the two-step kernel is half of that.
    launches = steps // spp
    ms_launch = ms / launches
    bytes_per_launch = 48.0 * cells * spp
    kernel_min_bytes = 48.0 * cells
    achieved = bytes_per_launch / (ms_launch * 1e-3) / 1e9
    if spp == 2:
        tl = lc["two_step"]
        kname = f"blocked2_kernel<float, {BLK_NAMES.get((tl['tile_x'], tl['tile_y']), tl['tile_y'])}>"
    else:
        kname = f"fused_step_kernel<float, {TILE_NAMES.get((lc['tile_x'], lc['tile_y']), lc['tile_y'])}>"
    del solver, fields
    torch.cuda.empty_cache()

    line = {
        "metric": METRIC,
        "value": round(gcells, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "512x256x256 periodic box, FP32, extended Faraday stencil "
                        "(seed-drawn set), Gaussian pulse along x + 1e-3 noise, "
                        "dt = 0.95 x stability bound, autotuned kernel "
                        f"({spp} step{'s' if spp == 2 else ''} per pass)",
            "grid": [SHAPE[2], SHAPE[1], SHAPE[0]],
            "cells": cells,
        },
        # the metric's roofline: Gcell-updates/s x 48 B (the one-step bytes of
        # a cell-update) / 8 TB/s
        "hbm_roofline_pct": round(100.0 * gcells * 48.0 / HBM_PEAK_GBS, 2),
        "steps_per_pass": spp,
        "bytes_per_cell_update": 48.0 / spp,
        "wall_s": round(wall, 4),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(spp),
            "kernel": kname,
            "launch": lc,
            "bytes_per_launch": bytes_per_launch,
            "cell_updates_per_launch": cells * spp,
            "kernel_state_bytes_per_launch": kernel_min_bytes,
            "kernel_state_GBs": round(kernel_min_bytes / (ms_launch * 1e-3) / 1e9, 1),
            "ms_per_launch": round(ms_launch, 5),
        },
        "cpu_baseline": None,
    }
    if not args.no_adj:
        line["fwd_adj"] = fwd_adj_ratio()
        torch.cuda.empty_cache()
        line["adjoint_512x256x256"] = adjoint_step_rate()
        torch.cuda.empty_cache()
    if not args.no_extra:
        line["fp64_512x256x256"] = fp64_step()
        torch.cuda.empty_cache()
        line["sustained_1024x256x256"] = sustained_large()
        torch.cuda.empty_cache()
        line["batched_64_boxes"] = batched_boxes()
        torch.cuda.empty_cache()
        line["batched_grads_16x96cube"] = batched_grads()
        torch.cuda.empty_cache()
        line["plane_2048x2048"] = plane_2d()
        torch.cuda.empty_cache()
        line["dispersion_norm"] = norm_bench()
    if args.calib:
        line["calib_copy"] = calib_copy()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(f64, coeffs, dt, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
