"""Sampled oracle results of the 64-box batched workload after 500 steps.

Calls only the oracle and the seeded input generators.  Each box runs in the
FP64 C oracle with the operator its FP32 weights define, from FP32-rounded
inputs (the FP32 convention of tests/_fp32.py); 256 uniformly drawn sites per
box are stored.  Output: tests/golden/c3_boxes_fp32.npz
Usage: python tests/golden/make_c3_samples.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic as S  # noqa: E402
from tests import _fp32  # noqa: E402
from tests.workloads import c3_boxes  # noqa: E402

STEPS = 500


def main():
    t = time.time()
    idx_all, vals_all = [], []
    for b, (shape, f0, c, dt) in enumerate(c3_boxes()):
        ce, spe = _fp32.effective(c, dt)
        out = oracle.c_run(_fp32.round_fields(f0), STEPS, ce, dt, spe)
        idx = S.rng(9000 + b).choice(out[0].size, size=256, replace=False)
        idx_all.append(idx)
        vals_all.append(np.stack([o.reshape(-1)[idx] for o in out], axis=1))
        print(f"box {b} {shape}: {time.time() - t:.0f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_boxes_fp32.npz")
    np.savez_compressed(path, idx=np.stack(idx_all), vals=np.stack(vals_all), steps=STEPS)
    print("wrote", path)


if __name__ == "__main__":
    main()
