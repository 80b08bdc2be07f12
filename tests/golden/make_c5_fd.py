"""FP64 central finite differences of the batched coefficient-tuning loss:
16 boxes of 96^3, 300 steps, one pulse, one extended set per box.

Calls only the oracle (C oracle, FP64) and the seeded input generators.
For box b it stores the directional derivative of that box's probe misfit
along a seeded unit direction in the 12 coefficients (seed 530 + b),
h = 1e-6 absolute, and the loss.  Output: tests/golden/c5_fd.npz.
Usage: python tests/golden/make_c5_fd.py   (32 oracle runs)
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
from tests.workloads import c5_boxes, probe_loss  # noqa: E402

STEPS = 300
H = 1e-6


def main():
    boxes = c5_boxes(steps=STEPS)
    t = time.time()
    dirs, dd, coeffs, dts = [], [], [], []
    for b, (f0, c, dt, sp, xp, tgt) in enumerate(boxes):
        v = S.unit_vector(530 + b, 12)
        L = lambda cc: probe_loss(oracle.c_run(f0, STEPS, cc, dt, sp), xp, tgt)
        d = (L(c + H * v) - L(c - H * v)) / (2 * H)
        dirs.append(v)
        dd.append(d)
        coeffs.append(c)
        dts.append(dt)
        print(f"box {b}: {d:.10e} ({time.time() - t:.0f}s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_fd.npz")
    np.savez(path, dirs=np.array(dirs), dir_deriv=np.array(dd), coeffs=np.array(coeffs), dt=np.array(dts),
             h=H, steps=STEPS)
    print("wrote", path)


if __name__ == "__main__":
    main()
