"""FP64 central finite differences of the batched coefficient-tuning loss:
16 boxes of 96^3, 300 steps, one pulse, one extended set per box.

Calls only the oracle (C oracle, FP64) and the seeded input generators.
For box b it stores the directional derivatives of that box's probe misfit
along two seeded unit directions in the 12 coefficients (seeds 530 + b and
560 + b), h = 1e-6 absolute, and for boxes 0, 5, 8 and 15 the central
difference of every one of the 12 coefficients.
Output: tests/golden/c5_fd.npz.
Usage: python tests/golden/make_c5_fd.py   (160 oracle runs)
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


FULL = (0, 5, 8, 15)  # boxes whose 12 coefficient derivatives are all stored


def main():
    boxes = c5_boxes(steps=STEPS)
    t = time.time()
    dirs, dd, dirs2, dd2, coeffs, dts = [], [], [], [], [], []
    full = np.zeros((len(FULL), 12))
    for b, (f0, c, dt, sp, xp, tgt) in enumerate(boxes):
        L = lambda cc: probe_loss(oracle.c_run(f0, STEPS, cc, dt, sp), xp, tgt)
        for seed, vs, ds in ((530 + b, dirs, dd), (560 + b, dirs2, dd2)):
            v = S.unit_vector(seed, 12)
            vs.append(v)
            ds.append((L(c + H * v) - L(c - H * v)) / (2 * H))
        coeffs.append(c)
        dts.append(dt)
        if b in FULL:
            for j in range(12):
                e = np.zeros(12)
                e[j] = H
                full[FULL.index(b), j] = (L(c + e) - L(c - e)) / (2 * H)
        print(f"box {b}: {dd[-1]:.10e} {dd2[-1]:.10e} ({time.time() - t:.0f}s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_fd.npz")
    np.savez(path, dirs=np.array(dirs), dir_deriv=np.array(dd), dirs2=np.array(dirs2), dir_deriv2=np.array(dd2),
             full_boxes=np.array(FULL), full_grad=full, coeffs=np.array(coeffs), dt=np.array(dts),
             h=H, steps=STEPS)
    print("wrote", path)


if __name__ == "__main__":
    main()
