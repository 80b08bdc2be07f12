"""FP64 central finite differences of the 128^3 pulse misfit loss (200 steps).

Calls only the oracle (C oracle, FP64) and the seeded input generators.
Stores dL/dcoeff for the 12 coefficients (h = 1e-6 absolute), the
directional derivative of L along a seeded unit direction in the initial E,
and the loss itself.  Output: tests/golden/c4_fd.npz.
Usage: python tests/golden/make_c4_fd.py   (about 27 oracle runs)
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
from tests.workloads import c4_inputs, probe_loss  # noqa: E402

STEPS = 200
H = 1e-6


def main():
    f0, c, dt, sp, xp, tgt = c4_inputs()
    L = lambda f, cc: probe_loss(oracle.c_run(f, STEPS, cc, dt, sp), xp, tgt)
    t = time.time()
    L0 = L(f0, c)
    g = np.zeros(12)
    for j in range(12):
        cp, cm = c.copy(), c.copy()
        cp[j] += H
        cm[j] -= H
        g[j] = (L(f0, cp) - L(f0, cm)) / (2 * H)
        print(f"coeff {j}: {g[j]:.10e} ({time.time() - t:.0f}s)", flush=True)
    u = [S.unit_vector(503 + a, f0[a].size).reshape(f0[a].shape) for a in range(3)]
    fp = [f0[a] + H * u[a] if a < 3 else f0[a] for a in range(6)]
    fm = [f0[a] - H * u[a] if a < 3 else f0[a] for a in range(6)]
    dE = (L(fp, c) - L(fm, c)) / (2 * H)
    print(f"dir E0: {dE:.10e}  loss {L0:.10e}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_fd.npz")
    np.savez(path, grad_coeffs=g, dir_e0=dE, loss=L0, h=H, steps=STEPS, coeffs=c, dt=dt)
    print("wrote", path)


if __name__ == "__main__":
    main()
