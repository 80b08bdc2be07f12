"""Write sampled oracle results for the 1024x256x256 Gaussian-pulse workload
after 100 steps (the spot check of the sustained 5000-step run).

Calls only the oracle (and the seeded input generators).  For each variant the
FP64 C oracle runs 100 steps on the full grid; the script stores the six
components at 2048 uniformly drawn sites plus the 2048 sites where |Ey| is
largest.

  exact : the drawn coefficients, FP64 inputs (for FP64 parity);
  fp32  : the operator the FP32 weights define, FP32-rounded inputs (the FP32
          parity convention of tests/_fp32.py).

Usage: python tests/golden/make_c5a_samples.py   (about 2 min per variant on
8 cores, ~10 GB of host memory).  Output: tests/golden/c5a_pulse_<variant>.npz
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
from tests.workloads import c5a_inputs  # noqa: E402

STEPS = 100


def main(variants):
    f0, c, dt, sp = c5a_inputs()
    for var in variants:
        if var == "exact":
            fin, cc, spp = f0, c, sp
        else:
            cc, spp = _fp32.effective(c, dt, sp)
            fin = _fp32.round_fields(f0)
        t = time.time()
        out = oracle.c_run(fin, STEPS, cc, dt, spp)
        g = S.rng(2025)
        n = out[0].size
        uni = g.choice(n, size=2048, replace=False)
        top = np.argsort(np.abs(out[1]).reshape(-1))[-2048:]
        idx = np.unique(np.concatenate([uni, top]))
        vals = np.stack([o.reshape(-1)[idx] for o in out], axis=1)
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"c5a_pulse_{var}.npz")
        np.savez_compressed(path, idx=idx, vals=vals, steps=STEPS, coeffs=c, dt=dt)
        print(f"{var}: {time.time() - t:.0f}s -> {path}", flush=True)
        del out, fin


if __name__ == "__main__":
    main(sys.argv[1:] or ["exact", "fp32"])
