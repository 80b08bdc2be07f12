"""FP64 central finite differences of the 128^3 pulse misfit loss (200 steps).

Calls only the oracle (C oracle, FP64) and the seeded input generators.
Stores dL/dcoeff for the 12 coefficients (h = 1e-6 absolute), the
directional derivative of L along a seeded unit direction in the initial E,
dL/dE0 at 16 sampled entries (8 drawn among the 4096 largest |E0_y| sites of
the pulse, 8 drawn uniformly; components drawn among Ex, Ey, Ez; seed 504),
and the loss itself.  Output: tests/golden/c4_fd.npz.
Usage: python tests/golden/make_c4_fd.py [entries]   (about 59 oracle runs;
"entries" computes only the sampled entries and adds them to the stored file)
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


def sampled_entries(f0):
    """(component, flat index) of the 16 sampled initial-E entries."""
    g = S.rng(504)
    top = np.argsort(np.abs(f0[1]).reshape(-1))[-4096:]
    sites = np.concatenate([g.choice(top, 8, replace=False), g.choice(f0[1].size, 8, replace=False)])
    comps = g.integers(0, 3, 16)
    return comps, sites


def entries_fd(f0, c, L):
    comps, sites = sampled_entries(f0)
    vals = np.zeros(16)
    t = time.time()
    for q in range(16):
        fp = [x.copy() if a == comps[q] else x for a, x in enumerate(f0)]
        fm = [x.copy() if a == comps[q] else x for a, x in enumerate(f0)]
        fp[comps[q]].reshape(-1)[sites[q]] += H
        fm[comps[q]].reshape(-1)[sites[q]] -= H
        vals[q] = (L(fp, c) - L(fm, c)) / (2 * H)
        print(f"entry {q} (comp {comps[q]}, site {sites[q]}): {vals[q]:.10e} ({time.time() - t:.0f}s)", flush=True)
    return comps, sites, vals


def main(only_entries=False):
    f0, c, dt, sp, xp, tgt = c4_inputs()
    L = lambda f, cc: probe_loss(oracle.c_run(f, STEPS, cc, dt, sp), xp, tgt)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_fd.npz")
    if only_entries:
        old = dict(np.load(path))
        assert np.array_equal(old["coeffs"], c) and float(old["dt"]) == dt
        old["e0_comp"], old["e0_site"], old["e0_grad"] = entries_fd(f0, c, L)
        np.savez(path, **old)
        print("wrote", path)
        return
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
    ec, es, ev = entries_fd(f0, c, L)
    np.savez(path, grad_coeffs=g, dir_e0=dE, loss=L0, h=H, steps=STEPS, coeffs=c, dt=dt,
             e0_comp=ec, e0_site=es, e0_grad=ev)
    print("wrote", path)


if __name__ == "__main__":
    main(only_entries=sys.argv[1:] == ["entries"])
