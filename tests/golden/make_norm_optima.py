"""Minima of the dispersion norm f_w (Sec. 4, eq. norm) for the optimised
stencils of Table 1 (min.1-min.4) and Table 3 (min.6), computed with the
oracle's norm and scipy's bounded minimisers (2D, midpoint rule as in the
tests: n = 600, or 1200 with the eq. norm_x_axis weight).

Calls only the oracle and scipy.  Output: tests/golden/norm_optima.npz with,
per row, the optimal parameters (min.2-4: delta; min.1: beta, delta, dt, f;
min.6: beta, delta_x, f).
Usage: python tests/golden/make_norm_optima.py   (a few minutes)
"""
from __future__ import annotations

import os
import sys

import numpy as np
from scipy.optimize import minimize, minimize_scalar

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fdtd as O  # noqa: E402
from tests._pins import coeffs_2d  # noqa: E402

BIG = 1e3


def stable(c, dt):
    lo, hi = O.stability_range(c, dims=2)
    return lo >= -1e-12 * max(1.0, abs(hi)) and hi > 0 and dt * dt * hi <= 1.0


def eqbeta(dt, n=600):
    def f(d):
        c = coeffs_2d(d, d, d)
        return O.norm_fw(dt, c, dims=2, n=n) if stable(c, dt) else BIG
    r = minimize_scalar(f, bounds=(-0.125, 0.125), method="bounded", options={"xatol": 1e-9})
    return np.array([r.x, r.fun])


def min1(n=600):
    def f(v):
        b, d, t = v
        c = coeffs_2d(b, d, d)
        lo, hi = O.stability_range(c, dims=2)
        if lo < -1e-12 * max(1.0, abs(hi)) or hi <= 0:
            return BIG
        return O.norm_fw(t / np.sqrt(hi), c, dims=2, n=n)
    best = None
    for b0 in (0.0, 0.1):
        for d0 in (-0.1, 0.0):
            for t0 in (0.5, 0.95):
                r = minimize(f, [b0, d0, t0], method="L-BFGS-B",
                             bounds=[(-0.125, 0.25), (-0.125, 0.125), (0.1, 1.0)],
                             options={"ftol": 1e-15, "gtol": 1e-12})
                if best is None or r.fun < best.fun:
                    best = r
    b, d, t = best.x
    hi = O.stability_range(coeffs_2d(b, d, d), dims=2)[1]
    return np.array([b, d, t / np.sqrt(hi), best.fun])


def min6(n=1200):
    w = lambda k: np.exp(-(k[..., 1] / 0.1) ** 2)
    def f(v):
        b, dx = v
        c = coeffs_2d(b, dx, 0.0)
        return O.norm_fw(0.999, c, dims=2, n=n, weight=w) if stable(c, 0.999) else BIG
    r = minimize(f, [0.127, -0.0005], method="Nelder-Mead", options={"xatol": 1e-10, "fatol": 1e-16,
                                                                    "maxiter": 4000})
    return np.array([r.x[0], r.x[1], r.fun])


def main():
    out = {"min.2": eqbeta(0.95 / np.sqrt(2)), "min.3": eqbeta(0.5), "min.4": eqbeta(0.1), "min.1": min1(),
           "min.6": min6()}
    for k, v in out.items():
        print(k, v, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "norm_optima.npz")
    np.savez(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()
