"""Minima of the dispersion norm f_w (Sec. 4, eq. norm) for the optimised
stencils of Table 1 (min.1-min.4) and Table 3 (min.6), computed with the
oracle's norm and the oracle's plain bounded search (successive grid
refinement, ``oracle.search``), 2D, midpoint rule as in the tests: n = 600,
or 1200 with the eq. norm_x_axis weight.

Calls only the oracle.  Output: tests/golden/norm_optima.npz with, per row,
the optimal parameters (min.2-4: delta, f; min.1: beta, delta, dt, f;
min.6: beta, delta_x, f).
Usage: python tests/golden/make_norm_optima.py   (several minutes)
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fdtd as O  # noqa: E402
from oracle.search import refine_grid_search  # noqa: E402
from tests._pins import coeffs_2d  # noqa: E402

TOL = 1e-10


def stable(c, dt):
    lo, hi = O.stability_range(c, dims=2)
    return lo >= -1e-12 * max(1.0, abs(hi)) and hi > 0 and dt * dt * hi <= 1.0


def eqbeta(dt, n=600):
    """Table 1 min.2-4: eq.(beta) with delta_x = delta_y = beta = d, dt fixed."""
    def f(x):
        c = coeffs_2d(x[0], x[0], x[0])
        return O.norm_fw(dt, c, dims=2, n=n) if stable(c, dt) else np.inf
    x, v, _ = refine_grid_search(f, [-0.125], [0.125], points=9, tol=TOL)
    return np.array([x[0], v])


def min1(n=600):
    """Table 1 min.1: beta, delta = delta_x = delta_y free, dt a fraction t of
    the stencil's own stability bound."""
    def f(x):
        b, d, t = x
        c = coeffs_2d(b, d, d)
        lo, hi = O.stability_range(c, dims=2)
        if lo < -1e-12 * max(1.0, abs(hi)) or hi <= 0:
            return np.inf
        return O.norm_fw(t / np.sqrt(hi), c, dims=2, n=n)
    x, v, _ = refine_grid_search(f, [-0.125, -0.125, 0.1], [0.25, 0.125, 1.0], points=7, tol=TOL)
    b, d, t = x
    hi = O.stability_range(coeffs_2d(b, d, d), dims=2)[1]
    return np.array([b, d, t / np.sqrt(hi), v])


def min6(n=1200):
    """Table 3 min.6: c dt/dx = 0.999, beta_xy = beta_yx = b and delta_x free,
    delta_y = 0, weight exp(-(k_y/0.1)^2) (eq. norm_x_axis)."""
    w = lambda k: np.exp(-(k[..., 1] / 0.1) ** 2)
    def f(x):
        c = coeffs_2d(x[0], x[1], 0.0)
        return O.norm_fw(0.999, c, dims=2, n=n, weight=w) if stable(c, 0.999) else np.inf
    x, v, _ = refine_grid_search(f, [0.10, -0.01], [0.15, 0.01], points=7, tol=TOL)
    return np.array([x[0], x[1], v])


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
