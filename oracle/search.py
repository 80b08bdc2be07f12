"""Plain bounded search for the minima of the dispersion norm (Sec. 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper minimises f_w over a few stencil parameters inside a box and under
the stability constraints of eq. constraints, and prints the optima (Tables 1
and 3).  The stored optima the tests compare against are found here by the
most direct bounded search there is, successive grid refinement: evaluate the
objective on a regular grid over the box, keep the best feasible grid point,
shrink the box around it, repeat.  Infeasible points (unstable stencils) are
reported by the objective as +inf and never kept, so a minimum on the
stability boundary is approached from the stable side.  No derivatives, no
line searches, no library minimiser.
"""
from __future__ import annotations

import itertools

import numpy as np


def refine_grid_search(f, lo, hi, points=5, shrink=0.5, tol=1e-10, max_levels=200):
    """Minimise f over the box lo <= x <= hi (arrays of equal length).

    Each level evaluates f at ``points`` equally spaced values per coordinate
    (the box's end points included) and keeps the best point with a finite
    value; the next box is centred on it with its widths scaled by ``shrink``,
    clipped to the original box.  With ``points`` = 5 and ``shrink`` = 1/2 the
    next box reaches one old grid spacing past the best point on each side,
    where the minimum of a smooth function lies once the grid resolves it.
    Stops when every width is below ``tol``.  Returns (x, f(x), evaluations);
    x is None when no grid point of the first level is feasible.
    """
    lo0 = np.asarray(lo, dtype=np.float64)
    hi0 = np.asarray(hi, dtype=np.float64)
    a, b = lo0.copy(), hi0.copy()
    best_x, best_f = None, np.inf
    evals = 0
    for _ in range(max_levels):
        axes = [np.linspace(a[j], b[j], points) for j in range(len(a))]
        for x in itertools.product(*axes):
            x = np.array(x)
            v = f(x)
            evals += 1
            if np.isfinite(v) and v < best_f:
                best_x, best_f = x, float(v)
        if best_x is None:
            return None, np.inf, evals
        if np.all(b - a < tol):
            break
        half = 0.5 * shrink * (b - a)
        a = np.maximum(lo0, best_x - half)
        b = np.minimum(hi0, best_x + half)
    return best_x, best_f, evals
