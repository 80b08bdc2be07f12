"""Dispersion norm f_w (Sec. 4, eq. norm) and stencil minimisation on the GPU.

``dispersion_norm`` evaluates f_w and its gradient for one stencil;
``Family`` describes an affine family of stencils (free parameters with
bounds, optional eq. alpha, a fixed time step or one tied to the stability
bound) and ``optimize_stencil`` minimises f_w over it (see include/xfdtd.h).
All arithmetic runs in the library.
"""
from __future__ import annotations

import ctypes

import torch

from . import _binding as B

NAMES = ["alpha_x", "beta_xy", "beta_xz", "delta_x", "alpha_y", "beta_yx", "beta_yz", "delta_y",
         "alpha_z", "beta_zx", "beta_zy", "delta_z", "dt"]
WEIGHTS = {"unit": B.XFDTD_WEIGHT_UNIT, "axis": B.XFDTD_WEIGHT_AXIS}


def _stream(device=None):
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def dispersion_norm(dt, coeffs, spacing=(1.0, 1.0, 1.0), dims=3, n=200, weight="unit", width=0.1,
                    device=None):
    """(f_w, gradient): gradient has 13 entries, d f_w / d coeffs then d f_w / d dt."""
    g = B.make_grid((1, 1, 1), spacing)
    f = ctypes.c_double()
    grad = (ctypes.c_double * 13)()
    B.check(B.lib().xfdtd_dispersion_norm(ctypes.byref(g), float(dt), B.dbl_array(coeffs, 12), int(dims),
                                          int(n), WEIGHTS[weight], float(width), ctypes.byref(f), grad,
                                          _stream(device)))
    return f.value, [grad[i] for i in range(13)]


class Family:
    """Affine family of stencils: quantity = base + sum_j map[quantity][j] x_j.

    ``base`` maps names of ``NAMES`` to values (default 0; set "dt" for a fixed
    time step).  ``param(lo, hi, **weights)`` adds a free parameter entering
    the named quantities with the given weights; ``dt_fraction(lo, hi)`` adds
    the parameter tau with dt = tau * (stability bound).  With
    ``alpha_rule`` the alphas follow eq. alpha.
    """

    def __init__(self, base=None, alpha_rule=True):
        self.base = [0.0] * 13
        for k, v in (base or {}).items():
            self.base[NAMES.index(k)] = float(v)
        self.alpha_rule = bool(alpha_rule)
        self.cols, self.lo, self.hi = [], [], []
        self.dt_param = -1

    def param(self, lo, hi, **weights):
        col = [0.0] * 13
        for k, v in weights.items():
            col[NAMES.index(k)] = float(v)
        self.cols.append(col)
        self.lo.append(float(lo))
        self.hi.append(float(hi))
        return self

    def dt_fraction(self, lo, hi):
        if self.dt_param >= 0:
            raise ValueError("only one time-step fraction")
        self.dt_param = len(self.cols)
        return self.param(lo, hi)

    def problem(self, dims, n, weight, width, starts, max_iter):
        m = len(self.cols)
        if not 1 <= m <= 8:
            raise ValueError("1 to 8 free parameters")
        p = B.StencilProblem()
        p.nparam = m
        p.alpha_rule = int(self.alpha_rule)
        p.dt_mode = 1 if self.dt_param >= 0 else 0
        p.dt_param = max(self.dt_param, 0)
        for r in range(13):
            p.base[r] = self.base[r]
            for j in range(m):
                p.map[r * 8 + j] = self.cols[j][r]
        for j in range(m):
            p.lo[j], p.hi[j] = self.lo[j], self.hi[j]
        p.dims, p.weight, p.width, p.n = int(dims), WEIGHTS[weight], float(width), int(n)
        p.starts, p.max_iter = int(starts), int(max_iter)
        return p


def optimize_stencil(family, spacing=(1.0, 1.0, 1.0), dims=2, n=1000, weight="unit", width=0.1, starts=3,
                     max_iter=200, device=None):
    """Minimise f_w over ``family``; returns dict(x, coeffs, dt, f, evals)."""
    p = family.problem(dims, n, weight, width, starts, max_iter)
    g = B.make_grid((1, 1, 1), spacing)
    x = (ctypes.c_double * 8)()
    c = (ctypes.c_double * 12)()
    dt, f, ev = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    B.check(B.lib().xfdtd_optimize_stencil(ctypes.byref(g), ctypes.byref(p), x, c, ctypes.byref(dt),
                                           ctypes.byref(f), ctypes.byref(ev), _stream(device)))
    return {"x": [x[j] for j in range(p.nparam)], "coeffs": [c[i] for i in range(12)], "dt": dt.value,
            "f": f.value, "evals": ev.value}
