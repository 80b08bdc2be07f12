"""Seeded synthetic workloads of the benchmark configurations (shared by the
tests and the golden-value script; inputs only, no solver arithmetic beyond the
oracle's stability bound used to pick dt)."""
from __future__ import annotations

import synthetic as S
from oracle import fdtd as O

C2_SHAPE = (256, 256, 512)  # (nz, ny, nx): x is the propagation axis


def c2_inputs(shape=C2_SHAPE):
    """512x256x256 box: extended set (seed 201), Gaussian pulse along x with
    wavelength 16, waist 32, duration 40 cells, x0 = nx/4, plus U(-1e-3, 1e-3)
    noise (seed 202); dt = 0.95 x the stability bound."""
    beta, delta = S.extended_beta_delta(201)
    c = O.coeffs_from(beta, delta)
    sp = (1.0, 1.0, 1.0)
    dt = 0.95 * O.cfl_dt(c, sp)
    f = S.gaussian_pulse(shape, dt, wavelength=16.0, waist=32.0, duration=40.0)
    f = S.add_noise(f, 1e-3, 202)
    return f, c, dt, sp
