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


C5A_SHAPE = (256, 256, 1024)


def c5a_inputs(shape=C5A_SHAPE):
    """1024x256x256 box: extended set (seed 601), Gaussian pulse along x with
    wavelength 20, waist 40, duration 50 cells (the 512x256x256 pulse scaled),
    x0 = nx/4, no noise; dt = 0.95 x the stability bound."""
    beta, delta = S.extended_beta_delta(601)
    c = O.coeffs_from(beta, delta)
    sp = (1.0, 1.0, 1.0)
    dt = 0.95 * O.cfl_dt(c, sp)
    f = S.gaussian_pulse(shape, dt, wavelength=20.0, waist=40.0, duration=50.0)
    return f, c, dt, sp


def pulse_target_loss_setup(shape, steps, wavelength, waist, duration, x0, dt):
    """Probe plane and target of the field-misfit loss.

    The target is the initial continuum pulse rigidly translated by steps*dt
    along x (the analytic vacuum pulse, c = 1), sampled at the E sites; the
    probe plane is the y-z plane at x-index round(x0 + steps*dt) mod nx.
    Returns (probe_index, [Ex*, Ey*, Ez*] on that plane, each (nz, ny)).
    """
    nz, ny, nx = shape
    shift = x0 + steps * dt
    xc = shift % nx
    tgt = S.gaussian_pulse(shape, dt, wavelength=wavelength, waist=waist, duration=duration, x0=xc)
    xp = int(round(shift)) % nx
    return xp, [t[:, :, xp].copy() for t in tgt[:3]]


def c4_inputs(shape=(128, 128, 128), steps=200, scale=1.0):
    """128^3 box: extended set (seed 501), Gaussian pulse along x with
    wavelength 12, waist 24, duration 30 cells (the 512x256x256 pulse scaled
    to wavelength 12), x0 = nx/4, plus 1e-3 noise (seed 502); dt = 0.95 x
    the stability bound.  ``scale`` shrinks waist and duration for smaller
    copies of the box (the 24^3 copy uses waist 4.5, duration 7.5)."""
    beta, delta = S.extended_beta_delta(501)
    c = O.coeffs_from(beta, delta)
    sp = (1.0, 1.0, 1.0)
    dt = 0.95 * O.cfl_dt(c, sp)
    nz, ny, nx = shape
    x0 = 0.25 * nx
    lam, w0, dur = 12.0, 24.0 * scale, 30.0 * scale
    if scale != 1.0:
        w0, dur = 4.5, 7.5
    f = S.gaussian_pulse(shape, dt, wavelength=lam, waist=w0, duration=dur, x0=x0)
    f = S.add_noise(f, 1e-3, 502)
    xp, tgt = pulse_target_loss_setup(shape, steps, lam, w0, dur, x0, dt)
    return f, c, dt, sp, xp, tgt


def probe_loss(fields, xp, tgt):
    """L = 1/2 sum over the probe plane and the three E components of the
    squared misfit (numpy)."""
    import numpy as np
    return 0.5 * sum(float(np.sum((fields[a][:, :, xp] - tgt[a]) ** 2)) for a in range(3))


def c3_boxes(count=64):
    """64 boxes with edges iid in {32, 48, 64, 96, 128} (seed 301); box b has
    its own extended set (seed 302 + b), U(-1, 1) fields (seed 400 + b) and
    dt = 0.95 x its stability bound.  Returns [(shape, fields, coeffs, dt)]."""
    out = []
    for b, (nx, ny, nz) in enumerate(S.box_edges(count, 301)):
        beta, delta = S.extended_beta_delta(302 + b)
        c = O.coeffs_from(beta, delta)
        dt = 0.95 * O.cfl_dt(c)
        shape = (nz, ny, nx)
        out.append((shape, S.uniform_fields(shape, 400 + b), c, dt))
    return out


def c5_boxes(count=16, shape=(96, 96, 96), steps=300):
    """Batched coefficient tuning: ``count`` boxes of 96^3 holding the same
    pulse (wavelength 12, waist 16, duration 16 cells, centred at x0 = nx/2,
    plus 1e-3 noise, seed 521), box b with its own extended set (seed
    520 + 10 b) and dt = 0.95 x its stability bound; the loss of box b is the
    probe misfit against its own translated target.  Returns
    [(fields, coeffs, dt, sp, xp, tgt)]."""
    nz, ny, nx = shape
    lam, w0, dur, x0 = 12.0, 16.0, 16.0, 0.5 * nx
    sp = (1.0, 1.0, 1.0)
    out = []
    for b in range(count):
        beta, delta = S.extended_beta_delta(520 + 10 * b)
        c = O.coeffs_from(beta, delta)
        dt = 0.95 * O.cfl_dt(c, sp)
        f = S.gaussian_pulse(shape, dt, wavelength=lam, waist=w0, duration=dur, x0=x0)
        f = S.add_noise(f, 1e-3, 521)
        xp, tgt = pulse_target_loss_setup(shape, steps, lam, w0, dur, x0, dt)
        out.append((f, c, dt, sp, xp, tgt))
    return out

