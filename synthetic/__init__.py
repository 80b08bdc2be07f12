"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and lays out initial fields; it holds none of
the solver's arithmetic (no stencil, no dispersion relation, no stability bound,
no eq.(alpha) completion).  Everything is generated in float64 with
``numpy.random.default_rng(seed)``; callers cast to the dtype they need.

Field layout used everywhere in this project: six separate arrays
``Ex, Ey, Ez, Bx, By, Bz``, each of shape ``(nz, ny, nx)`` (x fastest).  Integer
index ``(i, j, k)`` of a component sits at the staggered position of the Yee
cell (Sec. 2 and the update equations of App. A):

    Ex (i+1/2, j, k)      Bx (i, j+1/2, k+1/2)
    Ey (i, j+1/2, k)      By (i+1/2, j, k+1/2)
    Ez (i, j, k+1/2)      Bz (i+1/2, j+1/2, k)

E is at integer time levels, B at half-integer ones.
"""
from __future__ import annotations

import math

import numpy as np

# Half-cell offsets (in units of the cell size) of each component, in the
# order Ex, Ey, Ez, Bx, By, Bz, as (x, y, z) offsets.
STAGGER = (
    (0.5, 0.0, 0.0),
    (0.0, 0.5, 0.0),
    (0.0, 0.0, 0.5),
    (0.0, 0.5, 0.5),
    (0.5, 0.0, 0.5),
    (0.5, 0.5, 0.0),
)
COMPONENTS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def extended_beta_delta(seed: int, beta_max: float = 0.125,
                        delta_min: float = -0.05):
    """Draw one extended coefficient set's free parameters.

    Per axis a (independently): beta_ab = beta_ac ~ U[0, beta_max] and
    delta_a ~ U[delta_min, 0].  Returns ``(beta, delta)`` with ``beta`` of shape
    (3, 2) ordered as (xy, xz), (yx, yz), (zx, zy) and ``delta`` of shape (3,).
    alpha is not drawn: it follows from the consistency condition, which the
    caller applies.
    """
    g = rng(seed)
    b = g.uniform(0.0, beta_max, size=3)
    d = g.uniform(delta_min, 0.0, size=3)
    beta = np.stack([b, b], axis=1)
    return beta, d


def distinct_beta_delta(seed: int, scale: float = 0.06):
    """Draw six distinct betas and three distinct deltas (small magnitudes).

    Used where every coefficient must act differently (e.g. to catch a swapped
    beta_xy/beta_yx in a test).  Returns ``(beta[3,2], delta[3])``.
    """
    g = rng(seed)
    beta = g.uniform(0.1 * scale, scale, size=(3, 2))
    delta = g.uniform(-0.5 * scale, -0.05 * scale, size=3)
    return beta, delta


def mode_numbers(seed: int, lo: int = 1, hi: int = 8):
    """Three integer Fourier mode numbers, each uniform in {lo..hi}."""
    return tuple(int(v) for v in rng(seed).integers(lo, hi + 1, size=3))


def uniform_fields(shape, seed: int, amp: float = 1.0):
    """Six independent U(-amp, amp) arrays of shape ``(nz, ny, nx)``."""
    g = rng(seed)
    return [g.uniform(-amp, amp, size=tuple(shape)) for _ in range(6)]


def unit_vector(seed: int, n: int):
    """A seeded random unit vector of length n (float64)."""
    v = rng(seed).standard_normal(n)
    return v / np.linalg.norm(v)


def positions(shape, comp: int, spacing=(1.0, 1.0, 1.0)):
    """Physical coordinates (x, y, z) broadcastable to ``(nz, ny, nx)`` for a
    component's staggered sites."""
    nz, ny, nx = shape
    ox, oy, oz = STAGGER[comp]
    dx, dy, dz = spacing
    x = (np.arange(nx) + ox) * dx
    y = (np.arange(ny) + oy) * dy
    z = (np.arange(nz) + oz) * dz
    return x[None, None, :], y[None, :, None], z[:, None, None]


def gaussian_pulse(shape, dt: float, wavelength: float, waist: float,
                   duration: float, x0: float | None = None,
                   spacing=(1.0, 1.0, 1.0)):
    """Linearly polarised vacuum Gaussian pulse travelling along +x.

    E_y = exp(-(xi/L)^2) exp(-r^2/w0^2) sin(k0 xi),  xi = x - x0 - t,
    r^2 = (y-yc)^2 + (z-zc)^2, k0 = 2 pi / wavelength, and B_z = E_y (c = 1).
    ``waist`` is the 1/e field radius w0; ``duration`` is the intensity FWHM,
    so L = duration / sqrt(2 ln 2).  E is sampled at t = 0 and B at t = -dt/2,
    each at its own staggered sites.  The remaining components are zero.
    Returns the six float64 arrays.
    """
    nz, ny, nx = shape
    dx, dy, dz = spacing
    if x0 is None:
        x0 = 0.25 * nx * dx
    yc = 0.5 * ny * dy
    zc = 0.5 * nz * dz
    L = duration / math.sqrt(2.0 * math.log(2.0))
    k0 = 2.0 * math.pi / wavelength

    def profile(comp, t):
        x, y, z = positions(shape, comp, spacing)
        xi = x - x0 - t
        r2 = (y - yc) ** 2 + (z - zc) ** 2
        return np.exp(-(xi / L) ** 2) * np.exp(-r2 / waist ** 2) * np.sin(k0 * xi)

    f = [np.zeros(shape) for _ in range(6)]
    f[1] = np.broadcast_to(profile(1, 0.0), shape).copy()
    f[5] = np.broadcast_to(profile(5, -0.5 * dt), shape).copy()
    return f


def add_noise(fields, amp: float, seed: int):
    """Add U(-amp, amp) noise to every component (returns new arrays)."""
    g = rng(seed)
    return [f + g.uniform(-amp, amp, size=f.shape) for f in fields]


def box_edges(count: int, seed: int, choices=(32, 48, 64, 96, 128)):
    """``count`` boxes with each edge drawn iid from ``choices``.

    Returns a list of (nx, ny, nz) tuples.
    """
    g = rng(seed)
    e = g.choice(np.asarray(choices), size=(count, 3))
    return [tuple(int(v) for v in row) for row in e]
