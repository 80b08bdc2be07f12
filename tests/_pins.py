"""Shared helpers for the oracle pin tests (CPU only).

Each ``pin_*`` function checks the oracle against something the paper or the
mathematics fixes and returns the measured error; the tests assert bounds on
them, and the mutation tests assert that a planted mistake breaks at least one.
"""
from __future__ import annotations

import numpy as np

import synthetic as S
from oracle import fdtd as O


def golden_rows(path):
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def parse_dt(tok):
    return 0.95 / np.sqrt(2.0) if tok == "0.95/sqrt2" else float(tok)


def coeffs_2d(beta, delta_x, delta_y):
    """3D 12-vector of a 2D scheme: beta_xy = beta_yx = beta, no z coupling,
    alpha from eq.(alpha)."""
    return O.coeffs_from([[beta, 0.0], [beta, 0.0], [0.0, 0.0]], [delta_x, delta_y, 0.0])


def one_step_matrix(shape, coeffs, dt, d=(1.0, 1.0, 1.0)):
    """Columns = oracle step applied to every unit basis vector of the state."""
    nz, ny, nx = shape
    N = nx * ny * nz
    M = np.zeros((6 * N, 6 * N))
    for col in range(6 * N):
        f = [np.zeros(shape) for _ in range(6)]
        f[col // N].reshape(-1)[col % N] = 1.0
        g = O.step(f, coeffs, dt, d)
        M[:, col] = np.concatenate([x.reshape(-1) for x in g])
    return M


def expected_spectrum(shape, coeffs, dt, d=(1.0, 1.0, 1.0)):
    """Per discrete k: e^{+-i omega dt} twice each plus two static modes (1)."""
    nz, ny, nx = shape
    angles = []
    for mz in range(nz):
        for my in range(ny):
            for mx in range(nx):
                k = np.array([2 * np.pi * mx / (nx * d[0]), 2 * np.pi * my / (ny * d[1]),
                              2 * np.pi * mz / (nz * d[2])])
                w = float(O.omega(k, dt, coeffs, d))
                angles += [w * dt, w * dt, -w * dt, -w * dt, 0.0, 0.0]
    return np.sort(np.asarray(angles))


def pin_spectrum(shape=(4, 5, 6), seed=11, coeffs=None, d=(1.0, 1.0, 1.0)):
    """Max |angle error| and max ||lambda| - 1| of the one-step map's spectrum
    versus the closed-form dispersion relation (Sec. 3)."""
    if coeffs is None:
        beta, delta = S.distinct_beta_delta(seed)
        coeffs = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(coeffs, d)
    M = one_step_matrix(shape, coeffs, dt, d)
    lam = np.linalg.eigvals(M)
    got = np.sort(np.angle(lam))
    exp = expected_spectrum(shape, coeffs, dt, d)
    return float(np.max(np.abs(got - exp))), float(np.max(np.abs(np.abs(lam) - 1.0)))


def rel_l2(a, b):
    num = np.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b)))
    den = np.sqrt(sum(float(np.sum(y ** 2)) for y in b))
    return num / den


def pin_plane_wave(shape=(16, 16, 16), nsteps=60, seed=102, coeff_seed=7, d=(1.0, 1.0, 1.0)):
    """Relative L2 error of the oracle after nsteps against the exact eigenmode."""
    beta, delta = S.distinct_beta_delta(coeff_seed)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c, d)
    nz, ny, nx = shape
    modes = S.mode_numbers(seed, 1, max(1, min(nx, ny, nz) // 4))
    f0, *_ = O.plane_wave(shape, modes, dt, c, d)
    got = O.run(f0, nsteps, c, dt, d)
    exp = O.plane_wave_at(shape, modes, dt, c, nsteps, d)
    return rel_l2(got, exp)


def pin_wave_equation(shape=(6, 7, 8), seed=21, d=(1.0, 1.0, 1.0)):
    """Residual of the discrete wave equations of App. A:
    D_t^2 B = Delta* B - D (D*.B) and D_t^2 E = Delta* E - D*(D.E)."""
    beta, delta = S.distinct_beta_delta(seed)
    c = O.coeffs_from(beta, delta)
    dt = 0.9 * O.cfl_dt(c, d)
    f = S.uniform_fields(shape, seed + 1)
    f1 = O.step(f, c, dt, d)
    f2 = O.step(f1, c, dt, d)
    res = 0.0
    B0, B1, B2 = f[3:], f1[3:], f2[3:]
    divs = O.div_star_B(B1, c, d)
    for a in range(3):
        lhs = (B2[a] - 2 * B1[a] + B0[a]) / dt ** 2
        rhs = O.laplacian_star(B1[a], c, d) - O.back_diff(divs, a, d)
        res = max(res, float(np.abs(lhs - rhs).max()))
    E0, E1, E2 = f[:3], f1[:3], f2[:3]
    rho = O.div_E(E1, d)
    for a in range(3):
        lhs = (E2[a] - 2 * E1[a] + E0[a]) / dt ** 2
        rhs = O.laplacian_star(E1[a], c, d) - O.ext_diff(rho, a, c, d)
        res = max(res, float(np.abs(lhs - rhs).max()))
    return res
