"""Pins of the oracle's leapfrog step against what the paper fixes.

* brute force: the spectrum of the explicit one-step matrix equals the
  closed-form dispersion relation of Sec. 3 (all 12 coefficients distinct);
* closed form: an exact discrete eigenmode is advanced to rounding level;
* App. A: the discrete wave equations with the extended Laplacian hold;
* special cases: the Yee limit and the 1D dispersion-free step c dt = dx;
* the plain-C oracle agrees with the numpy oracle.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import fdtd as O
import oracle
from tests import _pins as P


def test_one_step_spectrum_matches_dispersion_relation():
    ang, mod = P.pin_spectrum((4, 5, 6), seed=11)
    assert ang < 1e-12, ang
    assert mod < 1e-12, mod


def test_one_step_spectrum_anisotropic_spacing():
    beta, delta = S.distinct_beta_delta(12)
    c = O.coeffs_from(beta, delta)
    ang, mod = P.pin_spectrum((3, 4, 5), coeffs=c, d=(1.0, 1.7, 0.6))
    assert ang < 1e-12 and mod < 1e-12, (ang, mod)


def test_plane_wave_eigenmode():
    err = P.pin_plane_wave((16, 16, 16), nsteps=60)
    assert err < 1e-12, err


def test_plane_wave_eigenmode_yee_and_anisotropic():
    c = O.yee_coeffs()
    d = (1.0, 0.5, 2.0)
    dt = 0.95 * O.cfl_dt(c, d)
    f0, *_ = O.plane_wave((8, 12, 10), (2, 3, 1), dt, c, d)
    got = O.run(f0, 40, c, dt, d)
    exp = O.plane_wave_at((8, 12, 10), (2, 3, 1), dt, c, 40, d)
    assert P.rel_l2(got, exp) < 1e-12


@pytest.mark.parametrize("nsteps", [0, 1, 37])
def test_plane_wave_sample_equals_the_stepped_mode(nsteps):
    """The sampled closed form (used where the full field would not fit) at
    flat storage indices equals the oracle's own leapfrog run of the mode,
    on a non-cubic grid with anisotropic spacing and six distinct betas, for
    every component: pins its index decoding, staggering and time levels."""
    shape, modes, d = (6, 5, 7), (2, 1, 3), (1.0, 1.7, 0.8)
    beta, delta = S.distinct_beta_delta(14)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c, d)
    f0, *_ = O.plane_wave(shape, modes, dt, c, d)
    got = O.run(f0, nsteps, c, dt, d) if nsteps else f0
    params = O.plane_wave_params(shape, modes, dt, c, d)
    idx = S.rng(15).integers(0, np.prod(shape), 64)
    idx = np.concatenate([idx, [0, np.prod(shape) - 1, shape[2] - 1, shape[2] * shape[1]]])
    for comp in range(6):
        exp = O.plane_wave_sample(shape, params, comp, idx, nsteps, dt, d)
        ref = got[comp].reshape(-1)[idx]
        assert np.abs(exp - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), comp
        full = O.plane_wave_at(shape, modes, dt, c, nsteps, d)[comp].reshape(-1)[idx]
        assert np.abs(exp - full).max() < 1e-13, comp  # same closed form, phases summed in another order


def test_discrete_wave_equations_app_a():
    assert P.pin_wave_equation() < 1e-10


def test_yee_limit_textbook_update():
    """beta = delta = 0, alpha = 1 gives the textbook Yee curl: D*_a = D_a."""
    c = O.yee_coeffs()
    d = (1.0, 1.3, 0.7)
    X = S.uniform_fields((5, 6, 7), 3)[0]
    for a in range(3):
        assert np.abs(O.ext_diff(X, a, c, d) - O.fwd_diff(X, a, d)).max() < 1e-14


def test_1d_yee_magic_time_step():
    """Sec. 3: in 1D the Yee scheme is dispersion-free at c dt = dx; a discrete
    right-moving wave shifts exactly one cell per step."""
    n = 32
    g = S.rng(5)
    ey = g.uniform(-1, 1, n)
    f = [np.zeros((1, 1, n)) for _ in range(6)]
    f[1][0, 0, :] = ey
    # a wave f(x - t) has Bz = Ey; Bz sits half a cell up and half a step
    # back, so B_z^{-1/2}[i] = f(i + 1) = Ey^0[i + 1]
    f[5][0, 0, :] = np.roll(ey, -1)
    out = O.run(f, 10, O.yee_coeffs(), 1.0)
    assert np.abs(out[1][0, 0] - np.roll(ey, 10)).max() < 1e-13


def test_c_oracle_matches_numpy_oracle():
    beta, delta = S.distinct_beta_delta(31)
    c = O.coeffs_from(beta, delta)
    d = (1.0, 0.8, 1.25)
    dt = 0.95 * O.cfl_dt(c, d)
    f = S.uniform_fields((9, 7, 11), 32)
    a = O.run(f, 12, c, dt, d)
    b = oracle.c_run(f, 12, c, dt, d)
    assert P.rel_l2(b, a) < 1e-14


def test_c_oracle_step_at_matches_full_step():
    beta, delta = S.distinct_beta_delta(33)
    c = O.coeffs_from(beta, delta)
    dt = 0.9 * O.cfl_dt(c)
    f = S.uniform_fields((5, 6, 7), 34)
    idx = np.arange(0, 210, 5)
    full = O.step(f, c, dt, (1.0, 1.0, 1.0))
    exp = np.stack([x.reshape(-1)[idx] for x in full], axis=1)
    got = oracle.c_step_at(f, idx, c, dt)
    assert np.abs(got - exp).max() < 1e-14


@pytest.mark.parametrize("shape", [(1, 1, 5), (1, 4, 1), (3, 1, 1), (2, 2, 2)])
def test_degenerate_grids_wrap(shape):
    """Axes of length 1 or 2: the wide taps wrap onto the same cells; the
    eigenmode of a k = 0 axis is constant along it."""
    beta, delta = S.distinct_beta_delta(41)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c)
    f = S.uniform_fields(shape, 42)
    a = O.run(f, 5, c, dt)
    b = oracle.c_run(f, 5, c, dt)
    assert P.rel_l2(b, a) < 1e-13
