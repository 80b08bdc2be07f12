"""Divergence invariants of the oracle (Sec. 2.1-2.2, App. A).

* D*.B (eq. divstarb) is conserved by the update for any coefficients;
* D.E (eq. divE) is conserved in vacuum;
* the plain D.B is conserved only when eq.(beta) holds (beta_ij = delta_j);
* the FFT projection leaves D*.B at rounding level.
"""
import numpy as np

import synthetic as S
from oracle import fdtd as O

D = (1.0, 0.9, 1.2)


def _setup(seed, coeffs):
    f = S.uniform_fields((8, 9, 10), seed)
    B = O.project_div_star_free(f[3:], coeffs, D)
    return f[:3] + B


def test_projection_zeroes_div_star_b():
    beta, delta = S.extended_beta_delta(103)
    c = O.coeffs_from(beta, delta)
    f = _setup(103, c)
    assert np.abs(O.div_star_B(f[3:], c, D)).max() < 1e-13


def test_div_star_b_and_div_e_conserved():
    beta, delta = S.distinct_beta_delta(104)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c, D)
    f = S.uniform_fields((8, 9, 10), 105)          # not projected: any D*.B
    db0 = O.div_star_B(f[3:], c, D)
    de0 = O.div_E(f[:3], D)
    g = O.run(f, 60, c, dt, D)
    assert np.abs(O.div_star_B(g[3:], c, D) - db0).max() < 1e-12
    assert np.abs(O.div_E(g[:3], D) - de0).max() < 1e-12


def test_plain_div_b_drifts_without_eq_beta():
    beta, delta = S.extended_beta_delta(106)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c, D)
    f = _setup(106, c)
    g = O.run(f, 40, c, dt, D)
    drift = np.abs(O.div_B(g[3:], D) - O.div_B(f[3:], D)).max()
    assert drift > 1e-3


def test_plain_div_b_conserved_with_eq_beta():
    """eq.(beta): beta_ij = delta_j makes D.B a conserved quantity too."""
    delta = np.array([-0.02, -0.035, -0.01])
    beta = np.array([[delta[1], delta[2]], [delta[0], delta[2]], [delta[0], delta[1]]])
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c, D)
    f = S.uniform_fields((8, 9, 10), 107)
    g = O.run(f, 40, c, dt, D)
    drift = np.abs(O.div_B(g[3:], D) - O.div_B(f[3:], D)).max()
    assert drift < 1e-12


def test_current_term_continuity_and_sign():
    """App. A eq. update4-6 with the mu_0 J term (c = mu_0 = 1): D.D x B = 0
    makes D.E^{n+1} - D.E^n = -dt D.J exactly; with B = 0 a uniform current
    changes E by exactly -dt J; J = 0 is the vacuum update."""
    f = S.uniform_fields((8, 9, 10), 108)
    J = S.uniform_fields((8, 9, 10), 109)[:3]
    dt = 0.37
    E1 = O.ampere_current(f[:3], f[3:], J, dt, D)
    lhs = O.div_E(E1, D) - O.div_E(f[:3], D)
    rhs = -dt * O.div_E(J, D)
    assert np.abs(lhs - rhs).max() < 1e-13
    zero = [np.zeros_like(x) for x in J]
    assert all(np.array_equal(a, b) for a, b in zip(O.ampere_current(f[:3], f[3:], zero, dt, D),
                                                    O.ampere(f[:3], f[3:], dt, D)))
    Bz = [np.zeros_like(x) for x in J]
    Ju = [np.full_like(x, v) for x, v in zip(J, (0.5, -1.25, 2.0))]
    E2 = O.ampere_current(f[:3], Bz, Ju, dt, D)
    for a in range(3):
        assert np.abs(E2[a] - (f[a] - dt * Ju[a])).max() < 1e-15
