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
