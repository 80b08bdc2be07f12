"""Pins of the oracle's dispersion relation, stability bound and norm.

* Table 1's time steps against the exact stability bound (eq. constraints);
  the Yee bound in closed form; KKT maximum = dense-grid maximum;
* App. B: the corrected closed form of F; the sign printed there contradicts
  Table 1 (min.1 would be unstable at its own printed time step);
* Table 2's phase-velocity extremes; group velocity = numerical d omega/dk;
* App. B: omega depends on the symmetric part of beta-hat only;
* Tables 1 and 3: dispersion norms f_w (eq. norm).
"""
import os

import numpy as np
import pytest

import synthetic as S
from oracle import fdtd as O
from tests import _pins as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense_F_range(c, d=(1.0, 1.0, 1.0), n=61, dims=3):
    th = np.linspace(0.0, np.pi, n)
    if dims == 3:
        g = np.stack(np.meshgrid(th / d[0], th / d[1], th / d[2], indexing="ij"), -1)
    else:
        g = np.stack(np.meshgrid(th / d[0], th / d[1], [0.0], indexing="ij"), -1)
    F = O.dispersion_rhs(g, c, d)
    return F.min(), F.max()


def test_yee_cfl_closed_form():
    for d in [(1, 1, 1), (1.0, 0.5, 2.0), (0.3, 0.3, 1.1)]:
        exp = 1.0 / np.sqrt(sum(1.0 / v ** 2 for v in d))
        assert abs(O.cfl_dt(O.yee_coeffs(), d) - exp) < 1e-14


@pytest.mark.parametrize("seed", range(12))
def test_kkt_extrema_match_dense_grid(seed):
    g = S.rng(900 + seed)
    beta = g.uniform(-0.05, 0.2, (3, 2))
    delta = g.uniform(-0.2, 0.05, 3)
    c = O.coeffs_from(beta, delta)
    d = tuple(g.uniform(0.5, 2.0, 3))
    fmin, fmax = O.stability_range(c, d)
    gmin, gmax = dense_F_range(c, d, n=81)
    # the dense grid can only under-estimate the true max / over-estimate the min
    assert fmax >= gmax - 1e-12 and fmin <= gmin + 1e-12
    assert fmax - gmax < 2e-3 * abs(fmax) + 1e-12
    assert gmin - fmin < 2e-3 * max(abs(fmax), 1.0)


def test_extended_draws_are_stable_and_max_not_always_at_corner():
    off_corner = 0
    for seed in range(40):
        beta, delta = S.extended_beta_delta(1000 + seed)
        c = O.coeffs_from(beta, delta)
        fmin, fmax = O.stability_range(c)
        assert fmin >= -1e-15
        corner = float(O.dispersion_rhs(np.array([np.pi, np.pi, np.pi]), c))
        if fmax > corner * (1 + 1e-9):
            off_corner += 1
    assert off_corner > 0


def test_table1_time_steps_against_stability_bound():
    rows = P.golden_rows(os.path.join(GOLD, "table1_norms.txt"))
    for name, fw, dts, b, dxv, dyv, eqb in rows:
        dt = P.parse_dt(dts)
        c = P.coeffs_2d(float(b), float(dxv), float(dyv))
        cfl = O.cfl_dt(c, dims=2)
        # every printed time step is stable (rounding of the printed
        # coefficients allows 1e-3 relative)
        assert dt <= cfl * (1 + 1e-3), (name, dt, cfl)
        if name == "Yee":
            assert abs(cfl - 1 / np.sqrt(2)) < 1e-14
        if name == "NDFX":
            # Sec. 5: NDFX is stable at c dt = dx exactly
            assert abs(cfl - 1.0) < 1e-12
        if name in ("Lehe", "min.1", "min.2"):
            # these sit within 0.2% of their bound
            assert cfl < dt * 1.002, (name, dt, cfl)


def appb_F(k, c, d, sign_beta):
    """App. B's closed form: sum s_i^2 (1 - 4 dx_i^2 delta_i s_i^2)
    + sign_beta * 4 sum_{i != j} dx_j^2 beta_ij s_i^2 s_j^2."""
    k = np.asarray(k, dtype=float)
    s2 = [(np.sin(0.5 * k[..., a] * d[a]) / d[a]) ** 2 for a in range(3)]
    F = 0.0
    for i in range(3):
        F = F + s2[i] * (1 - 4 * d[i] ** 2 * c[4 * i + 3] * s2[i])
        for j in range(3):
            if j == i:
                continue
            bij = c[4 * i + 1 + O.TRANSVERSE[i].index(j)]
            F = F + sign_beta * 4 * d[j] ** 2 * bij * s2[i] * s2[j]
    return F


def test_appendix_b_form_and_its_sign():
    beta, delta = S.distinct_beta_delta(77)
    c = O.coeffs_from(beta, delta)
    d = (1.0, 0.7, 1.4)
    k = S.rng(78).uniform(0, np.pi, (200, 3)) / np.asarray(d)
    F = O.dispersion_rhs(k, c, d)
    # with eq.(alpha), the App. B form holds with a minus sign on the beta term
    assert np.abs(appb_F(k, c, d, -1.0) - F).max() < 1e-14
    # the printed plus sign would make Table 1's min.1 unstable at its dt
    c1 = P.coeffs_2d(0.110, -0.125, -0.125)
    th = np.linspace(0, np.pi, 401)
    g = np.stack(np.meshgrid(th, th, [0.0], indexing="ij"), -1)
    printed_cfl = 1 / np.sqrt(appb_F(g, c1, (1, 1, 1), +1.0).max())
    assert printed_cfl < 0.686 < O.cfl_dt(c1, dims=2)


def vph_extremes(c, dt, n=801):
    th = np.linspace(0, np.pi, n)
    g = np.stack(np.meshgrid(th, th, [0.0], indexing="ij"), -1).reshape(-1, 3)[1:]
    _, vph, _ = O.dispersion(g, dt, c)
    return np.nanmin(vph), np.nanmax(vph)


def test_table2_phase_velocity_extremes():
    t1 = {r[0]: r for r in P.golden_rows(os.path.join(GOLD, "table1_norms.txt"))}
    for name, lo, hi in P.golden_rows(os.path.join(GOLD, "table2_vph.txt")):
        _, fw, dts, b, dxv, dyv, _ = t1[name]
        c = P.coeffs_2d(float(b), float(dxv), float(dyv))
        vmin, vmax = vph_extremes(c, P.parse_dt(dts))
        # two printed decimals of a quantity computed from coefficients that
        # are themselves printed to 2-3 digits
        assert abs(vmin - float(lo)) < 0.012, (name, vmin, lo)
        assert abs(vmax - float(hi)) < 0.012, (name, vmax, hi)


def test_group_velocity_is_derivative_of_omega():
    beta, delta = S.distinct_beta_delta(55)
    c = O.coeffs_from(beta, delta)
    d = (1.0, 0.6, 1.3)
    dt = 0.95 * O.cfl_dt(c, d)
    k = S.rng(56).uniform(0.05, 0.95, (300, 3)) * np.pi / np.asarray(d)
    _, _, vg = O.dispersion(k, dt, c, d)
    h = 1e-6
    for a in range(3):
        kp, km = k.copy(), k.copy()
        kp[:, a] += h
        km[:, a] -= h
        fd = (O.omega(kp, dt, c, d) - O.omega(km, dt, c, d)) / (2 * h)
        assert np.abs(fd - vg[:, a]).max() < 1e-8


def test_continuum_limit():
    beta, delta = S.distinct_beta_delta(57)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c)
    k = np.array([[1e-4, 2e-4, -1e-4], [3e-4, 0, 0]])
    w, vph, vg = O.dispersion(k, dt, c)
    assert np.abs(vph - 1).max() < 1e-6
    assert np.abs(np.linalg.norm(vg, axis=-1) - 1).max() < 1e-6


def test_omega_depends_on_symmetric_beta_hat_only():
    """App. B: only the symmetric part of beta_hat_ij = dx_j^2 beta_ij enters."""
    d = np.array([1.0, 0.8, 1.5])
    beta, delta = S.distinct_beta_delta(58)
    c = O.coeffs_from(beta, delta)
    bh = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            if i != j:
                bh[i, j] = d[j] ** 2 * c[4 * i + 1 + O.TRANSVERSE[i].index(j)]
    # add an antisymmetric part to beta_hat, keep alpha fixed
    anti = np.array([[0, 0.01, -0.02], [-0.01, 0, 0.015], [0.02, -0.015, 0]])
    c2 = c.copy()
    for i in range(3):
        for j in range(3):
            if i != j:
                c2[4 * i + 1 + O.TRANSVERSE[i].index(j)] = (bh[i, j] + anti[i, j]) / d[j] ** 2
    # alpha must follow eq.(alpha) for the App. B rewrite: recompute it
    for i in range(3):
        c2[4 * i] = 1 - 2 * c2[4 * i + 1] - 2 * c2[4 * i + 2] - 3 * c2[4 * i + 3]
    # the antisymmetric change shifts alpha, which App. B absorbs; compare F
    k = S.rng(59).uniform(0, np.pi, (100, 3)) / d
    F1 = appb_F(k, c, d, -1.0)
    F2 = appb_F(k, c2, d, -1.0)
    assert np.abs(F1 - F2).max() < 1e-14
    assert np.abs(O.dispersion_rhs(k, c2, d) - F2).max() < 1e-14
    assert np.abs(O.dispersion_rhs(k, c2, d) - O.dispersion_rhs(k, c, d)).max() < 1e-14
    # and a symmetric change does move it
    c3 = c.copy()
    c3[1] += 0.01
    c3[0] -= 0.02
    assert np.abs(O.dispersion_rhs(k, c3, d) - F1).max() > 1e-4


def test_table1_norms():
    for name, fw, dts, b, dxv, dyv, _ in P.golden_rows(os.path.join(GOLD, "table1_norms.txt")):
        c = P.coeffs_2d(float(b), float(dxv), float(dyv))
        got = O.norm_fw(P.parse_dt(dts), c, dims=2, n=600)
        # printed to 2 digits, from coefficients printed to 2-3 digits; every
        # row reproduces within 4% (0.08 -> 5%: one printed digit)
        tol = 0.05 if float(fw) < 0.1 else 0.04
        assert abs(got - float(fw)) <= tol * float(fw) + 1e-3, (name, got, fw)


def test_table3_weighted_norms_reproducible_rows():
    """eq. norm_x_axis weight.  Yee, NDFX, Cowan and min.6 reproduce; the Lehe
    and min.5 rows do not follow from their printed coefficients (a factor of
    about ten) and are recorded as unpinned."""
    w = lambda k: np.exp(-(k[..., 1] / 0.1) ** 2)
    got = {}
    for name, fw, dts, b, dxv, dyv in P.golden_rows(os.path.join(GOLD, "table3_weighted.txt")):
        c = P.coeffs_2d(float(b), float(dxv), float(dyv))
        got[name] = (O.norm_fw(P.parse_dt(dts), c, dims=2, n=1200, weight=w), float(fw))
    for name in ("Yee", "NDFX"):
        v, ref = got[name]
        assert abs(v - ref) < 0.12 * ref, (name, v, ref)
    for name in ("Cowan", "min.6"):
        v, ref = got[name]
        assert 0.5 * ref < v < 1.5 * ref, (name, v, ref)
    # ranking printed in Table 3 among the reproducible rows
    assert got["NDFX"][0] < got["min.6"][0] < got["Cowan"][0] < got["Yee"][0]
