"""The oracle's adjoint: scatter-form transposes of the two updates.

Pinned by the dot-product identity <M x, y> = <x, M^T y> against the
gather-form forward step, and by central finite differences of a loss
through the forward oracle (coefficients and initial E).
"""
import numpy as np

import synthetic as S
from oracle import fdtd as O

D = (1.0, 0.8, 1.3)


def _inner(a, b):
    return sum(float(np.sum(x * y)) for x, y in zip(a, b))


def test_dot_product_identity_one_step():
    beta, delta = S.distinct_beta_delta(201)
    c = O.coeffs_from(beta, delta)
    dt = 0.95 * O.cfl_dt(c, D)
    x = S.uniform_fields((5, 6, 7), 202)
    y = S.uniform_fields((5, 6, 7), 203)
    Mx = O.step(x, c, dt, D)
    MTy, _ = O.adjoint_step(y, x[:3], c, dt, D)
    lhs, rhs = _inner(Mx, y), _inner(x, MTy)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def _loss_setup(seed):
    beta, delta = S.distinct_beta_delta(seed)
    c = O.coeffs_from(beta, delta)
    dt = 0.9 * O.cfl_dt(c, D)
    f0 = S.uniform_fields((4, 5, 6), seed + 1)
    target = S.uniform_fields((4, 5, 6), seed + 2)
    return c, dt, f0, target


def _loss(fN, target):
    # half the squared misfit of E on one probe plane (x-index 2)
    return 0.5 * sum(float(np.sum((fN[a][:, :, 2] - target[a][:, :, 2]) ** 2)) for a in range(3))


def _grad_out(target):
    def g(fN):
        out = [np.zeros_like(x) for x in fN]
        for a in range(3):
            out[a][:, :, 2] = fN[a][:, :, 2] - target[a][:, :, 2]
        return out
    return g


def test_coefficient_gradient_matches_finite_differences():
    c, dt, f0, target = _loss_setup(210)
    n = 15
    _, gf, gc = O.run_with_adjoint(f0, n, c, dt, D, _grad_out(target))
    h = 1e-6
    for j in range(12):
        cp, cm = c.copy(), c.copy()
        cp[j] += h
        cm[j] -= h
        fd = (_loss(O.run(f0, n, cp, dt, D), target) - _loss(O.run(f0, n, cm, dt, D), target)) / (2 * h)
        assert abs(fd - gc[j]) <= 1e-7 * max(abs(fd), 1e-3 * np.abs(gc).max()), (j, fd, gc[j])


def test_initial_field_gradient_matches_finite_differences():
    c, dt, f0, target = _loss_setup(220)
    n = 12
    _, gf, _ = O.run_with_adjoint(f0, n, c, dt, D, _grad_out(target))
    u = [S.unit_vector(221 + a, f0[a].size).reshape(f0[a].shape) for a in range(6)]
    h = 1e-6
    fp = [f0[a] + h * u[a] for a in range(6)]
    fm = [f0[a] - h * u[a] for a in range(6)]
    fd = (_loss(O.run(fp, n, c, dt, D), target) - _loss(O.run(fm, n, c, dt, D), target)) / (2 * h)
    ad = _inner(gf, u)
    assert abs(fd - ad) < 1e-7 * abs(fd)
    # sampled single entries of dL/dE0
    g = S.rng(222)
    for _ in range(8):
        comp = int(g.integers(0, 3))
        p = tuple(int(g.integers(0, s)) for s in f0[0].shape)
        fp = [x.copy() for x in f0]
        fm = [x.copy() for x in f0]
        fp[comp][p] += h
        fm[comp][p] -= h
        fd = (_loss(O.run(fp, n, c, dt, D), target) - _loss(O.run(fm, n, c, dt, D), target)) / (2 * h)
        assert abs(fd - gf[comp][p]) <= 1e-7 * max(abs(fd), 1e-3 * np.abs(gf[comp]).max())
