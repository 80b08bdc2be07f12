"""Pins of the oracle's bounded search (oracle/search.py), which writes the
stored optima of Tables 1 and 3: known minima of smooth functions in a box,
in the interior, on a face, and on the boundary of an infeasible region
(+inf outside, approached from the feasible side)."""
import numpy as np

from oracle.search import refine_grid_search


def test_interior_minimum_of_a_rotated_quadratic():
    x0 = np.array([0.0731, -0.0412, 0.6123])
    A = np.array([[3.0, 0.8, -0.2], [0.8, 1.5, 0.3], [-0.2, 0.3, 2.0]])  # positive definite

    def f(x):
        d = x - x0
        return float(d @ A @ d) + 0.25

    x, v, n = refine_grid_search(f, [-0.125, -0.125, 0.1], [0.25, 0.125, 1.0], points=7, tol=1e-10)
    assert np.max(np.abs(x - x0)) < 1e-8
    assert abs(v - 0.25) < 1e-14
    assert n > 0


def test_minimum_on_a_face_of_the_box():
    # unconstrained minimum at x = 0.3 lies outside [-0.125, 0.125]: the box
    # minimum is the face x = 0.125, with y free at its own optimum
    def f(x):
        return (x[0] - 0.3) ** 2 + (x[1] + 0.0005) ** 2

    x, v, _ = refine_grid_search(f, [-0.125, -0.01], [0.125, 0.01], points=7, tol=1e-10)
    assert abs(x[0] - 0.125) < 1e-12
    assert abs(x[1] + 0.0005) < 1e-8
    assert abs(v - (0.175 ** 2)) < 1e-12


def test_minimum_on_an_infeasible_boundary_is_approached_from_inside():
    # f decreases towards x = 0.6868; beyond it the point is infeasible (+inf),
    # as an unstable time step is for the dispersion norm
    bound = 0.6868

    def f(x):
        return np.inf if x[0] > bound else (1.0 - x[0]) ** 2

    x, v, _ = refine_grid_search(f, [0.1], [1.0], points=9, tol=1e-11)
    assert x[0] <= bound and bound - x[0] < 1e-9
    assert np.isfinite(v)


def test_no_feasible_point_returns_none():
    x, v, _ = refine_grid_search(lambda x: np.inf, [0.0, 0.0], [1.0, 1.0])
    assert x is None and v == np.inf
