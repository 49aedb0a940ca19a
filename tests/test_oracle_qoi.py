"""Pins of the oracle's quantity-of-interest studies (Sec. 3.6) against a
closed form, its derivative, the symmetries the discrete problems inherit
from the grid, and exact quadrature of bilinear fields."""
import math

import numpy as np
import pytest

from oracle import qoi as Q
from paper_2204_06083_amd import workloads as W


def _exact(a):
    """u = C (x^2/a^2 + y^2 a^2 - 1) with Lap u = 3 (the paper's source) gives
    C = 3 / (2 (a^2 + a^-2)) and u(0, 0) = -C."""
    a = np.asarray(a, dtype=np.float64)
    return -3.0 / (2.0 * (a * a + 1.0 / (a * a)))


def _dexact(a):
    a = np.asarray(a, dtype=np.float64)
    return 3.0 * (2.0 * a - 2.0 / a ** 3) / (2.0 * (a * a + 1.0 / (a * a)) ** 2)


def _center(g):
    return lambda u: Q.node_value(g, u, (0.0, 0.0))


def test_trapezoid_weights_integrate_bilinear_fields_exactly():
    g = W.qoi_rotated_grid()
    w = W.qoi_rectangle_weights(g)
    X, Y = g.mesh()
    assert abs(Q.weighted_sum(w, np.ones(g.shape)) - 2.0) <= 1e-12
    assert abs(Q.weighted_sum(w, X)) <= 1e-12
    assert abs(Q.weighted_sum(w, (X + 1.0) * (Y + 0.5)) - 1.0) <= 1e-12
    assert abs(Q.weighted_sum(w, X * X) - 2.0 / 3.0) <= 2.0 * g.h ** 2   # trapezoid error of x^2
    assert not np.any(w[np.abs(Y) > 0.5 + 1e-9]) and not np.any(w[np.abs(X) > 1.0 + 1e-9])
    with pytest.raises(ValueError):
        W.qoi_rectangle_weights(g, rect=((-1.0, 1.005), (-0.5, 0.5)))


def test_ellipse_qoi_converges_to_the_closed_form_at_second_order():
    avals = (0.5, 0.8, 1.0, 1.25, 1.7, 2.0)
    errs = []
    for n in (128, 256):
        g = W.qoi_ellipse_grid(n)
        f = np.full(g.shape, W.QOI_SOURCE)
        q = Q.sweep(g, [W.psi_area_ellipse(g, a) for a in avals], f, _center(g))
        errs.append(np.abs(q - _exact(avals)).max())
    assert errs[1] <= 1e-3
    assert errs[0] / errs[1] >= 3.0, errs


def test_ellipse_qoi_symmetry_minimum_and_derivative():
    """Q(a) = Q(1/a) (the discrete problem of 1/a is the transpose of that of
    a), the minimum at a = 1, and the central-difference derivative of the
    sweep against the closed-form derivative."""
    g = W.qoi_ellipse_grid(256)
    f = np.full(g.shape, W.QOI_SOURCE)
    a = W.qoi_ellipse_params(61)
    step = a[1] - a[0]
    q = Q.sweep(g, [W.psi_area_ellipse(g, x) for x in a], f, _center(g))
    for i, j in ((0, 60), (12, 30), (5, 44)):
        assert abs(a[i] * a[j] - 1.0) <= 1e-12
        assert abs(q[i] - q[j]) <= 1e-12 * abs(q[i])
    assert a[np.argmin(q)] == 1.0
    d = Q.central_differences(q, step)
    assert np.abs(d - Q.central_differences(_exact(a), step)).max() <= 5e-3
    assert np.abs(d - _dexact(a[1:-1])).max() <= 1e-2
    # the derivative changes sign once, at a = 1
    sgn = np.sign(d)
    assert np.all(sgn[a[1:-1] < 0.99] < 0) and np.all(sgn[a[1:-1] > 1.01] > 0)


def test_rotated_ellipse_qoi_symmetries():
    """On the paper's 501^2 grid of [-5, 5]^2, reflecting y maps the ellipse of
    angle theta to that of -theta and leaves the rectangle and the grid in
    place; theta + pi is the same ellipse.  (Angles where grid nodes lie on
    the ellipse are avoided: their classification is decided by rounding.)"""
    g = W.qoi_rotated_grid()
    f = np.full(g.shape, W.QOI_SOURCE)
    w = W.qoi_rectangle_weights(g)
    th = [0.3, -0.3, 0.3 + math.pi, math.pi - 0.3, 1.1]
    q = Q.sweep(g, [W.psi_rotated_ellipse(g, t) for t in th], f, lambda u: Q.weighted_sum(w, u))
    for i in (1, 2, 3):
        assert abs(q[i] - q[0]) <= 1e-10 * abs(q[0]), (q[i], q[0])
    assert abs(q[4] - q[0]) > 1e-3 * abs(q[0])        # and a different angle differs
    # the solution is negative inside (maximum principle for Lap u = 3 > 0)
    assert np.all(q < 0)
