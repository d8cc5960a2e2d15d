"""Pins of the oracle's shapes, deposition, gather and push.

Checked against scipy's B-spline basis (a library routine), conservation
and symmetry properties, and closed-form solutions of the Boris rotation.
"""

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import particles as pt


@pytest.mark.parametrize("order", [1, 3])
def test_shape_matches_scipy_cardinal_bspline(order):
    """Weights equal the cardinal B-spline of degree `order` centred on each node."""
    knots = np.arange(order + 2) - (order + 1) / 2.0
    basis = BSpline.basis_element(knots, extrapolate=False)
    delta = np.linspace(0.0, 0.999, 37)
    w, rel = pt.bspline_weights(delta, order)
    for j, r in enumerate(rel):
        dist = delta - r          # particle position relative to node
        ref = np.nan_to_num(basis(dist))
        np.testing.assert_allclose(w[:, j], ref, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=0, atol=1e-15)


def test_cubic_weights_at_known_offsets():
    w, _ = pt.bspline_weights(np.array([0.0, 0.5]), 3)
    np.testing.assert_allclose(w[0], [1 / 6, 4 / 6, 1 / 6, 0.0], atol=1e-16)
    np.testing.assert_allclose(w[1], [1 / 48, 23 / 48, 23 / 48, 1 / 48], atol=1e-16)


@pytest.mark.parametrize("order", [1, 3])
def test_deposit_charge_and_shift(order):
    rng = np.random.default_rng(1)
    shape, spacing = (6, 5, 8), (1.0, 0.5, 2.0)
    L = np.array(shape) * np.array(spacing)
    x = rng.random((50, 3)) * L
    vals = rng.standard_normal(50)
    rho = pt.deposit(x, vals, shape, spacing, order)[0]
    assert abs(rho.sum() - vals.sum()) <= 1e-13
    # shifting every particle by one cell shifts the deposit by one node
    xs = pt.wrap(x + np.array([spacing[0], 0, 0]), L)
    rhos = pt.deposit(xs, vals, shape, spacing, order)[0]
    np.testing.assert_allclose(rhos, np.roll(rho, 1, axis=0), atol=1e-13)


def test_single_particle_cic_deposit():
    shape, spacing = (4, 4, 4), (1.0, 1.0, 1.0)
    x = np.array([[1.25, 2.5, 3.75]])       # wraps in z to node 0
    rho = pt.deposit(x, np.ones(1), shape, spacing, 1)[0]
    expect = np.zeros(shape)
    for i, wi in ((1, 0.75), (2, 0.25)):
        for j, wj in ((2, 0.5), (3, 0.5)):
            for k, wk in ((3, 0.25), (0, 0.75)):
                expect[i, j, k] += wi * wj * wk
    np.testing.assert_allclose(rho, expect, atol=1e-16)


@pytest.mark.parametrize("order", [1, 3])
def test_uniform_velocity_current_is_rho_v(order):
    rng = np.random.default_rng(2)
    shape, spacing = (4, 6, 8), (1.0, 1.0, 1.0)
    x = rng.random((40, 3)) * np.array(shape)
    v = np.array([0.1, -0.3, 0.7])
    J = pt.deposit(x, np.tile(v, (40, 1)), shape, spacing, order)
    rho = pt.deposit(x, np.ones(40), shape, spacing, order)[0]
    for a in range(3):
        np.testing.assert_allclose(J[a], rho * v[a], atol=1e-14)


@pytest.mark.parametrize("order", [1, 3])
def test_gather_is_adjoint_of_deposit(order):
    rng = np.random.default_rng(3)
    shape, spacing = (5, 6, 7), (1.0, 1.0, 1.0)
    x = rng.random((30, 3)) * np.array(shape)
    F = rng.standard_normal(shape)
    g = pt.gather([F], x, shape, spacing, order)[0]
    for p in range(30):
        d = pt.deposit(x[p:p + 1], np.ones(1), shape, spacing, order)[0]
        assert abs(np.sum(d * F) - g[p]) <= 1e-13


@pytest.mark.parametrize("order", [1, 3])
def test_gather_reproduces_constant_and_linear_fields(order):
    shape, spacing = (16, 16, 16), (1.0, 1.0, 1.0)
    gx = np.arange(16.0)
    lin = np.broadcast_to(gx[:, None, None] * 0.3 + 2.0, shape)
    rng = np.random.default_rng(4)
    x = 4.0 + 8.0 * rng.random((25, 3))        # away from the periodic seam
    const = pt.gather([np.full(shape, 1.5)], x, shape, spacing, order)[0]
    np.testing.assert_allclose(const, 1.5, atol=1e-14)
    got = pt.gather([lin], x, shape, spacing, order)[0]
    np.testing.assert_allclose(got, x[:, 0] * 0.3 + 2.0, atol=1e-13)


def test_boris_uniform_magnetic_field_rotation():
    """|u| is conserved; the rotation angle per step is 2 atan(|q| B dt / (2 m gamma))."""
    q, m, dt = -1.0, 1.0, 0.7
    u = np.array([[3.0, 0.0, 1.5]])
    Bz = 2.0
    gamma = np.sqrt(1 + np.sum(u * u))
    un = pt.boris_push(u, np.zeros((1, 3)), np.array([[0.0, 0.0, Bz]]), q, m, dt)
    assert abs(np.linalg.norm(un) - np.linalg.norm(u)) <= 1e-14
    angle = np.arctan2(un[0, 1], un[0, 0]) - np.arctan2(u[0, 1], u[0, 0])
    expect = 2 * np.arctan(abs(q) * Bz * dt / (2 * m * gamma))
    # an electron (q < 0) rotates counter-clockwise about +z
    assert abs(angle - expect) <= 1e-14
    assert un[0, 2] == u[0, 2]


def test_boris_uniform_electric_field():
    q, m, dt = -1.0, 2.0, 0.3
    u = np.array([[0.1, 0.2, -5.0]])
    E = np.array([[0.5, -1.0, 2.0]])
    un = pt.boris_push(u, E, np.zeros((1, 3)), q, m, dt)
    np.testing.assert_allclose(un, u + q * E * dt / m, atol=1e-15)


def test_static_on_grid_when_v_equals_v_gal():
    rng = np.random.default_rng(6)
    uz = -np.sqrt(30.0 ** 2 - 1)
    u = np.tile([0.0, 0.0, uz], (20, 1))
    v = pt.lab_velocity(u)
    v_gal = (0.0, 0.0, uz / np.sqrt(1 + uz * uz))
    x = rng.random((20, 3)) * 8
    x2 = pt.half_move(pt.half_move(x, v, v_gal, 1.0, np.array([8.0] * 3)), v, v_gal, 1.0,
                      np.array([8.0] * 3))
    assert np.array_equal(x, x2)


def test_wrap_stays_in_box():
    L = np.array([4.0, 4.0, 4.0])
    x = np.array([[-1e-17, 4.0, 8.5]])
    w = pt.wrap(x, L)
    assert np.all(w >= 0) and np.all(w < L)
