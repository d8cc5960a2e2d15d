"""Pins of the finite-order (modified-k) option of the oracle.

The weights of the centered first-derivative stencils are checked against
the linear moment conditions that define them (solved here) and against
the printed textbook values of orders 2, 4 and 6; the symbol [k] against
the stencil applied in real space; its error against the truncation-error
law of centered differences; its limit against the exact k.  A full step
with a finite-order solve keeps the drifting Coulomb field of a plasma at
rest in the Galilean frame, and with the current correction keeps the
discrete Gauss law i[k].E = rho from a consistent start.
"""

from math import factorial

import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import pic
from oracle import spectral as sp
from workload import get_config


@pytest.mark.parametrize("M", range(1, 9))
def test_weights_solve_the_moment_conditions(M):
    """f_{i+l} - f_{i-l} = 2 sum_j (l d)^(2j+1) f^(2j+1) / (2j+1)!: the stencil
    is the derivative when sum_l a_l 2 l = 1 and sum_l a_l l^(2j+1) = 0 for
    j = 1 .. M-1."""
    l = np.arange(1, M + 1, dtype=np.float64)
    A = np.array([2.0 * l ** (2 * j + 1) for j in range(M)])
    rhs = np.zeros(M)
    rhs[0] = 1.0
    a = np.linalg.solve(A, rhs)
    assert np.allclose(sp.centered_difference_weights(M), a, rtol=1e-9, atol=1e-12)


def test_weights_of_orders_two_four_six():
    # (f1 - f-1) / 2;  (8 (f1 - f-1) - (f2 - f-2)) / 12;
    # (45 (f1 - f-1) - 9 (f2 - f-2) + (f3 - f-3)) / 60
    assert sp.centered_difference_weights(1) == [0.5]
    assert np.allclose(sp.centered_difference_weights(2), [8 / 12, -1 / 12], rtol=0, atol=1e-16)
    assert np.allclose(sp.centered_difference_weights(3), [45 / 60, -9 / 60, 1 / 60],
                       rtol=0, atol=1e-16)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("order", [2, 4, 6, 10])
def test_symbol_is_the_real_space_stencil(axis, order):
    """Multiplying the spectrum by i [k] and transforming back applies the
    stencil on the periodic grid (sign, factor and FFT index order)."""
    rng = np.random.default_rng(40 + order + axis)
    shape, spacing = (16, 8, 12), (0.5, 1.0, 0.8)
    f = rng.standard_normal(shape)
    stencil = [0, 0, 0]
    stencil[axis] = order
    k = sp.wavevectors(shape, spacing, tuple(stencil))
    spectral = sp.inverse(1j * k[axis] * sp.forward(f))
    a = sp.centered_difference_weights(order // 2)
    real = sum(al * (np.roll(f, -l, axis) - np.roll(f, l, axis))
               for l, al in enumerate(a, start=1)) / spacing[axis]
    assert np.max(np.abs(spectral - real)) <= 1e-13 * np.max(np.abs(real))


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_error_follows_the_truncation_law(M):
    """[k] / k = 1 - (M!)^2 / (2M+1)! (k d)^(2M) + O((k d)^(2M+2)): the
    centered difference of order 2M lags by its truncation error."""
    d = 0.7
    n = 2048
    k = sp.axis_wavenumbers(n, d)[1:40]           # k d from 0.003 to 0.12
    got = sp.modified_wavenumbers(n, d, 2 * M)[1:40] / k - 1.0
    lead = -factorial(M) ** 2 / factorial(2 * M + 1) * (k * d) ** (2 * M)
    sel = np.abs(lead) > 1e-11                    # well above rounding
    assert sel.sum() >= 5
    assert np.allclose(got[sel] / lead[sel], 1.0, rtol=0, atol=0.01)


def test_spectral_limit_and_positivity():
    n, d = 256, 1.0
    k = sp.axis_wavenumbers(n, d)
    low = (np.abs(k) * d <= np.pi / 2) & (k != 0)
    prev = np.inf
    for M in (1, 2, 4, 8, 16, 32):
        km = sp.modified_wavenumbers(n, d, 2 * M)
        err = np.max(np.abs(km[low] / k[low] - 1.0))
        assert err < prev
        prev = err
        # odd in k, and of the sign of k off k = 0 and the Nyquist index
        inner = (k != 0) & (np.abs(k) * d < np.pi * (1 - 1e-12))
        assert np.all(km[inner] * np.sign(k[inner]) > 0)
        assert np.allclose(km[1:n // 2], -km[n - 1:n // 2:-1], rtol=0, atol=1e-14)
    assert prev <= 1e-10
    assert np.array_equal(sp.modified_wavenumbers(n, d, 0), k)
    with pytest.raises(ValueError):
        sp.modified_wavenumbers(n, d, 3)


def _sim(cfg, stencil, correction=False):
    g = pic.Grid(cfg.shape, cfg.spacing, cfg.dt, cfg.order)
    return pic.Simulation(g, pic.Species(cfg.q, cfg.m, cfg.w), cfg.v_gal(),
                          current_correction=correction, stencil=stencil)


def _cold_start(cfg, stencil):
    """Cold electrons at v = v_gal (at rest on the Galilean grid) and the
    drifting Coulomb field of their charge, built with the symbol [k]."""
    sim = _sim(cfg, stencil)
    rng = np.random.Generator(np.random.PCG64(91))
    n = 3 * cfg.n_cells
    L = np.array(cfg.shape) * np.array(cfg.spacing)
    x = rng.random((n, 3)) * L
    u = np.zeros((n, 3))
    u[:, 2] = cfg.drift_u()
    rho = sp.forward(sim.deposit_charge(x))
    rho[sim.mask] = 0
    k, v = sim.k, np.asarray(cfg.v_gal())
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    kv = k[0] * v[0] + k[1] * v[1] + k[2] * v[2]
    phi = np.where(sim.mask, 0, rho / np.where(sim.mask, 1.0, k2 - kv * kv))
    E = [sp.inverse(-1j * k[a] * phi + 1j * kv * v[a] * phi) for a in range(3)]
    kxv = sp.cross(k, v)
    B = [sp.inverse(1j * kxv[a] * phi) for a in range(3)]
    return sim, x, u, E, B


def test_drifting_coulomb_field_is_a_fixed_point_of_the_finite_order_step():
    cfg = get_config("c1_cic_fp64").with_(shape=(8, 8, 16), ppc=3)
    sim, x, u, E, B = _cold_start(cfg, (4, 6, 8))
    st0 = sim.initial_state(x, u, E, B)
    st1 = sim.step(st0)
    assert np.array_equal(st1.x, st0.x)
    scale = max(np.max(np.abs(a)) for a in st0.E_hat + st0.B_hat)
    err = max(np.max(np.abs(a - b)) for a, b in zip(st1.E_hat + st1.B_hat,
                                                     st0.E_hat + st0.B_hat))
    assert err <= 1e-12 * scale
    # with the exact k in the coefficients but [k] in the update the field
    # is no longer stationary: the step does use one vector throughout
    exact = _sim(cfg, (0, 0, 0))
    E1, _ = sp.galilean_psatd_update(st0.E_hat, st0.B_hat, st1.J_hat, st0.rho_hat,
                                     st1.rho_new_hat, sim.k, exact.coef, sim.mask)
    assert max(np.max(np.abs(a - b)) for a, b in zip(E1, st0.E_hat)) > 1e-3 * scale


def test_gauss_law_kept_with_correction_and_stencil():
    """Thermal electrons with the current correction: i[k].E^n = rho^n holds
    after every step from E^0 = the Coulomb field of rho^0."""
    cfg = get_config("c1_cic_fp64").with_(shape=(8, 8, 16), ppc=3)
    _, x, u, E, B = _cold_start(cfg, (2, 4, 16))
    sim = _sim(cfg, (2, 4, 16), correction=True)
    rng = np.random.Generator(np.random.PCG64(92))
    u = u + 0.3 * rng.standard_normal(u.shape)
    st = sim.initial_state(x, u, E, B)
    scale = np.max(np.abs(st.rho_hat))
    assert np.max(np.abs(dg.gauss_residual(st.E_hat, st.rho_hat, sim.k))) <= 1e-12 * scale
    for _ in range(3):
        st = sim.step(st)
        g = dg.gauss_residual(st.E_hat, st.rho_hat, sim.k)
        assert np.max(np.abs(g)) <= 1e-11 * scale
