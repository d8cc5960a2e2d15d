"""Pins of the Galilean continuity residual and of the optional current
correction (oracle, CPU)."""

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import diagnostics as dg
from oracle import pic
from oracle import spectral as sp
from workload import get_config, particles_for


def random_spectral(shape, rng, n=1):
    out = []
    for _ in range(n):
        a = sp.forward(rng.standard_normal(shape))
        a[sp.held_zero_mask(shape)] = 0
        out.append(a)
    return out


def test_continuity_residual_against_ode_solution():
    """The residual vanishes on the exact solution of the k-space continuity
    ODE d rho / dt = i (k.v_gal) rho - i k.J (J constant), propagated here
    with a matrix exponential of the augmented 2x2 system per mode."""
    rng = np.random.Generator(np.random.PCG64(81))
    for kdotv, dt in [(0.7, 1.0), (-2.3, 0.5), (1e-9, 1.0), (0.0, 0.8), (5.9, 1.0)]:
        rho0 = complex(rng.standard_normal(), rng.standard_normal())
        kJ = complex(rng.standard_normal(), rng.standard_normal())
        M = np.array([[1j * kdotv, -1j * kJ], [0.0, 0.0]])
        rho1 = (expm(M * dt) @ np.array([rho0, 1.0]))[0]
        k = (np.array([0.0]), np.array([0.0]), np.array([1.0]))
        v = (0.0, 0.0, kdotv)
        J = (np.array([0.0]), np.array([0.0]), np.array([kJ]))
        R = dg.continuity_residual(np.array([rho0]), np.array([rho1]), J, k, v, dt)
        assert abs(R[0]) <= 1e-13 * max(abs(rho0), abs(rho1), abs(kJ)), (kdotv, R)


@pytest.mark.parametrize("v_gal", [(0.0, 0.0, -0.995), (0.1, -0.2, 0.6), (0.0, 0.0, 0.0)])
def test_correction_satisfies_continuity_and_keeps_transverse_part(v_gal):
    shape, spacing, dt = (8, 8, 16), (1.0, 1.0, 0.7), 0.7
    rng = np.random.Generator(np.random.PCG64(82))
    J = tuple(random_spectral(shape, rng, 3))
    rho0, rho1 = random_spectral(shape, rng, 2)
    k = sp.wavevectors(shape, spacing)
    mask = sp.held_zero_mask(shape)
    Jc = sp.galilean_current_correction(J, rho0, rho1, k, v_gal, dt, mask)
    R = dg.continuity_residual(rho0, rho1, Jc, k, v_gal, dt)
    R[mask] = 0
    assert np.max(np.abs(R)) <= 1e-12 * np.max(np.abs(rho1))
    # transverse part unchanged: k x J_c = k x J
    kxJ, kxJc = sp.cross(k, J), sp.cross(k, Jc)
    for a in range(3):
        d = np.where(mask, 0, kxJc[a] - kxJ[a])
        assert np.max(np.abs(d)) <= 1e-12 * np.max(np.abs(kxJ[a]))
    # correcting twice changes nothing more
    Jcc = sp.galilean_current_correction(Jc, rho0, rho1, k, v_gal, dt, mask)
    for a in range(3):
        assert np.max(np.abs(Jcc[a] - Jc[a])) <= 1e-12 * np.max(np.abs(Jc[a]))


def test_correction_at_v_gal_zero_is_the_standard_form():
    """v_gal = 0: k.J_c = i (rho^{n+1} - rho^n) / dt."""
    shape, spacing, dt = (8, 16, 8), (0.8, 1.0, 1.1), 0.9
    rng = np.random.Generator(np.random.PCG64(83))
    J = tuple(random_spectral(shape, rng, 3))
    rho0, rho1 = random_spectral(shape, rng, 2)
    k = sp.wavevectors(shape, spacing)
    mask = sp.held_zero_mask(shape)
    Jc = sp.galilean_current_correction(J, rho0, rho1, k, (0.0, 0.0, 0.0), dt, mask)
    kJc = k[0] * Jc[0] + k[1] * Jc[1] + k[2] * Jc[2]
    expect = 1j * (rho1 - rho0) / dt
    expect[mask] = 0
    assert np.max(np.abs(kJc - expect)) <= 1e-12 * np.max(np.abs(expect))


def test_gauss_error_evolves_exactly_with_correction():
    """With corrected currents the Gauss error G = i k.E - rho is multiplied
    by theta^2 C every step, for a hot plasma that crosses cells; without
    the correction the continuity residual adds to it."""
    cfg = get_config("c1_cic_fp64").with_(shape=(8, 8, 16), u_th=0.4, galilean=True)
    p = particles_for(cfg)
    out = {}
    for corr in (True, False):
        g = pic.Grid(cfg.shape, cfg.spacing, cfg.dt, cfg.order)
        sim = pic.Simulation(g, pic.Species(cfg.q, cfg.m, cfg.w), cfg.v_gal(),
                             current_correction=corr)
        st = sim.initial_state(p["x"], p["u"])
        G = dg.gauss_residual(st.E_hat, st.rho_hat, sim.k)
        worst = 0.0
        for _ in range(5):
            st = sim.step(st)
            G1 = dg.gauss_residual(st.E_hat, st.rho_hat, sim.k)
            expect = sim.coef["c_EE"] * G
            d = np.where(sim.mask, 0, G1 - expect)
            worst = max(worst, float(np.max(np.abs(d)) / np.max(np.abs(st.rho_hat))))
            G = G1
        out[corr] = worst
    assert out[True] <= 1e-12
    assert out[False] >= 1e-6
