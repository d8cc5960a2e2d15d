"""Pins of the quasi-cylindrical (azimuthal-mode) oracle.

The forward Hankel transform reproduces the analytic Fourier-Bessel
coefficients of r^m exp(-r^2 / 2 s^2); the forward and backward transforms
of a mode invert each other; and the spectral mapping of a mode to the
Cartesian wavevector at azimuth 0 reproduces the curl and divergence of
explicit Bessel-mode fields computed by finite differences in 3D Cartesian
coordinates (pinning the mode convention, the +-combinations, their Hankel
orders and the factors of i).  The update itself is the Cartesian update,
pinned elsewhere, at that wavevector.
"""

import numpy as np
import pytest
from scipy import special

from oracle import cylindrical as cy
from oracle import spectral as sp


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_forward_transform_gives_fourier_bessel_coefficients(m):
    """f(r) = r^m exp(-r^2 / 2 s^2) has Hankel transform s^(2m+2) k^m
    exp(-k^2 s^2 / 2); on [0, R] its Fourier-Bessel coefficients are
    2 H(k_i) / (R^2 J_{m+1}(alpha_i)^2) up to the tail beyond R."""
    nr, dr = 64, 0.25
    R = nr * dr
    s = R / 8
    r = cy.radial_grid(nr, dr)
    f = r ** m * np.exp(-r ** 2 / (2 * s * s))
    c = cy.forward_matrix(m, m, nr, dr) @ f
    alpha = special.jn_zeros(m, nr)
    k = alpha / R
    ref = 2 * s ** (2 * m + 2) * k ** m * np.exp(-k * k * s * s / 2) / (
        R * R * special.jv(m + 1, alpha) ** 2)
    assert np.max(np.abs(c - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("m", [0, 1, 3])
def test_mode_transforms_invert(m):
    rng = np.random.default_rng(70 + m)
    nz, nr, dr, dz = 16, 24, 0.5, 0.7
    G = tuple(rng.standard_normal((nz, nr)) + 1j * rng.standard_normal((nz, nr))
              for _ in range(3))
    F = cy.from_spectral(G, m, dr, dz)
    G2 = cy.to_spectral(F, m, dr, dz)
    for a, b in zip(G, G2):
        assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(a))
    f = cy.scalar_from_spectral(G[0], m, dr, dz)
    assert np.max(np.abs(cy.scalar_to_spectral(f, m, dr, dz) - G[0])) <= 1e-10 * np.max(
        np.abs(G[0]))


def _mode_field(G, m, kr, kz):
    """Cartesian components, as functions of (x, y, z), of the mode-m field
    with one spectral component (k_r, k_z) and amplitudes (G_+, G_-, G_z)."""
    gp, gm, gz = G

    def F(x, y, z):
        r = np.hypot(x, y)
        th = np.arctan2(y, x)
        ez = np.exp(1j * kz * z)
        a = gp * special.jv(m + 1, kr * r) * np.exp(1j * (m + 1) * th)
        b = gm * special.jv(m - 1, kr * r) * np.exp(1j * (m - 1) * th)
        c = gz * special.jv(m, kr * r) * np.exp(1j * m * th)
        return np.array([(a + b) * ez, -1j * (a - b) * ez, c * ez])
    return F


@pytest.mark.parametrize("m", [0, 1, 2])
def test_mapping_reproduces_curl_and_divergence(m):
    rng = np.random.default_rng(80 + m)
    kr, kz = 1.3, -0.7
    G = tuple(complex(*rng.standard_normal(2)) for _ in range(3))
    F = _mode_field(G, m, kr, kz)
    # spectral curl and divergence through the Cartesian wavevector (k_r, 0, k_z)
    Fc = cy.to_cartesian(G)
    k = (kr, 0.0, kz)
    curl_c = tuple(1j * c for c in sp.cross(k, Fc))
    C = _mode_field(cy.from_cartesian(curl_c), m, kr, kz)
    div = 1j * (k[0] * Fc[0] + k[2] * Fc[2])
    h = 1e-5
    for _ in range(12):
        x, y, z = rng.uniform(-2.0, 2.0, 3)
        d = [(F(*(np.array([x, y, z]) + h * e)) - F(*(np.array([x, y, z]) - h * e))) / (2 * h)
             for e in np.eye(3)]
        # d[a][c] = dF_c / dx_a
        curl = np.array([d[1][2] - d[2][1], d[2][0] - d[0][2], d[0][1] - d[1][0]])
        got = C(x, y, z)
        assert np.max(np.abs(got - curl)) <= 1e-7 * (1 + np.max(np.abs(curl)))
        num_div = d[0][0] + d[1][1] + d[2][2]
        r = np.hypot(x, y)
        th = np.arctan2(y, x)
        spec_div = div * special.jv(m, kr * r) * np.exp(1j * m * th) * np.exp(1j * kz * z)
        assert abs(num_div - spec_div) <= 1e-7 * (1 + abs(num_div))


def test_mode_update_keeps_gauss_law():
    """From i k.E = rho^n and rho^{n+1} following the Galilean continuity
    equation, the mode update gives i k.E' = rho^{n+1} (through the
    mapping), as the Cartesian update does."""
    rng = np.random.default_rng(90)
    m, nz, nr, dr, dz, dt, v = 1, 8, 12, 0.5, 0.5, 0.4, -0.9
    kz = cy.axis_kz(nz, dz)[:, None] * np.ones((1, nr))
    kr = np.ones((nz, 1)) * cy.spectral_kr(m, nr, dr)[None, :]
    cplx = lambda: rng.standard_normal((nz, nr)) + 1j * rng.standard_normal((nz, nr))
    E = tuple(cplx() for _ in range(3))
    B = tuple(cplx() for _ in range(3))
    J = tuple(cplx() for _ in range(3))
    Ec, Jc = cy.to_cartesian(E), cy.to_cartesian(J)
    rho0 = 1j * (kr * Ec[0] + kz * Ec[2])
    kJ = kr * Jc[0] + kz * Jc[2]
    th2 = np.exp(1j * kz * v * dt)
    rho1 = th2 * rho0 + np.where(kz == 0, -1j * dt * kJ,
                                 (1 - th2) * kJ / np.where(kz == 0, 1.0, kz * v))
    En, _ = cy.mode_update(E, B, J, rho0, rho1, m, nr, dr, nz, dz, v, dt)
    Enc = cy.to_cartesian(En)
    g = 1j * (kr * Enc[0] + kz * Enc[2]) - rho1
    live = ~cy.held_mask(nz, nr)
    assert np.max(np.abs(g[live])) <= 1e-11 * np.max(np.abs(rho1))
