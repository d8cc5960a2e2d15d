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
    kr = np.ones((nz, 1)) * cy.update_kr(m, nr, dr)[None, :]
    cplx = lambda: rng.standard_normal((nz, nr)) + 1j * rng.standard_normal((nz, nr))
    E = cy.hold(tuple(cplx() for _ in range(3)), m)
    B = cy.hold(tuple(cplx() for _ in range(3)), m)
    J = cy.hold(tuple(cplx() for _ in range(3)), m)
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


# ---- particles: deposition and gather by azimuthal mode ----------------------

def _spline(order):
    """scipy's centred cardinal B-spline of the order (node spacing 1)."""
    from scipy.interpolate import BSpline
    b = BSpline.basis_element(np.arange(order + 2) - (order + 1) / 2, extrapolate=False)
    return lambda x: np.nan_to_num(b(x))


@pytest.mark.parametrize("order", [1, 3])
def test_node_volumes_are_the_folded_shape_integrals(order):
    nr, dr, dz = 6, 0.7, 0.9
    B = _spline(order)
    r = np.linspace(0.0, (nr + 2) * dr, 400001)
    for j in range(nr):
        # node j's weight plus that of its mirror -j-1 across the axis
        w = B(r / dr - (j + 0.5)) + B(r / dr + (j + 0.5))
        ref = 2 * np.pi * dz * np.trapezoid(w * r, r)
        assert abs(cy.node_volumes(nr, dr, dz, order)[j] - ref) <= 1e-9 * ref, j


def _cyl_particles(rng, n, rmax, lz):
    r = rmax * np.sqrt(rng.uniform(0, 1, n))
    th = rng.uniform(0, 2 * np.pi, n)
    r[:5] = [0.0, 0.01, 0.2, 0.34, 0.5]   # on and near the axis
    return r * np.cos(th), r * np.sin(th), rng.uniform(0, lz, n)


@pytest.mark.parametrize("order", [1, 3])
def test_charge_sums_exactly_up_to_the_axis(order):
    rng = np.random.default_rng(100)
    nz, nr, dz, dr = 8, 6, 0.5, 0.7
    x, y, z = _cyl_particles(rng, 2000, (nr - 2) * dr, nz * dz)
    qw = rng.uniform(0.5, 1.5, len(x))
    g0 = cy.deposit_mode(x, y, z, qw, 0, "scalar", nr, dr, nz, dz, order)
    vol = cy.node_volumes(nr, dr, dz, order)
    assert abs(np.sum(vol[None, :] * g0.real) - qw.sum()) <= 1e-12 * qw.sum()
    assert np.max(np.abs(g0.imag)) == 0.0


@pytest.mark.parametrize("order", [1, 3])
def test_uniform_fields_are_gathered_exactly_everywhere(order):
    """A uniform Cartesian field is mode 0 (F_z) plus mode 1 with
    (F_r, F_theta) = (F_x - i F_y, F_y + i F_x); linear weights reproduce it
    exactly at every point, on and near the axis too, only if the axis fold
    signs, the sign of theta and the rotation back to x, y are right."""
    rng = np.random.default_rng(101)
    nz, nr, dz, dr = 8, 5, 0.5, 0.7
    x, y, z = _cyl_particles(rng, 500, (nr - 2) * dr, nz * dz)
    F = np.array([0.3, -1.2, 0.7])
    one = np.ones((nz, nr))
    G = [(0 * one + 0j, 0 * one + 0j, F[2] * one + 0j),
         ((F[0] - 1j * F[1]) * one, (F[1] + 1j * F[0]) * one, 0 * one + 0j)]
    got = cy.gather_vector(G, x, y, z, nr, dr, nz, dz, order)
    assert np.max(np.abs(got - F[None, :])) <= 1e-14


@pytest.mark.parametrize("order", [1, 3])
def test_deposit_and_gather_are_adjoint(order):
    """sum_p q w v.E(x_p) = Re sum_m (1/c_m) sum_nodes V g_m conj(D_m) over
    the three components, for random mode fields g and the deposited
    currents D: ties the deposit's c_m, angle sign, volumes and fold to
    the gather's."""
    rng = np.random.default_rng(102)
    nz, nr, nm, dz, dr = 8, 6, 3, 0.5, 0.7
    x, y, z = _cyl_particles(rng, 300, (nr - 0.5) * dr, nz * dz)
    v = rng.standard_normal((len(x), 3))
    qw = 0.8
    cplx = lambda: rng.standard_normal((nz, nr)) + 1j * rng.standard_normal((nz, nr))
    G = [(cplx(), cplx(), cplx()) for _ in range(nm)]
    lhs = qw * np.sum(v * cy.gather_vector(G, x, y, z, nr, dr, nz, dz, order))
    D = cy.deposit_current(x, y, z, v, qw, nm, nr, dr, nz, dz, order)
    vol = cy.node_volumes(nr, dr, dz, order)[None, :]
    c = lambda m: 1.0 if m == 0 else 2.0
    rhs = sum(np.real(np.sum(vol * G[m][a] * np.conj(D[m][a]))) / c(m)
              for m in range(nm) for a in range(3))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(v)) * qw


@pytest.mark.parametrize("order", [1, 3])
def test_mode_content_of_particles(order):
    nz, nr, dz, dr = 8, 6, 0.5, 0.7
    # one particle off the axis: g_m = c_m exp(-i m theta) g_0 node by node
    th = 0.9
    x, y, z = np.array([2.1 * np.cos(th)]), np.array([2.1 * np.sin(th)]), np.array([1.3])
    g = [cy.deposit_mode(x, y, z, np.ones(1), m, "scalar", nr, dr, nz, dz, order)
         for m in range(4)]
    for m in range(1, 4):
        assert np.allclose(g[m], 2.0 * np.exp(-1j * m * th) * g[0], rtol=0, atol=1e-15)
    # three particles at equal angles on a ring: modes 1 and 2 vanish
    ths = th + 2 * np.pi * np.arange(3) / 3
    x, y, z = 2.1 * np.cos(ths), 2.1 * np.sin(ths), np.full(3, 1.3)
    g = [cy.deposit_mode(x, y, z, np.ones(3), m, "scalar", nr, dr, nz, dz, order)
         for m in range(4)]
    for m in (1, 2):
        assert np.max(np.abs(g[m])) <= 1e-14 * np.max(np.abs(g[0]))
    assert np.max(np.abs(g[3])) >= 0.5 * np.max(np.abs(g[0]))


def test_angular_density_modulation_is_its_mode_one_content():
    """Particles at N equal angles on one ring, weighted 1 + a cos(theta),
    describe the density rho_0 (1 + a cos theta), whose stored mode 1 is
    rho_0 a (the physical field is Re sum g_m exp(i m theta)): g_1 / g_0 = a
    at every node, and a phase shift of the modulation rotates g_1."""
    nz, nr, dz, dr = 8, 6, 0.5, 0.7
    a, phi, N = 0.37, 0.6, 7
    th = 2 * np.pi * np.arange(N) / N + 0.2
    x, y, z = 2.3 * np.cos(th), 2.3 * np.sin(th), np.full(N, 1.1)
    w = 1.0 + a * np.cos(th - phi)
    g0 = cy.deposit_mode(x, y, z, w, 0, "scalar", nr, dr, nz, dz)
    g1 = cy.deposit_mode(x, y, z, w, 1, "scalar", nr, dr, nz, dz)
    live = np.abs(g0) > 0
    assert np.allclose(g1[live] / g0[live], a * np.exp(-1j * phi), rtol=0, atol=1e-14)


def _drifting_column(galilean, steps, seed=1, nz=64, nr=12, n=20000, gamma=10.0, rp=8.0,
                     nmodes=2):
    rng = np.random.default_rng(seed)
    r = rp * np.sqrt(rng.uniform(0, 1, n))
    th = rng.uniform(0, 2 * np.pi, n)
    x = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(0, nz, n)], 1)
    uz = -np.sqrt(gamma * gamma - 1.0)
    u = np.zeros((n, 3))
    u[:, 2] = uz
    vz = uz / np.sqrt(1.0 + uz * uz)
    w = np.pi * rp * rp * nz / n
    bg = cy.uniform_cylinder_background(1.0, rp, vz, nmodes, nr, 1.0, nz, 1.0)
    sim = cy.CylindricalPIC(nz, nr, nmodes, 1.0, 1.0, 1.0, -1.0, 1.0, w,
                            vz if galilean else 0.0, background=bg)
    st = sim.initial_state(x, u, electrostatic=True)
    W = []
    for _ in range(steps):
        st = sim.step(st)
        W.append(cy.field_energy(st["E"], nr, 1.0, 1.0) + cy.field_energy(st["B"], nr, 1.0, 1.0))
    return np.array(W)


def test_nci_pair_in_the_quasi_cylindrical_geometry():
    """The paper's contrast in its own (quasi-cylindrical) geometry, modes 0
    and 1: an electron column (gamma 10, density 1, radius 8, on a
    neutralising ion column) drifting along -z stays quiet on the Galilean
    grid and grows under standard PSATD.  Calibrated on this oracle (80
    steps, dt = dz / c): Galilean max W = 8.8 W(1), standard W(80) = 120 W(1),
    18 times the Galilean W(80); the bars leave a factor of about 2 to 3.
    (With mode 0 alone: 11.3, 329 and 52.)"""
    gal = _drifting_column(True, 80)
    std = _drifting_column(False, 80)
    assert gal.max() <= 25.0 * gal[0]
    assert std[-1] >= 50.0 * std[0]
    assert std[-1] >= 8.0 * gal[-1]


def test_electrostatic_start_satisfies_gauss():
    rng = np.random.default_rng(103)
    nz, nr, dz, dr = 16, 10, 0.8, 0.6
    x, y, z = _cyl_particles(rng, 3000, (nr - 1) * dr, nz * dz)
    sim = cy.CylindricalPIC(nz, nr, 2, dz, dr, 0.5, -1.0, 1.0, 0.3, 0.0)
    st = sim.initial_state(np.stack([x, y, z], 1), np.zeros((len(x), 3)), electrostatic=True)
    live = ~cy.held_mask(nz, nr)
    for m in range(2):
        kz = cy.axis_kz(nz, dz)[:, None] * np.ones((1, nr))
        kr = np.ones((nz, 1)) * cy.update_kr(m, nr, dr)[None, :]
        Ec = cy.to_cartesian(st["E_hat"][m])
        gauss = 1j * (kr * Ec[0] + kz * Ec[2]) - cy.hold_scalar(st["rho_hat"][m], m)
        keep = live & ((kr * kr + kz * kz) > 0)
        assert np.max(np.abs(gauss[keep])) <= 1e-12 * np.max(np.abs(st["rho_hat"][m]))
        # and curl-free: k x E = 0
        assert np.max(np.abs((kz * Ec[0] - kr * Ec[2])[live])) <= 1e-12 * np.max(np.abs(Ec[0]))


@pytest.mark.parametrize("m", [1, 2, 3])
def test_order_m_minus_1_set_is_complete(m):
    """On the zeros of J_m the functions J_{m-1}(k_i r) are a Dini series
    that needs r^{m-1} (k_r = 0) to be complete.  With it, G_- = (r/R)^{m-1}
    is one coefficient; the mode's field (F_r, F_theta) = (G_-, i G_-)
    (for m = 1: the uniform field E_x = 1) then has zero divergence
    spectrally, and the transforms still invert."""
    nz, nr, dz, dr = 8, 16, 0.5, 0.4
    r = cy.radial_grid(nr, dr)
    gm = np.ones((nz, 1)) * (r / (nr * dr))[None, :] ** (m - 1) + 0j
    F = (gm, 1j * gm, np.zeros_like(gm))     # G_- = (F_r - i F_theta) / 2 = gm, G_+ = 0
    G = cy.to_spectral(F, m, dr, dz)
    assert np.max(np.abs(G[1][0, :-1])) <= 1e-10 * nz  # only the k_r = 0 column
    assert abs(G[1][0, -1] - nz) <= 1e-10 * nz          # (the z transform's factor nz)
    kz = cy.axis_kz(nz, dz)[:, None] * np.ones((1, nr))
    kr = np.ones((nz, 1)) * cy.update_kr(m, nr, dr)[None, :]
    Ec = cy.to_cartesian(G)
    assert np.max(np.abs(1j * (kr * Ec[0] + kz * Ec[2]))) <= 1e-10 * nz
    back = cy.from_spectral(G, m, dr, dz)
    for a, b in zip(back, F):
        assert np.max(np.abs(a - b)) <= 1e-10


def test_sideways_current_keeps_continuity_in_mode_one():
    """A uniform column moving along x: its mode-1 charge change and the
    spectral divergence of its mode-1 current agree as well as in mode 0
    (direct deposition is not charge-conserving, so neither is exact).
    Without the k_r = 0 function the mode-1 mismatch was about 8000 times
    the charge change."""
    rng = np.random.default_rng(105)
    nz, nr, dz, dr, dt = 8, 12, 1.0, 1.0, 0.05
    n, rp = 20000, 6.0
    r = rp * np.sqrt(rng.uniform(0, 1, n))
    th = rng.uniform(0, 2 * np.pi, n)
    x = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(0, nz * dz, n)], 1)
    v = np.tile([0.5, 0.0, 0.0], (n, 1))
    xh, xn = x + v * dt / 2, x + v * dt
    res = []
    for m in (0, 1):
        r0 = cy.deposit_mode(x[:, 0], x[:, 1], x[:, 2], np.ones(n), m, "scalar", nr, dr, nz, dz)
        r1 = cy.deposit_mode(xn[:, 0], xn[:, 1], xn[:, 2], np.ones(n), m, "scalar", nr, dr, nz,
                             dz)
        J = cy.deposit_current(xh[:, 0], xh[:, 1], xh[:, 2], v, 1.0, 2, nr, dr, nz, dz)[m]
        dr_dt = cy.hold_scalar((cy.scalar_to_spectral(r1, m, dr, dz)
                                - cy.scalar_to_spectral(r0, m, dr, dz)) / dt, m)
        Ec = cy.to_cartesian(cy.hold(cy.to_spectral(J, m, dr, dz), m))
        kz = cy.axis_kz(nz, dz)[:, None] * np.ones((1, nr))
        kr = np.ones((nz, 1)) * cy.update_kr(m, nr, dr)[None, :]
        live = ~cy.held_mask(nz, nr)
        div = 1j * (kr * Ec[0] + kz * Ec[2])
        res.append(np.linalg.norm((dr_dt + div)[live]) / np.linalg.norm(dr_dt[live]))
    assert res[1] <= 3.0 * max(res[0], 1.0)


@pytest.mark.parametrize("m", [0, 1, 2])
def test_vacuum_propagation_is_exact_for_any_dt(m):
    """Without sources every spectral mode evolves exactly, so N steps of dt
    equal one step of N dt, for any dt (the cylindrical counterpart of the
    Cartesian plane-wave pin), with v_gal = 0 and relativistic."""
    rng = np.random.default_rng(110 + m)
    nz, nr, dz, dr = 16, 12, 0.7, 0.5
    cplx = lambda: rng.standard_normal((nz, nr)) + 1j * rng.standard_normal((nz, nr))
    E = cy.hold(tuple(cplx() for _ in range(3)), m)
    B = cy.hold(tuple(cplx() for _ in range(3)), m)
    zero = np.zeros((nz, nr), dtype=complex)
    # a vacuum field: divergence-free (project out the longitudinal part)
    kz = cy.axis_kz(nz, dz)[:, None] * np.ones((1, nr))
    kr = np.ones((nz, 1)) * cy.update_kr(m, nr, dr)[None, :]
    k2 = np.where(kr * kr + kz * kz > 0, kr * kr + kz * kz, 1.0)

    def transverse(G):
        Fc = list(cy.to_cartesian(G))
        kd = (kr * Fc[0] + kz * Fc[2]) / k2
        Fc[0] = Fc[0] - kr * kd
        Fc[2] = Fc[2] - kz * kd
        return cy.hold(cy.from_cartesian(tuple(Fc)), m)

    E, B = transverse(E), transverse(B)
    for v in (0.0, -0.95):
        for dt, n in ((0.3, 7), (2.1, 3)):
            a, b = E, B
            for _ in range(n):
                a, b = cy.mode_update(a, b, (zero, zero, zero), zero, zero, m, nr, dr, nz, dz,
                                      v, dt)
            c, d = cy.mode_update(E, B, (zero, zero, zero), zero, zero, m, nr, dr, nz, dz, v,
                                  n * dt)
            for x, y in zip(a + b, c + d):
                assert np.max(np.abs(x - y)) <= 1e-11 * np.max(np.abs(np.stack(E))), (v, dt)


@pytest.mark.parametrize("order", [1, 3])
def test_uniform_density_deposits_uniformly_up_to_the_axis(order):
    """A column of density 1 sampled finely (equal-area radii, any angles,
    a regular z lattice) deposits density 1 on every node whose support lies
    inside the column, the axis nodes included: the axis fold (node j < 0
    onto -j-1) and the node volumes must agree for that.  On the nodes that
    straddle the column's edge it deposits the share of the node's shape
    volume inside it, which is the neutralising background's profile."""
    nz, nr, dz, dr = 4, 10, 1.0, 0.5
    R = 7 * dr
    nrad, nzp = 6000, 8
    r = R * np.sqrt((np.arange(nrad) + 0.5) / nrad)
    th = 2.399963 * np.arange(nrad)              # any angles
    zs = (np.arange(nz * nzp) + 0.5) * dz / nzp
    rr = np.repeat(r, len(zs))
    tt = np.repeat(th, len(zs))
    zz = np.tile(zs, nrad)
    w = np.pi * R * R * nz * dz / len(rr)
    g0 = cy.deposit_mode(rr * np.cos(tt), rr * np.sin(tt), zz, np.full(len(rr), w), 0,
                         "scalar", nr, dr, nz, dz, order)
    reach = (order + 1) // 2
    inside = [j for j in range(nr) if (j + 0.5 + reach) * dr <= R]
    assert np.max(np.abs(g0[:, inside] - 1.0)) <= 2e-6, g0[0, inside]
    bg = cy.uniform_cylinder_background(1.0, R, 0.3, 1, nr, dr, nz, dz, order)[0]
    edge = [j for j in range(nr) if (j + 0.5 - reach) * dr < R < (j + 0.5 + reach) * dr]
    assert len(edge) == 2 * reach
    assert np.max(np.abs(g0 - bg[0])) <= 2e-6, (g0[0], bg[0][0])
    assert np.max(np.abs(bg[1][2] - 0.3 * bg[0])) == 0.0


@pytest.mark.parametrize("order", [1, 3])
def test_field_energy_closed_form(order):
    """A uniform mode-0 F_z = 1 and a uniform mode-1 F_r = a: the norm is
    nz (1 + |a|^2 / c_1) times the summed node volumes, which are
    2 pi dz dr^2 (nr^2 / 2 + e) with e the axis nodes' excess over (j + 1/2):
    1/24 for linear shapes (13/24 on node 0) and 1/8 for cubic ones
    ((1199 + 2881) / 1920 on nodes 0 and 1, against 2)."""
    nz, nr, dz, dr = 8, 6, 0.5, 0.7
    a = 0.3 - 0.4j
    one = np.ones((nz, nr), dtype=complex)
    zero = np.zeros((nz, nr), dtype=complex)
    G = [(zero, zero, one), (a * one, zero, zero)]
    excess = 1.0 / 24.0 if order == 1 else 1.0 / 8.0
    vol = 2 * np.pi * dz * dr * dr * (nr * nr / 2.0 + excess)
    expect = nz * vol * (1.0 + abs(a) ** 2 / 2.0)
    assert abs(cy.field_energy(G, nr, dr, dz, order) - expect) <= 1e-12 * expect
