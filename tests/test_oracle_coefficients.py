"""Pins of the oracle's coefficients and k-space update.

Each test checks the oracle against something other than itself: the
paper's printed closed forms evaluated in 50-digit arithmetic (mpmath), the
exact solution of the per-mode Galilean Maxwell system by a matrix
exponential (scipy), closed forms of standard PSATD, exact plane waves and
the exact drifting-Coulomb equilibrium.
"""

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg

from oracle import coefficients as co
from oracle import diagnostics as dg
from oracle import spectral as sp

mp.mp.dps = 50


def printed_closed_form(phi, nu):
    """theta, chi_1, chi_2, chi_3 exactly as printed (50 digits)."""
    phi = mp.mpf(phi)
    nu = mp.mpf(nu)
    th = mp.exp(1j * nu * phi / 2)
    ths = mp.exp(-1j * nu * phi / 2)
    C = mp.cos(phi)
    S = mp.sin(phi)
    chi1 = (ths - C * th + 1j * nu * th * S) / (1 - nu ** 2)
    chi2 = (chi1 - th * (1 - C)) / (ths - th)
    chi3 = (chi1 - ths * (1 - C)) / (ths - th)
    return complex(th), complex(chi1), complex(chi2), complex(chi3)


def oracle_chis(phi, nu):
    """theta, chi_1..3 from the oracle for k along z with |k| = phi (c = dt = 1)."""
    k = (np.array([0.0]), np.array([0.0]), np.array([phi]))
    coef = co.galilean_psatd_coefficients(k, (0.0, 0.0, nu), 1.0)
    return (coef["theta"][0], coef["chi1"][0], coef["chi2"][0], coef["chi3"][0])


# points that stress the printed form: gamma = 50 along k, small phi,
# large phi, and generic points
HARD_POINTS = [
    (2 * np.pi / 512, -np.sqrt(1 - 1 / 2500.0)),
    (2 * np.pi / 256, np.sqrt(1 - 1 / 2500.0)),
    (0.0123, 0.9998),
    (5.44, 0.9998),
    (5.44, -0.99875),
    (1e-3, 0.5),
    (3.0, 0.3),
    (np.pi, -0.7),
]


@pytest.mark.parametrize("phi,nu", HARD_POINTS)
def test_chis_match_printed_closed_form_hard_points(phi, nu):
    got = oracle_chis(phi, nu)
    ref = printed_closed_form(phi, nu)
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-13 * abs(r)


def test_chis_match_printed_closed_form_random():
    rng = np.random.default_rng(7)
    for _ in range(150):
        phi = rng.uniform(0.005, 9.0)
        nu = rng.uniform(-0.9999, 0.9999)
        if abs(nu * phi) < 1e-3:
            continue
        got = oracle_chis(phi, nu)
        ref = printed_closed_form(phi, nu)
        for g, r in zip(got, ref):
            assert abs(g - r) <= 1e-12 * abs(r), (phi, nu)


@pytest.mark.parametrize("phi", [1e-3, 0.05, 0.7, 2.0, 5.44, 8.5])
def test_standard_psatd_limit(phi):
    """v_gal = 0: theta = 1, chi_1 = 1 - C, chi_2 = 1 - S/phi, chi_3 = C - S/phi."""
    th, chi1, chi2, chi3 = oracle_chis(phi, 0.0)
    p = mp.mpf(phi)
    assert th == 1.0
    assert abs(chi1 - complex(1 - mp.cos(p))) <= 1e-14 * abs(complex(1 - mp.cos(p)))
    ref2 = complex(1 - mp.sin(p) / p)
    ref3 = complex(mp.cos(p) - mp.sin(p) / p)
    assert abs(chi2 - ref2) <= 1e-12 * abs(ref2)
    assert abs(chi3 - ref3) <= 1e-12 * abs(ref3)


def test_k_to_zero_limits():
    dt = 0.7
    k = (np.array([0.0, 1e-7]), np.array([0.0, 0.0]), np.array([0.0, 1e-7]))
    c = co.galilean_psatd_coefficients(k, (0.0, 0.0, -0.99), dt)
    lim = {"c_EE": 1.0, "s": dt, "c_BJ": dt * dt / 2, "c_EJ": -dt,
           "c_R1": -dt * dt / 6, "c_R0": -dt * dt / 3}
    for key, val in lim.items():
        assert abs(c[key][0] - val) <= 1e-15 * abs(val)
        assert abs(c[key][1] - val) <= 1e-6 * abs(val), key


def test_hermitian_symmetry():
    shape, spacing = (8, 6, 10), (1.0, 0.8, 1.3)
    k = sp.wavevectors(shape, spacing)
    v = (0.1, -0.2, -0.95)
    c = co.galilean_psatd_coefficients(k, v, 0.9)
    kneg = tuple(-a for a in k)
    cn = co.galilean_psatd_coefficients(kneg, v, 0.9)
    for key in ("c_EE", "s", "c_BJ", "c_EJ", "c_R1", "c_R0"):
        assert np.max(np.abs(cn[key] - np.conj(c[key]))) <= 1e-15 * np.max(np.abs(c[key]))


def exact_propagator(k, v, dt, E, B, J):
    """Exact per-mode solution of the Galilean Maxwell system in Fourier space
    with J constant over the step in the Galilean coordinates:
       dB/dt = i(k.v) B - i k x E,  dE/dt = i(k.v) E + c^2 i k x B - J/eps0.
    Solved through the matrix exponential of the 7x7 augmented system."""
    kv = float(np.dot(k, v))
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]], dtype=complex)
    A = np.zeros((7, 7), dtype=complex)
    A[0:3, 0:3] = 1j * kv * np.eye(3)
    A[0:3, 3:6] = -1j * K
    A[3:6, 3:6] = 1j * kv * np.eye(3)
    A[3:6, 0:3] = 1j * K
    A[3:6, 6] = -np.asarray(J)
    z = np.concatenate([B, E, [1.0]])
    out = scipy.linalg.expm(A * dt) @ z
    return out[3:6], out[0:3]


def _random_consistent_mode(rng, k, v, dt):
    """Random E, B, J at one mode with div B = 0, Gauss's law for rho^n, and
    rho^{n+1} from the Galilean continuity equation with constant J."""
    cplx = lambda: rng.standard_normal(3) + 1j * rng.standard_normal(3)
    B = cplx()
    B -= k * np.dot(k, B) / np.dot(k, k)
    E = cplx()
    J = cplx()
    rho_old = 1j * np.dot(k, E)
    kv = np.dot(k, v)
    theta2 = np.exp(1j * kv * dt)
    if abs(kv) > 0:
        rho_new = theta2 * rho_old + (1 - theta2) * np.dot(k, J) / kv
    else:
        rho_new = rho_old - 1j * dt * np.dot(k, J)
    return E, B, J, rho_old, rho_new


def _apply_oracle_update(k, v, dt, E, B, J, rho_old, rho_new):
    kk = tuple(np.array([a]) for a in k)
    coef = co.galilean_psatd_coefficients(kk, v, dt)
    mask = np.zeros(1, dtype=bool)
    En, Bn = sp.galilean_psatd_update(
        tuple(np.array([e]) for e in E), tuple(np.array([b]) for b in B),
        tuple(np.array([j]) for j in J), np.array([rho_old]), np.array([rho_new]),
        kk, coef, mask)
    return np.array([a[0] for a in En]), np.array([a[0] for a in Bn])


def test_update_matches_exact_propagator():
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(200):
        gamma = rng.uniform(1.0, 60.0)
        beta = np.sqrt(1 - 1 / gamma ** 2)
        direction = rng.standard_normal(3)
        direction /= np.linalg.norm(direction)
        v = beta * direction if rng.random() < 0.8 else np.zeros(3)
        k = rng.standard_normal(3) * rng.uniform(0.05, 2.0)
        if rng.random() < 0.3:           # k nearly parallel to v
            k = np.linalg.norm(k) * (direction + 1e-3 * rng.standard_normal(3))
        dt = rng.uniform(0.1, 3.0)
        if abs(np.dot(k, v)) * dt > 0.99 * 2 * np.pi:
            continue
        E, B, J, r0, r1 = _random_consistent_mode(rng, k, v, dt)
        En, Bn = _apply_oracle_update(k, v, dt, E, B, J, r0, r1)
        Ee, Be = exact_propagator(k, v, dt, E, B, J)
        scale = np.linalg.norm(np.concatenate([Ee, Be]))
        worst = max(worst, np.linalg.norm(np.concatenate([En - Ee, Bn - Be])) / scale)
    assert worst <= 1e-10, worst


@pytest.mark.parametrize("dt", [0.3, 1.0, 2.7])
def test_vacuum_plane_wave_exact_for_any_dt(dt):
    """A transverse vacuum wave keeps its lab-frame form x = x' + v_gal t:
    E^N = (theta^2 (C - i S))^N E^0 mode by mode, and energy is conserved."""
    shape, spacing = (4, 4, 32), (1.0, 1.0, 1.0)
    k = sp.wavevectors(shape, spacing)
    mask = sp.held_zero_mask(shape)
    v = (0.0, 0.0, -0.995)
    coef = co.galilean_psatd_coefficients(k, v, dt)
    z = np.arange(shape[2]) * spacing[2]
    m = 3
    kz = 2 * np.pi * m / (shape[2] * spacing[2])
    Ex0 = np.broadcast_to(np.cos(kz * z), shape).copy()
    By0 = Ex0.copy()            # B = k^ x E / c for propagation along +z
    zeros = np.zeros(shape)
    E = (sp.forward(Ex0), sp.forward(zeros), sp.forward(zeros))
    B = (sp.forward(zeros), sp.forward(By0), sp.forward(zeros))
    zero_spec = np.zeros(shape, dtype=complex)
    nsteps = 7
    for _ in range(nsteps):
        E, B = sp.galilean_psatd_update(E, B, (zero_spec,) * 3, zero_spec, zero_spec,
                                        k, coef, mask)
    t = nsteps * dt
    # lab frame: Ex(x, t) = cos(kz (x - c t)), evaluated at x = x' + v_gal t
    Ex_exact = np.broadcast_to(np.cos(kz * (z + v[2] * t - t)), shape)
    Ex = sp.inverse(E[0])
    By = sp.inverse(B[1])
    assert np.max(np.abs(Ex - Ex_exact)) <= 1e-12
    assert np.max(np.abs(By - Ex_exact)) <= 1e-12
    we, wb = dg.field_energy((Ex,), (By,), 1.0)
    we0, wb0 = dg.field_energy((Ex0,), (By0,), 1.0)
    assert abs((we + wb) - (we0 + wb0)) <= 1e-12 * (we0 + wb0)


def _drifting_coulomb(k, v, rho_hat, mask, c=1.0, eps0=1.0):
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    kv = k[0] * v[0] + k[1] * v[1] + k[2] * v[2]
    den = np.where(mask, 1.0, eps0 * (k2 - kv * kv / (c * c)))
    phi = np.where(mask, 0.0, rho_hat / den)
    E = tuple(-1j * k[a] * phi + 1j * kv * v[a] * phi / (c * c) for a in range(3))
    kxv = sp.cross(k, v)
    B = tuple(1j * kxv[a] * phi / (c * c) for a in range(3))
    return E, B


def test_drifting_coulomb_field_is_a_fixed_point():
    """Charges static on the Galilean grid (J = rho v_gal, rho^{n+1} = rho^n)
    with their uniformly moving field: the update returns the same fields."""
    rng = np.random.default_rng(3)
    shape, spacing = (8, 8, 16), (1.0, 1.0, 1.0)
    k = sp.wavevectors(shape, spacing)
    mask = sp.held_zero_mask(shape)
    v = np.array([0.05, -0.02, -0.998])
    coef = co.galilean_psatd_coefficients(k, v, 1.0)
    rho = sp.forward(rng.standard_normal(shape))
    rho[mask] = 0
    E, B = _drifting_coulomb(k, v, rho, mask)
    J = tuple(rho * v[a] for a in range(3))
    En, Bn = sp.galilean_psatd_update(E, B, J, rho, rho, k, coef, mask)
    scale = max(np.max(np.abs(a)) for a in E + B)
    err = max(np.max(np.abs(a - b)) for a, b in zip(En + Bn, E + B))
    assert err <= 1e-13 * scale


def test_gauss_law_and_div_b_preserved():
    rng = np.random.default_rng(5)
    shape, spacing = (8, 8, 16), (1.0, 0.9, 1.1)
    k = sp.wavevectors(shape, spacing)
    mask = sp.held_zero_mask(shape)
    v = np.array([0.0, 0.0, -0.99])
    dt = 1.1
    coef = co.galilean_psatd_coefficients(k, v, dt)
    cplx = lambda: sp.forward(rng.standard_normal(shape))
    E = tuple(cplx() for _ in range(3))
    Braw = tuple(cplx() for _ in range(3))
    k2 = np.where(mask, 1.0, k[0] ** 2 + k[1] ** 2 + k[2] ** 2)
    kB = (k[0] * Braw[0] + k[1] * Braw[1] + k[2] * Braw[2]) / k2
    B = tuple(np.where(mask, 0, Braw[a] - k[a] * kB) for a in range(3))
    E = tuple(np.where(mask, 0, e) for e in E)
    J = tuple(np.where(mask, 0, cplx()) for _ in range(3))
    rho_old = 1j * (k[0] * E[0] + k[1] * E[1] + k[2] * E[2])
    kv = k[0] * v[0] + k[1] * v[1] + k[2] * v[2]
    theta2 = np.exp(1j * kv * dt)
    kJ = k[0] * J[0] + k[1] * J[1] + k[2] * J[2]
    safe = np.where(kv == 0, 1.0, kv)
    rho_new = np.where(kv == 0, rho_old - 1j * dt * kJ,
                       theta2 * rho_old + (1 - theta2) * kJ / safe)
    rho_new = np.where(mask, 0, rho_new)
    R = dg.continuity_residual(rho_old, rho_new, J, k, v, dt)
    assert np.max(np.abs(R)) <= 1e-12 * np.max(np.abs(rho_new))
    En, Bn = sp.galilean_psatd_update(E, B, J, rho_old, rho_new, k, coef, mask)
    g = dg.gauss_residual(En, rho_new, k)
    assert np.max(np.abs(g)) <= 1e-12 * np.max(np.abs(rho_new))
    assert np.max(np.abs(dg.divergence_b(Bn, k))) <= 1e-12 * max(np.max(np.abs(b)) for b in Bn)


def test_gauss_error_multiplied_by_theta2_cos():
    """An inconsistent start: the Gauss error is multiplied by theta^2 C."""
    rng = np.random.default_rng(9)
    k = np.array([0.3, -0.4, 1.1])
    v = np.array([0.0, 0.0, -0.97])
    dt = 0.8
    E, B, J, r0, r1 = _random_consistent_mode(rng, k, v, dt)
    err0 = 0.37 - 0.21j
    r0_bad = r0 - err0          # i k.E - rho^n = err0
    # rho^{n+1} still follows continuity from the (inconsistent) rho^n
    kv = np.dot(k, v)
    theta2 = np.exp(1j * kv * dt)
    r1_bad = theta2 * r0_bad + (1 - theta2) * np.dot(k, J) / kv
    En, _ = _apply_oracle_update(k, v, dt, E, B, J, r0_bad, r1_bad)
    err1 = 1j * np.dot(k, En) - r1_bad
    kmag = np.linalg.norm(k)
    assert abs(err1 - theta2 * np.cos(kmag * dt) * err0) <= 1e-13


def test_max_galilean_phase_on_named_workloads():
    from workload import CONFIGS

    for cfg in CONFIGS.values():
        ph = co.max_galilean_phase(cfg.shape, cfg.spacing, cfg.v_gal(), cfg.dt)
        assert ph < 2 * np.pi * (1 - 1e-6)


def test_max_galilean_phase_hand_value():
    """Hand-computed largest Galilean phase: on a 16x16x64 grid with unit
    spacing, the largest non-Nyquist k_z is 2 pi 31 / 64, so with v_gal =
    (0, 0, -beta), beta = sqrt(1 - 1/gamma^2) at gamma = 10, and dt = 1 the
    phase is beta 2 pi 31 / 64 = 3.0281625... (a dropped Nyquist exclusion
    gives beta pi, a dropped 2 pi gives 0.48...)."""
    beta = np.sqrt(1.0 - 1.0 / 100.0)
    got = co.max_galilean_phase((16, 16, 64), (1.0, 1.0, 1.0), (0.0, 0.0, -beta), 1.0)
    assert abs(got - 3.0281625596149095) <= 1e-13
    # half the time step halves it; twice the spacing along z halves it
    assert abs(co.max_galilean_phase((16, 16, 64), (1.0, 1.0, 1.0), (0.0, 0.0, -beta), 0.5)
               - 0.5 * 3.0281625596149095) <= 1e-13
    assert abs(co.max_galilean_phase((16, 16, 64), (1.0, 1.0, 2.0), (0.0, 0.0, -beta), 1.0)
               - 0.5 * 3.0281625596149095) <= 1e-13


def test_max_galilean_phase_brute_force():
    """The largest |k.v_gal| dt over every mode of a small oblique case,
    enumerated one by one from numpy's FFT frequencies with the Nyquist
    planes left out, equals the oracle's per-axis sum."""
    shape, spacing = (8, 6, 10), (1.0, 0.7, 1.3)
    v, dt = (0.3, -0.2, 0.5), 0.9
    best = 0.0
    f = [2 * np.pi * np.fft.fftfreq(n, d) for n, d in zip(shape, spacing)]
    for i in range(shape[0]):
        for j in range(shape[1]):
            for k in range(shape[2]):
                if i == shape[0] // 2 or j == shape[1] // 2 or k == shape[2] // 2:
                    continue
                ph = abs(f[0][i] * v[0] + f[1][j] * v[1] + f[2][k] * v[2]) * dt
                best = max(best, ph)
    got = co.max_galilean_phase(shape, spacing, v, dt)
    assert abs(got - best) <= 1e-14 * best
