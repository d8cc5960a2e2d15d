"""Pins of the oracle's back-transformation to lab-frame snapshots.

The Lorentz transformation of the fields keeps the two field invariants,
inverts with the opposite boost, and multiplies a wave along the boost by
the Doppler factor; the plane timing is the lab time of the grid event; a
history linear in time is interpolated exactly; and a vacuum wave advanced
by the Galilean-PSATD update and back-transformed is the lab-frame wave
(Doppler-shifted in amplitude and wavenumber) within the error bound of
linear interpolation in time.
"""

import numpy as np
import pytest

from oracle import btd
from oracle import coefficients as co
from oracle import spectral as sp

BETAS = [-0.9, 0.3, 0.999]


def _fields(rng, shape=(3, 4, 5)):
    return ([rng.standard_normal(shape) for _ in range(3)],
            [rng.standard_normal(shape) for _ in range(3)])


@pytest.mark.parametrize("beta", BETAS)
def test_field_invariants(beta):
    rng = np.random.default_rng(61)
    E, B = _fields(rng)
    El, Bl = btd.lorentz_to_lab(E, B, beta)
    dot = lambda a, b: a[0] * b[0] + a[1] * b[1] + a[2] * b[2]
    g2 = 1.0 / (1.0 - beta * beta)
    scale = g2 * np.max(dot(E, E) + dot(B, B))
    assert np.max(np.abs(dot(El, Bl) - dot(E, B))) <= 1e-13 * scale
    assert np.max(np.abs((dot(El, El) - dot(Bl, Bl)) - (dot(E, E) - dot(B, B)))) <= 1e-13 * scale


@pytest.mark.parametrize("beta", BETAS)
def test_opposite_boost_inverts(beta):
    rng = np.random.default_rng(62)
    E, B = _fields(rng)
    El, Bl = btd.lorentz_to_lab(E, B, beta)
    E2, B2 = btd.lorentz_to_lab(El, Bl, -beta)
    g2 = 1.0 / (1.0 - beta * beta)
    for a in range(3):
        assert np.max(np.abs(E2[a] - E[a])) <= 1e-13 * g2
        assert np.max(np.abs(B2[a] - B[a])) <= 1e-13 * g2


@pytest.mark.parametrize("beta", BETAS)
def test_wave_along_the_boost_gets_the_doppler_factor(beta):
    f = np.linspace(-1.0, 1.0, 7)
    z = np.zeros_like(f)
    El, Bl = btd.lorentz_to_lab((f, z, z), (z, f, z), beta)
    doppler = np.sqrt((1 + beta) / (1 - beta))
    assert np.allclose(El[0], doppler * f, rtol=1e-13, atol=0)
    assert np.allclose(Bl[1], doppler * f, rtol=1e-13, atol=0)
    assert not np.any(El[1]) and not np.any(Bl[0])


@pytest.mark.parametrize("beta", BETAS)
def test_plane_time_is_the_lab_time_of_the_grid_event(beta):
    """The Galilean node z'_k at boosted time t' is at z_b = z'_k - beta c t'
    (v_gal = -beta c); boosting that event to the lab gives t_lab = t_j and
    z_lab = gamma z'_k."""
    g = 1.0 / np.sqrt(1.0 - beta * beta)
    dz = 0.7
    for tj in (0.0, 13.25, -4.5):
        for k in (0, 3, 64):
            tp = btd.plane_time(tj, k, dz, beta)
            zb = k * dz - beta * tp
            assert abs(g * (tp + beta * zb) - tj) <= 1e-12 * max(1.0, abs(tj), g * g * k * dz)
            assert abs(g * (zb + beta * tp) - g * k * dz) <= 1e-12 * g * g * (1 + k * dz + abs(tp))


def test_linear_history_is_interpolated_exactly():
    rng = np.random.default_rng(63)
    shape, dz, beta = (2, 3, 16), 0.9, 0.6
    t0, dt, nlev = 1.25, 0.5, 12
    a = [rng.standard_normal(shape) for _ in range(6)]
    b = [rng.standard_normal(shape) for _ in range(6)]
    levels = []
    for n in range(nlev):
        t = t0 + n * dt
        F = [a[f] + b[f] * t for f in range(6)]
        levels.append((F[:3], F[3:]))
    g = 1.0 / np.sqrt(1 - beta * beta)
    t_snap = [4.0 / g, 7.0 / g, 30.0]
    snaps, filled = btd.back_transform(levels, t0, dt, t_snap, dz, beta)
    for j, tj in enumerate(t_snap):
        for k in range(shape[2]):
            tp = btd.plane_time(tj, k, dz, beta)
            inside = t0 < tp <= t0 + (nlev - 1) * dt
            assert filled[j][k] == inside
            if not inside:
                assert all(not np.any(snaps[j][f][:, :, k]) for f in range(6))
                continue
            F = [a[f][:, :, k] + b[f][:, :, k] * tp for f in range(6)]
            El, Bl = btd.lorentz_to_lab(F[:3], F[3:], beta)
            for f, v in enumerate(list(El) + list(Bl)):
                assert np.max(np.abs(snaps[j][f][:, :, k] - v)) <= 1e-12 * (1 + np.max(np.abs(v)))
    assert filled[0].any() and not filled[2].any()


def test_vacuum_wave_back_transformed_to_the_lab():
    """A wave along +z in the boosted frame, advanced by the Galilean-PSATD
    update with v_gal = -beta c (exact in vacuum for any dt), back-transforms
    to E_x = B_y = gamma (1 + beta) cos(k_lab (z_lab - c t)) with
    k_lab = gamma (1 + beta) k', within the bound of linear interpolation in
    time: at a Galilean node the wave oscillates at (1 + beta) c k', so the
    error is at most amplitude * ((1 + beta) c k' dt)^2 / 8."""
    shape, spacing, dt, beta = (4, 4, 64), (1.0, 1.0, 1.0), 1.0, 0.5
    v = (0.0, 0.0, -beta)
    k = sp.wavevectors(shape, spacing)
    mask = sp.held_zero_mask(shape)
    coef = co.galilean_psatd_coefficients(k, v, dt)
    kp = 2 * np.pi * 2 / shape[2]
    z = np.arange(shape[2]) * spacing[2]
    Ex0 = np.broadcast_to(np.cos(kp * z), shape).copy()
    zeros = np.zeros(shape)
    E = (sp.forward(Ex0), sp.forward(zeros), sp.forward(zeros))
    B = (sp.forward(zeros), sp.forward(Ex0), sp.forward(zeros))
    zero_spec = np.zeros(shape, dtype=complex)
    levels = []
    for n in range(50):
        levels.append(([sp.inverse(a) for a in E], [sp.inverse(b) for b in B]))
        E, B = sp.galilean_psatd_update(E, B, (zero_spec,) * 3, zero_spec, zero_spec, k, coef,
                                        mask)
    g = 1.0 / np.sqrt(1 - beta * beta)
    t_snap = [46.5 / g, 60.0 / g]
    snaps, filled = btd.back_transform(levels, 0.0, dt, t_snap, spacing[2], beta)
    assert filled[0].all()                      # spans boosted times 4.5 .. 46.5
    assert 0 < filled[1].sum() < shape[2]       # planes past the last level missing
    amp = g * (1 + beta)
    klab = g * (1 + beta) * kp
    bound = amp * ((1 + beta) * kp * dt) ** 2 / 8
    for j, tj in enumerate(t_snap):
        zl = g * z[filled[j]]
        ref = amp * np.cos(klab * (zl - tj))
        for f in (0, 4):                          # E_x and B_y
            got = snaps[j][f][:, :, filled[j]]
            assert np.max(np.abs(got - ref[None, None, :])) <= bound * (1 + 1e-9) + 1e-12
        for f in (1, 2, 3, 5):
            assert np.max(np.abs(snaps[j][f])) <= 1e-12
