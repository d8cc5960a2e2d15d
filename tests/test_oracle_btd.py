"""Pins of the oracle's back-transformation to lab-frame snapshots.

The Lorentz transformation of the fields keeps the two field invariants,
inverts with the opposite boost, and multiplies a wave along the boost by
the Doppler factor; the plane timing is the lab time of the grid event; a
history linear in time is interpolated exactly; and a vacuum wave advanced
by the Galilean-PSATD update and back-transformed is the lab-frame wave
(Doppler-shifted in amplitude and wavenumber) within the error bound of
linear interpolation in time.  Particles at rest in the lab are recorded
once per snapshot their worldline passes, at z_lab = gamma z' with zero
lab momentum; a particle in uniform motion is recorded along the lab
worldline given by relativistic velocity addition, with a lab momentum on
the mass shell.
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


def _walk(x0, u, dt, nsteps, v_gal_z, t_snap, L):
    """Steps of constant momentum (no fields); crossings of every step."""
    recs = [[] for _ in t_snap]
    x = x0.copy()
    gp = np.sqrt(1.0 + np.sum(u * u, axis=1))
    step = (u / gp[:, None] - np.array([0.0, 0.0, v_gal_z])[None, :]) * dt
    for n in range(nsteps):
        x = x + step
        x = x - np.floor(x / L[None, :]) * L[None, :]
        for j, (idx, vals) in enumerate(btd.particle_crossings(x, u, dt, (n + 1) * dt, v_gal_z,
                                                                t_snap, L)):
            recs[j].append((n, idx, vals))
    return recs


def test_particles_at_rest_in_the_lab_are_recorded_once():
    """Particles at rest in the lab sit still on the Galilean grid: each is
    recorded exactly once per snapshot whose lab time its worldline passes,
    at z_lab = gamma z' with zero lab momentum."""
    rng = np.random.default_rng(64)
    beta, dt, nsteps = 0.8, 0.5, 40
    g = 1.0 / np.sqrt(1 - beta * beta)
    L = np.array([4.0, 4.0, 32.0])
    x0 = rng.random((500, 3)) * L
    u = np.zeros((500, 3))
    u[:, 2] = -g * beta
    t_snap = [3.0, 9.0, 40.0]
    recs = _walk(x0, u, dt, nsteps, -beta, t_snap, L)
    for j, tj in enumerate(t_snap):
        idx = np.concatenate([r[1] for r in recs[j]])
        vals = np.concatenate([r[2] for r in recs[j]])
        assert len(np.unique(idx)) == len(idx)
        # crossed within the run: t'_0 / gamma + gamma beta z < t_j <= t'_N / gamma + ...
        expect = np.nonzero((0.0 / g + g * beta * x0[:, 2] < tj)
                            & (tj <= nsteps * dt / g + g * beta * x0[:, 2]))[0]
        assert np.array_equal(np.sort(idx), expect)
        order = np.argsort(idx)
        assert np.allclose(vals[order, 2], g * x0[expect, 2], rtol=1e-13, atol=1e-12)
        assert np.max(np.abs(vals[:, 3:6])) <= 1e-12
    assert any(len(np.concatenate([r[1] for r in recs[j]])) > 50 for j in range(3))


def test_uniform_motion_has_the_lab_velocity_and_momentum():
    """A particle of constant boosted-frame velocity v' is recorded at
    successive snapshots with displacements of the lab velocity
    (v'_z + beta) / (1 + beta v'_z) along z and v'_x / (gamma (1 + beta
    v'_z)) across, and with a lab momentum on the mass shell:
    1 + |u_lab|^2 = (gamma (gamma'_p + beta u'_z))^2."""
    beta, dt, nsteps = 0.6, 0.25, 400
    g = 1.0 / np.sqrt(1 - beta * beta)
    L = np.array([1e6, 1e6, 1e6])                  # no wrap on the way
    u = np.array([[0.3, -0.2, 0.5], [0.0, 0.1, -1.4], [2.0, 0.0, 0.0]])
    x0 = np.full((3, 3), 5e5)
    t_lab0 = g * beta * 5e5                        # lab time of z' = 5e5 at t' = 0
    t_snap = [t_lab0 + 1.0 + 3.0 * j for j in range(15)]
    recs = _walk(x0, u, dt, nsteps, -beta, t_snap, L)
    gp = np.sqrt(1 + np.sum(u * u, axis=1))
    vp = u / gp[:, None]
    for p in range(3):
        pts = []
        for j, tj in enumerate(t_snap):
            for n, idx, vals in recs[j]:
                k = np.nonzero(idx == p)[0]
                if len(k):
                    pts.append((tj, vals[k[0]]))
        assert len(pts) >= 5, p
        den = 1 + beta * vp[p, 2]
        for (t1, a), (t2, b) in zip(pts, pts[1:]):
            dtl = t2 - t1
            assert abs((b[2] - a[2]) / dtl - (vp[p, 2] + beta) / den) <= 1e-9
            assert abs((b[0] - a[0]) / dtl - vp[p, 0] / (g * den)) <= 1e-9
            assert abs((b[1] - a[1]) / dtl - vp[p, 1] / (g * den)) <= 1e-9
        ul = pts[0][1][3:6]
        assert abs(1 + ul @ ul - (g * (gp[p] + beta * u[p, 2])) ** 2) <= 1e-10 * (1 + ul @ ul)
