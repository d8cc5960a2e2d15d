"""GPU parity of the quasi-cylindrical particle cycle (deposition and gather
by azimuthal mode, Boris push, Galilean moves) against the oracle's
CylindricalPIC, on the same seeded inputs, with linear (order 1) and cubic
(order 3) B-spline shapes.

Bars: one call or step from an identical state, relative L2 per field 1e-12
(FP64) and 1e-5 (mixed), particle positions and momenta within 1e-12 / 1e-5
of their scale; a 10-step axisymmetric history 1e-10 (FP64) and 1e-4 (mixed).
The forward Hankel transforms inside a step carry the derived FP64 bar of
the field-solve tests, max(1e-12, 8 kappa eps) (kappa of these grids is
small, so the bar is 1e-12).
"""

import numpy as np
import pytest

from oracle import cylindrical as cy
from paper_1608_00215_amd import galpic as gp
from tests.gpu_common import rel_l2, tol_for

pytestmark = pytest.mark.gpu

EPS64 = 2.0 ** -52


def _tol(precision, nr, dr, nmodes):
    base = tol_for(precision)
    if precision != gp.GP_FP64:
        return base
    kappa = max(np.linalg.cond(cy.backward_matrix(p, m, nr, dr))
                for m in range(nmodes) for p in (m - 1, m, m + 1))
    return max(base, 8.0 * kappa * EPS64)


def _round(a, precision):
    return a.astype(np.float32).astype(np.float64) if precision == gp.GP_MIXED else a


def _column(rng, n, rp, lz, precision, gamma=None, u_th=0.0):
    r = rp * np.sqrt(rng.uniform(0, 1, n))
    th = rng.uniform(0, 2 * np.pi, n)
    r[:6] = [0.0, 0.05, 0.2, 0.3, 0.45, 0.5]   # on and near the axis
    x = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(0, lz, n)], 1)
    u = u_th * rng.standard_normal((n, 3))
    if gamma is not None:
        u[:, 2] += -np.sqrt(gamma * gamma - 1.0)
    return _round(x, precision), _round(u, precision)


def _gpu_particles(x, u, precision):
    import torch

    dt = torch.float64 if precision == gp.GP_FP64 else torch.float32
    return [torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
            for a in (x[:, 0], x[:, 1], x[:, 2], u[:, 0], u[:, 1], u[:, 2])]


def _bg_arrays(bg, nmodes):
    rho = np.stack([bg[m][0] for m in range(nmodes)])
    J = [np.stack([bg[m][1][a] for m in range(nmodes)]) for a in range(3)]
    return rho, J


def _setup(precision, nz, nr, nmodes, dz, dr, dt, n, vz, seed, rp, gamma=None, u_th=0.0,
           fields=True, background=True, order=1):
    rng = np.random.default_rng(seed)
    x, u = _column(rng, n, rp, nz * dz, precision, gamma, u_th)
    q, mass = -1.0, 1.0
    w = np.pi * rp * rp * nz * dz / n
    bg = cy.uniform_cylinder_background(1.0, rp, vz, nmodes, nr, dr, nz, dz, order) \
        if background else None
    shp = (nz, nr)
    cplx = lambda: 0.05 * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
    E0 = [tuple(cplx() for _ in range(3)) for _ in range(nmodes)] if fields else None
    B0 = [tuple(cplx() for _ in range(3)) for _ in range(nmodes)] if fields else None
    if precision == gp.GP_MIXED and fields:
        c64 = lambda a: a.astype(np.complex64).astype(np.complex128)
        E0 = [tuple(c64(a) for a in e) for e in E0]
        B0 = [tuple(c64(a) for a in b) for b in B0]
    ctx = gp.QcContext(nz, nr, nmodes, dz, dr, dt, precision, shape_order=order)
    ctx.set_v_gal(vz)
    if background:
        rho_bg, J_bg = _bg_arrays(bg, nmodes)
        ctx.set_background(rho_bg, *J_bg)
    if fields:
        names = ("ER", "ET", "EZ", "BR", "BT", "BZ")
        for a in range(3):
            ctx.write(names[a], np.stack([E0[m][a] for m in range(nmodes)]))
            ctx.write(names[3 + a], np.stack([B0[m][a] for m in range(nmodes)]))
        ctx.fields_fwd()
    parts = _gpu_particles(x, u, precision)
    ctx.bind_particles(q, mass, w, *parts)
    # the oracle takes the particles in the order binding left them in
    x, u = _particles_back(parts)
    sim = cy.CylindricalPIC(nz, nr, nmodes, dz, dr, dt, q, mass, w, vz, background=bg,
                            order=order)
    st = sim.initial_state(x, u, E=E0, B=B0)
    return ctx, parts, sim, st


def _particles_back(parts):
    a = [p.cpu().numpy().astype(np.float64) for p in parts]
    return np.stack(a[:3], 1), np.stack(a[3:], 1)


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("background", [False, True])
@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_bound_charge(gpu_lib, precision, background, order):
    nz, nr, nm, dz, dr = 16, 14, 2, 0.9, 0.7
    ctx, parts, sim, st = _setup(precision, nz, nr, nm, dz, dr, 0.5, 3000, 0.0, 400,
                                 rp=(nr - 2) * dr, fields=False, background=background,
                                 order=order)
    tol = _tol(precision, nr, dr, nm)
    rho_real = ctx.read("RHO")
    rho_hat = ctx.read("RHO_HAT_OLD")
    x, _ = _particles_back(parts)
    ref = cy.deposit_charge(x[:, 0], x[:, 1], x[:, 2], sim.q * sim.w, nm, nr, dr, nz, dz,
                            order)
    if background:
        ref = [ref[m] + sim.background[m][0] for m in range(nm)]
    for m in range(nm):
        assert rel_l2(rho_real[m], ref[m]) <= tol_for(precision), ("rho", m)
        assert rel_l2(rho_hat[m], st["rho_hat"][m]) <= tol, ("rho^", m)
    ctx.close()


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_electrostatic_start(gpu_lib, precision, order):
    nz, nr, nm, dz, dr = 16, 14, 2, 0.9, 0.7
    ctx, parts, sim, _ = _setup(precision, nz, nr, nm, dz, dr, 0.5, 3000, 0.0, 401,
                                rp=(nr - 2) * dr, fields=False, background=True,
                                order=order)
    x, u = _particles_back(parts)
    st = sim.initial_state(x, u, electrostatic=True)
    ctx.electrostatic_fields()
    tol = _tol(precision, nr, dr, nm)
    got = [ctx.read(n) for n in ("E_PLUS", "E_MINUS", "E_Z_HAT")]
    real = [ctx.read(n) for n in ("ER", "ET", "EZ")]
    for m in range(nm):
        Er = cy.from_spectral(st["E_hat"][m], m, dr, dz)
        for a in range(3):
            assert rel_l2(got[a][m], st["E_hat"][m][a]) <= tol, ("E^", a, m)
            assert rel_l2(real[a][m], Er[a]) <= tol, ("E", a, m)
    ctx.close()


# (nz, nr, modes): the narrow grid deposits through the LDS window; the wide
# one needs 4 sources x 3 modes x (4 or 6) planes x 180 nodes x 16 bytes =
# 135 KiB (linear) or 203 KiB (cubic), above the 128 KiB the library gives the
# window, and takes the plain deposit kernel
GRIDS = {"narrow": (32, 16, 2), "wide": (8, 180, 3)}


@pytest.mark.parametrize("grid", ["narrow", "wide"])
@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_one_step(gpu_lib, precision, order, grid):
    """One whole step with modes 0 and 1 (and 2), relativistic drift, thermal
    spread, random initial fields, the ion background and Galilean moves."""
    nz, nr, nm = GRIDS[grid]
    dz, dr, dt = 0.8, 0.6, 0.5
    vz = -0.9
    ctx, parts, sim, st = _setup(precision, nz, nr, nm, dz, dr, dt, 4000, vz, 402,
                                 rp=(nr - 2) * dr, gamma=2.0, u_th=0.05, order=order)
    ctx.particle_step(1)
    ctx.synchronize()
    st1 = sim.step(st)
    tol = _tol(precision, nr, dr, nm)
    # the oracle's step returns its deposits with the background added, as
    # the library's source arrays hold them
    for a, name in enumerate(("JR", "JT", "JZ")):
        got = ctx.read(name)
        for m in range(nm):
            assert rel_l2(got[m], st1["J"][m][a]) <= tol_for(precision), (name, m)
    rho = ctx.read("RHO")
    for m in range(nm):
        assert rel_l2(rho[m], st1["rho"][m]) <= tol_for(precision), ("rho", m)
    for names, F in ((("ER", "ET", "EZ"), st1["E"]), (("BR", "BT", "BZ"), st1["B"])):
        for a, n in enumerate(names):
            got = ctx.read(n)
            for m in range(nm):
                assert rel_l2(got[m], F[m][a]) <= tol, (n, m)
    x, u = _particles_back(parts)
    # positions: a few roundings of the coordinate (float: 6e-8 relative)
    pos = 1e-12 if precision == gp.GP_FP64 else 1e-6
    lz = nz * dz
    dzp = np.abs(x[:, 2] - st1["x"][:, 2])
    dzp = np.minimum(dzp, lz - dzp)   # z wraps: compare on the circle
    assert np.max(np.abs(x[:, :2] - st1["x"][:, :2])) <= pos * (nr * dr)
    assert np.max(dzp) <= pos * lz
    mom = 1e-12 if precision == gp.GP_FP64 else 1e-5
    assert np.max(np.abs(u - st1["u"])) <= mom * np.max(np.abs(st1["u"]))
    ctx.close()


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_one_step_eight_modes(gpu_lib, precision, order):
    """The largest mode count a context takes (modes 0..7), one whole step
    with random initial fields, drift and thermal spread."""
    nz, nr, nm, dz, dr, dt = 16, 12, 8, 0.9, 0.7, 0.5
    ctx, parts, sim, st = _setup(precision, nz, nr, nm, dz, dr, dt, 3000, -0.8, 406,
                                 rp=(nr - 2) * dr, gamma=1.8, u_th=0.05, order=order)
    ctx.particle_step(1)
    ctx.synchronize()
    st1 = sim.step(st)
    tol = _tol(precision, nr, dr, nm)
    for a, name in enumerate(("JR", "JT", "JZ")):
        got = ctx.read(name)
        for m in range(nm):
            assert rel_l2(got[m], st1["J"][m][a]) <= tol_for(precision), (name, m)
    rho = ctx.read("RHO")
    for m in range(nm):
        assert rel_l2(rho[m], st1["rho"][m]) <= tol_for(precision), ("rho", m)
    for names, F in ((("ER", "ET", "EZ"), st1["E"]), (("BR", "BT", "BZ"), st1["B"])):
        for a, n in enumerate(names):
            got = ctx.read(n)
            for m in range(nm):
                assert rel_l2(got[m], F[m][a]) <= tol, (n, m)
    _, u = _particles_back(parts)
    mom = 1e-12 if precision == gp.GP_FP64 else 1e-5
    assert np.max(np.abs(u - st1["u"])) <= mom * np.max(np.abs(st1["u"]))
    ctx.close()


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_weights_past_the_last_node_are_dropped(gpu_lib, precision, order):
    """Particles out to a cell beyond the grid's last node: the weights
    that fall past node nr - 1 are dropped on both sides (deposit and
    gather), the rest match the oracle."""
    nz, nr, nm, dz, dr, dt = 16, 10, 2, 1.0, 1.0, 0.5
    ctx, parts, sim, st = _setup(precision, nz, nr, nm, dz, dr, dt, 3000, 0.0, 407,
                                 rp=(nr + 1) * dr, u_th=0.1, order=order, background=False)
    x0, _ = _particles_back(parts)
    assert np.max(np.hypot(x0[:, 0], x0[:, 1])) > (nr - 0.5) * dr   # some weights drop
    ctx.particle_step(1)
    ctx.synchronize()
    st1 = sim.step(st)
    for a, name in enumerate(("JR", "JT", "JZ")):
        got = ctx.read(name)
        for m in range(nm):
            assert rel_l2(got[m], st1["J"][m][a]) <= tol_for(precision), (name, m)
    rho = ctx.read("RHO")
    for m in range(nm):
        assert rel_l2(rho[m], st1["rho"][m]) <= tol_for(precision), ("rho", m)
    _, u = _particles_back(parts)
    mom = 1e-12 if precision == gp.GP_FP64 else 1e-5
    assert np.max(np.abs(u - st1["u"])) <= mom * np.max(np.abs(st1["u"]))
    ctx.close()


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("nm", [1, 2])
@pytest.mark.parametrize("galilean", [True, False])
@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_column_history(gpu_lib, precision, galilean, nm, order):
    """Ten steps of a drifting electron column (gamma 5, a small thermal
    spread) on its ion column, modes 0 (and 1), electrostatic start,
    Galilean or standard frame, linear or cubic shapes."""
    nz, nr, dz, dr, dt = 32, 12, 1.0, 1.0, 1.0
    gamma = 5.0
    uz = np.float32(-np.sqrt(gamma * gamma - 1.0))
    vz = float(uz / np.sqrt(1.0 + uz * uz)) if galilean else 0.0
    rp = 8.0
    rng = np.random.default_rng(403)
    x, u = _column(rng, 5000, rp, nz * dz, precision, gamma, u_th=0.02)
    n = len(x)
    w = np.pi * rp * rp * nz * dz / n
    v_ion = float(uz / np.sqrt(1.0 + uz * uz))
    bg = cy.uniform_cylinder_background(1.0, rp, v_ion, nm, nr, dr, nz, dz, order)
    ctx = gp.QcContext(nz, nr, nm, dz, dr, dt, precision, shape_order=order)
    ctx.set_v_gal(vz)
    rho_bg, J_bg = _bg_arrays(bg, nm)
    ctx.set_background(rho_bg, *J_bg)
    parts = _gpu_particles(x, u, precision)
    ctx.bind_particles(-1.0, 1.0, w, *parts)
    x, u = _particles_back(parts)   # in the order binding left them in
    ctx.electrostatic_fields()
    sim = cy.CylindricalPIC(nz, nr, nm, dz, dr, dt, -1.0, 1.0, w, vz, background=bg,
                            order=order)
    st = sim.initial_state(x, u, electrostatic=True)
    steps = 10
    ctx.particle_step(steps)
    ctx.synchronize()
    for _ in range(steps):
        st = sim.step(st)
    tol = 1e-10 if precision == gp.GP_FP64 else 1e-4
    # E and B of each mode as vectors
    for names, F in ((("ER", "ET", "EZ"), st["E"]), (("BR", "BT", "BZ"), st["B"])):
        for m in range(nm):
            got = np.stack([ctx.read(nme)[m] for nme in names])
            ref = np.stack([F[m][a] for a in range(3)])
            assert rel_l2(got, ref) <= tol, (names, m)
    xg, ug = _particles_back(parts)
    lz = nz * dz
    dzp = np.abs(xg[:, 2] - st["x"][:, 2])
    dzp = np.minimum(dzp, lz - dzp)
    assert np.max(np.abs(xg[:, :2] - st["x"][:, :2])) <= tol * 10 * rp
    assert np.max(dzp) <= tol * 10 * lz
    assert np.max(np.abs(ug - st["u"])) <= tol * 10 * np.max(np.abs(st["u"]))
    ctx.close()


def test_particle_errors(gpu_lib):
    import torch

    for bad in (2, 4, -1):
        with pytest.raises(gp.GalpicError) as e:
            gp.QcContext(16, 8, 1, 1.0, 1.0, 0.5, gp.GP_FP64, shape_order=bad)
        assert e.value.status == gp.GP_ERR_ARG, bad
    ctx = gp.QcContext(16, 8, 1, 1.0, 1.0, 0.5, gp.GP_FP64)
    with pytest.raises(gp.GalpicError) as e:
        ctx.particle_step(1)
    assert e.value.status == gp.GP_ERR_STATE
    a = torch.zeros(10, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        ctx.bind_particles(-1.0, 1.0, 1.0, a, a, a, a, a, a)   # float arrays, FP64 context
    b = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(gp.GalpicError):
        ctx.bind_particles(-1.0, 0.0, 1.0, b, b, b, b, b, b)   # mass 0
    # an empty particle set is valid: the cycle then only advances the fields
    e0 = torch.zeros(0, dtype=torch.float64, device="cuda")
    ctx.bind_particles(-1.0, 1.0, 1.0, e0, e0, e0, e0, e0, e0)
    ctx.particle_step(2)
    ctx.synchronize()
    ctx.close()


@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_binding_sorts_along_z(gpu_lib, precision):
    """The library reorders the particles along z at binding (all six
    arrays together); the deposit does not depend on the input order."""
    nz, nr, nm, dz, dr = 32, 12, 1, 1.0, 1.0
    rng = np.random.default_rng(404)
    x, u = _column(rng, 6000, 9.0, nz * dz, precision, gamma=3.0, u_th=0.1)
    perm = rng.permutation(len(x))
    xs, us = x[perm], u[perm]
    out = []
    for xin, uin in ((x, u), (xs, us)):
        ctx = gp.QcContext(nz, nr, nm, dz, dr, 0.5, precision)
        parts = _gpu_particles(xin, uin, precision)
        ctx.bind_particles(-1.0, 1.0, 0.2, *parts)
        xb, ub = _particles_back(parts)
        assert np.all(np.diff(xb[:, 2]) >= 0)
        # the same particles, moved together
        key = lambda a, b: np.lexsort((b[:, 2], a[:, 1], a[:, 0], a[:, 2]))
        ref = key(xin, uin)
        got = key(xb, ub)
        assert np.array_equal(xb[got], xin[ref]) and np.array_equal(ub[got], uin[ref])
        ctx.particle_step(2)
        ctx.synchronize()
        out.append(ctx.read("RHO"))
        ctx.close()
    assert rel_l2(out[1], out[0]) <= tol_for(precision)


@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_nci_pair_on_the_gpu(gpu_lib, precision):
    """The paper's contrast in its quasi-cylindrical geometry, run by the
    library: an electron column (gamma 10, density 1, radius 8, 20000
    particles, modes 0 and 1) drifting along -z on its ion column stays
    quiet on the Galilean grid and grows under standard PSATD; the bars of
    the oracle's pin (Galilean max W <= 25 W(1); standard W(80) >= 50 W(1)
    and >= 8 times the Galilean W(80))."""
    nz, nr, nm, n, gamma, rp = 64, 12, 2, 20000, 10.0, 8.0
    energies = {}
    for galilean in (True, False):
        rng = np.random.default_rng(1)
        r = rp * np.sqrt(rng.uniform(0, 1, n))
        th = rng.uniform(0, 2 * np.pi, n)
        x = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(0, nz, n)], 1)
        u = np.zeros((n, 3))
        u[:, 2] = -np.sqrt(gamma * gamma - 1.0)
        x, u = _round(x, precision), _round(u, precision)
        vz = float(u[0, 2] / np.sqrt(1.0 + u[0, 2] ** 2))
        w = np.pi * rp * rp * nz / n
        bg = cy.uniform_cylinder_background(1.0, rp, vz, nm, nr, 1.0, nz, 1.0)
        ctx = gp.QcContext(nz, nr, nm, 1.0, 1.0, 1.0, precision)
        ctx.set_v_gal(vz if galilean else 0.0)
        rho_bg, J_bg = _bg_arrays(bg, nm)
        ctx.set_background(rho_bg, *J_bg)
        parts = _gpu_particles(x, u, precision)
        ctx.bind_particles(-1.0, 1.0, w, *parts)
        ctx.electrostatic_fields()
        W = []
        for s in range(80):
            ctx.particle_step(1)
            if s == 0 or s % 10 == 9:
                G = lambda names: [tuple(ctx.read(nme)[m].astype(np.complex128) for nme in names)
                                   for m in range(nm)]
                W.append(cy.field_energy(G(("ER", "ET", "EZ")), nr, 1.0, 1.0)
                         + cy.field_energy(G(("BR", "BT", "BZ")), nr, 1.0, 1.0))
        energies[galilean] = np.array(W)
        ctx.close()
    gal, std = energies[True], energies[False]
    assert gal.max() <= 25.0 * gal[0], gal / gal[0]
    assert std[-1] >= 50.0 * std[0], std / std[0]
    assert std[-1] >= 8.0 * gal[-1], (std[-1], gal[-1])


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_column_workload_sampled(gpu_lib, precision, order):
    """The benchmarked column at its full size and launch configuration (nz
    512, nr 128, modes 0 and 1, an electron column of radius 96 with 24
    particles per (r, z) cell: 1,179,648 particles, gamma 20 along -z,
    Galilean frame), checked where the oracle can compute single outputs:
    rho at 24 sampled nodes after binding (the oracle deposits only the
    particles inside a node's support), and after one step the moved
    positions and pushed momenta of 2000 sampled particles (the oracle
    gathers from the library's own fields at the library's new positions)."""
    nz, nr, nm, dz, dr, dt, gamma, rp = 512, 128, 2, 1.0, 1.0, 1.0, 20.0, 96.0
    rng = np.random.default_rng(408)
    n = int(24 * nz * rp / dr)
    r = rp * np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    x = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(0.0, nz * dz, n)], 1)
    u = np.zeros((n, 3))
    u[:, 2] = -np.sqrt(gamma * gamma - 1.0)
    x, u = _round(x, precision), _round(u, precision)
    w = np.pi * rp * rp * nz * dz / n
    vz = float(u[0, 2] / np.sqrt(1.0 + u[0, 2] ** 2))
    ctx = gp.QcContext(nz, nr, nm, dz, dr, dt, precision, shape_order=order)
    ctx.set_v_gal(vz)
    parts = _gpu_particles(x, u, precision)
    ctx.bind_particles(-1.0, 1.0, w, *parts)
    x0, u0 = _particles_back(parts)
    rho = ctx.read("RHO")
    reach = (order + 1) // 2
    r0 = np.hypot(x0[:, 0], x0[:, 1])
    scale = np.max(np.abs(rho[0]))
    tol = 1e-12 if precision == gp.GP_FP64 else 1e-5
    for _ in range(24):
        k, j = int(rng.integers(0, nz)), int(rng.integers(0, 100))
        dzc = np.abs(x0[:, 2] / dz - k)
        dzc = np.minimum(dzc, nz - dzc)
        near = (dzc < reach + 1) & (r0 < (j + 1.5 + reach) * dr)
        xs = x0[near]
        for m in range(nm):
            ref = cy.deposit_mode(xs[:, 0], xs[:, 1], xs[:, 2], np.full(len(xs), -w), m,
                                  "scalar", nr, dr, nz, dz, order)[k, j]
            assert abs(rho[m][k, j] - ref) <= tol * scale, (k, j, m, rho[m][k, j], ref)
    ctx.electrostatic_fields()
    ctx.particle_step(1)
    ctx.synchronize()
    x1, u1 = _particles_back(parts)
    E = [tuple(ctx.read(nme)[m].astype(np.complex128) for nme in ("ER", "ET", "EZ"))
         for m in range(nm)]
    B = [tuple(ctx.read(nme)[m].astype(np.complex128) for nme in ("BR", "BT", "BZ"))
         for m in range(nm)]
    sim = cy.CylindricalPIC(nz, nr, nm, dz, dr, dt, -1.0, 1.0, w, vz, order=order)
    idx = rng.choice(n, 2000, replace=False)
    from oracle.particles import boris_push, lab_velocity
    v = lab_velocity(u0[idx])
    xr = sim._move(sim._move(x0[idx], v), v)
    dzp = np.abs(x1[idx, 2] - xr[:, 2])
    dzp = np.minimum(dzp, nz * dz - dzp)
    pos = 1e-12 if precision == gp.GP_FP64 else 1e-6
    assert np.max(np.abs(x1[idx, :2] - xr[:, :2])) <= pos * rp
    assert np.max(dzp) <= pos * nz * dz
    Ep = cy.gather_vector(E, x1[idx, 0], x1[idx, 1], x1[idx, 2], nr, dr, nz, dz, order)
    Bp = cy.gather_vector(B, x1[idx, 0], x1[idx, 1], x1[idx, 2], nr, dr, nz, dz, order)
    ur = boris_push(u0[idx], Ep, Bp, -1.0, 1.0, dt)
    # compare the change of u: rounding of u itself (a few ulp of |u|, 20
    # here) plus a relative error of the push
    du_ref = ur - u0[idx]
    du_gpu = u1[idx] - u0[idx]
    c_u, c_du = (1e-13, 1e-10) if precision == gp.GP_FP64 else (2e-6, 1e-5)
    err = np.max(np.abs(du_gpu - du_ref))
    assert err <= c_u * np.max(np.abs(u0)) + c_du * np.max(np.abs(du_ref)), \
        (err, np.max(np.abs(du_ref)))
    ctx.close()


@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_resort_along_z_keeps_the_history(gpu_lib, precision):
    """The device re-sort along z (gp_qc_set_resort) reorders the particles
    between steps and changes nothing else: twenty steps of the cubic
    column with the threshold at zero particles (so a re-sort at the 16th
    deposit) match the oracle's steps in binding order (fields per mode;
    positions and momenta as multisets, each coordinate sorted), and the
    particles have been reordered against a run without re-sorts."""
    nz, nr, nm, dz, dr, dt = 32, 12, 2, 1.0, 1.0, 1.0
    gamma = 5.0
    uz = np.float32(-np.sqrt(gamma * gamma - 1.0))
    vz = float(uz / np.sqrt(1.0 + uz * uz))
    rp = 8.0
    rng = np.random.default_rng(405)
    x0, u0 = _column(rng, 5000, rp, nz * dz, precision, gamma, u_th=0.05)
    w = np.pi * rp * rp * nz * dz / len(x0)
    bg = cy.uniform_cylinder_background(1.0, rp, vz, nm, nr, dr, nz, dz, 3)
    rho_bg, J_bg = _bg_arrays(bg, nm)
    runs = []
    for div in (1 << 30, 0):
        ctx = gp.QcContext(nz, nr, nm, dz, dr, dt, precision, shape_order=3)
        ctx.set_v_gal(vz)
        ctx.set_background(rho_bg, *J_bg)
        ctx.set_resort(div)
        parts = _gpu_particles(x0, u0, precision)
        ctx.bind_particles(-1.0, 1.0, w, *parts)
        xb, ub = _particles_back(parts)
        ctx.electrostatic_fields()
        ctx.particle_step(20)
        ctx.synchronize()
        runs.append((ctx, parts, xb, ub))
    sim = cy.CylindricalPIC(nz, nr, nm, dz, dr, dt, -1.0, 1.0, w, vz, background=bg, order=3)
    st = sim.initial_state(runs[0][2], runs[0][3], electrostatic=True)
    for _ in range(20):
        st = sim.step(st)
    tol = 1e-10 if precision == gp.GP_FP64 else 1e-4
    ctx, parts = runs[0][0], runs[0][1]
    for names, F in ((("ER", "ET", "EZ"), st["E"]), (("BR", "BT", "BZ"), st["B"])):
        for m in range(nm):
            got = np.stack([ctx.read(nme)[m] for nme in names])
            ref = np.stack([F[m][a] for a in range(3)])
            assert rel_l2(got, ref) <= tol, (names, m)
    xg, ug = _particles_back(parts)
    for a in range(3):
        assert np.max(np.abs(np.sort(xg[:, a]) - np.sort(st["x"][:, a]))) <= tol * 10 * nz * dz
        assert np.max(np.abs(np.sort(ug[:, a]) - np.sort(st["u"][:, a]))) <= \
            tol * 10 * np.max(np.abs(st["u"]))
    x_plain, _ = _particles_back(runs[1][1])
    assert not np.array_equal(xg, x_plain)   # reordered
    for r in runs:
        r[0].close()
