"""GPU parity of the optional Galilean current correction: one update call
against the oracle, a 10-step FP64 history against the oracle, and the
exact Gauss-error evolution it guarantees."""

import numpy as np
import pytest

from oracle import diagnostics as odg
from oracle import pic as opic
from oracle import spectral as osp
from paper_1608_00215_amd import galpic as gp
from workload import get_config, particles_for
from tests.gpu_common import half_k, half_mask, oracle_half_coefficients, rel_l2
from tests.test_gpu_calls import GRIDS, PRECISIONS, ctx_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("shape,spacing,dt", GRIDS)
def test_update_with_correction(gpu_lib, precision, shape, spacing, dt):
    ctx = ctx_for(shape, spacing, dt, precision)
    v = (0.05, 0.1, -0.97)
    ctx.set_v_gal(0, v)
    ctx.set_current_correction(True)
    rng = np.random.Generator(np.random.PCG64(91))
    hshape = (shape[0], shape[1], shape[2] // 2 + 1)
    cplx = lambda: rng.standard_normal(hshape) + 1j * rng.standard_normal(hshape)
    E, B, J = ([cplx() for _ in range(3)] for _ in range(3))
    r0, r1 = cplx(), cplx()
    for a, c in enumerate("XYZ"):
        ctx.write_field(0, f"E{c}_HAT", E[a])
        ctx.write_field(0, f"B{c}_HAT", B[a])
        ctx.write_field(0, f"J{c}_HAT", J[a])
    ctx.write_field(0, "RHO_HAT_OLD", r0)
    ctx.write_field(0, "RHO_HAT_NEW", r1)
    if precision == gp.GP_MIXED:
        E, B, J = ([x.astype(np.complex64).astype(np.complex128) for x in F] for F in (E, B, J))
        r0 = r0.astype(np.complex64).astype(np.complex128)
        r1 = r1.astype(np.complex64).astype(np.complex128)
    ctx.galilean_psatd_update()
    coef, k = oracle_half_coefficients(shape, spacing, v, dt)
    mask = half_mask(shape)
    Jc = osp.galilean_current_correction(tuple(J), r0, r1, k, v, dt, mask)
    En, Bn = osp.galilean_psatd_update(tuple(E), tuple(B), Jc, r0, r1, k, coef, mask)
    tol = 1e-13 if precision == gp.GP_FP64 else 1e-6
    for a, c in enumerate("XYZ"):
        assert rel_l2(ctx.read_field(0, f"E{c}_HAT"), En[a]) <= tol, c
        assert rel_l2(ctx.read_field(0, f"B{c}_HAT"), Bn[a]) <= tol, c
    ctx.close()


def _setup(cfg, precision, inp):
    ctx = gp.Context([gp.grid_from_config(cfg, precision)])
    ctx.set_v_gal(0, cfg.v_gal())
    ctx.set_current_correction(True)
    parts = gp.particles_from_inputs(inp, cfg, precision)
    ctx.bind_particles([parts])
    return ctx, parts


def test_history_with_correction_fp64(gpu_lib):
    """Hot Galilean plasma (particles cross cells every step), 10 steps with
    the correction on: energy every step and the final fields and momenta
    match the oracle run with the correction."""
    cfg = get_config("c1_cic_fp64").with_(u_th=0.3)
    inp = particles_for(cfg)
    ctx, parts = _setup(cfg, gp.GP_FP64, inp)
    g = opic.Grid(cfg.shape, cfg.spacing, cfg.dt, cfg.order)
    sim = opic.Simulation(g, opic.Species(cfg.q, cfg.m, cfg.w), cfg.v_gal(),
                          current_correction=True)
    st = sim.initial_state(inp["x"], inp["u"])
    for n in range(10):
        ctx.step()
        st = sim.step(st)
        we, wb = ctx.field_energy(0)
        ow, ob = odg.field_energy(st.E, st.B, 1.0)
        assert abs((we + wb) - (ow + ob)) <= 1e-10 * (ow + ob), n
    for a, c in enumerate("XYZ"):
        assert rel_l2(ctx.read_field(0, "E" + c), st.E[a]) <= 1e-10
        assert rel_l2(ctx.read_field(0, "B" + c), st.B[a]) <= 1e-10
    ids = parts.id_array()
    assert rel_l2(parts.momenta(), st.u[ids]) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("precision,tol", [(gp.GP_FP64, 1e-11), (gp.GP_MIXED, 2e-5)])
def test_gauss_error_evolves_exactly_gpu(gpu_lib, precision, tol):
    """With the correction on, G = i k.E - rho (rho^n after the step) is
    multiplied by theta^2 C each step, whatever the particles do."""
    cfg = get_config("c2_lite").with_(u_th=0.3)
    inp = particles_for(cfg)
    ctx, parts = _setup(cfg, precision, inp)
    kx, ky, kz = half_k(cfg.shape, cfg.spacing)
    mask = half_mask(cfg.shape)
    c_ee = ctx.read_field(0, "COEF0").astype(np.complex128)

    def gauss():
        E = [ctx.read_field(0, f"E{c}_HAT").astype(np.complex128) for c in "XYZ"]
        rho = ctx.read_field(0, "RHO_HAT_OLD").astype(np.complex128)
        return 1j * (kx * E[0] + ky * E[1] + kz * E[2]) - rho, rho

    G, _ = gauss()
    for n in range(4):
        ctx.step()
        G1, rho = gauss()
        d = np.where(mask, 0, G1 - c_ee * G)
        assert np.max(np.abs(d)) <= tol * np.max(np.abs(rho)), n
        G = G1
    ctx.close()
