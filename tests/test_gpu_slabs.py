"""GPU parity of the slab field solve (local transforms with guard cells,
gp_set_local_slabs) against the oracle's slab solve: the field cycle alone
from written fields and sources, over several cycles and slab layouts
(full-length windows, which reproduce the global solve, and short ones);
whole steps with particles (the fused particle pass between field cycles),
eagerly and through graph replay; switching back to the global solve; and
the arguments it refuses."""

import numpy as np
import pytest

from oracle import local as olc
from oracle import spectral as osp
from paper_1608_00215_amd import galpic as gp
from workload import get_config, particles_for
from tests.gpu_common import oracle_sim, rel_l2
from tests.test_gpu_step import compare_state

pytestmark = pytest.mark.gpu

SHAPE, SPACING, DT = (16, 16, 64), (1.0, 1.0, 0.5), 0.5
VGAL = (0.0, 0.0, -0.99)
STENCIL = (4, 4, 8)


def _ctx(precision, stencil=STENCIL, shape=SHAPE):
    g = {"nx": shape[0], "ny": shape[1], "nz": shape[2], "dx": SPACING[0], "dy": SPACING[1],
         "dz": SPACING[2], "dt": DT, "order": 3, "precision": precision,
         "stencil": stencil}
    ctx = gp.Context([g])
    ctx.set_v_gal(0, VGAL)
    return ctx


def _held_free(rng, n, real):
    mask = osp.held_zero_mask(SHAPE)
    out = []
    for _ in range(n):
        h = osp.forward(rng.standard_normal(SHAPE))
        h[mask] = 0
        out.append(osp.inverse(h).astype(real).astype(np.float64))
    return out


@pytest.mark.parametrize("precision,tol", [(gp.GP_FP64, 1e-12), (gp.GP_MIXED, 1e-5)])
@pytest.mark.parametrize("n_slabs,guard", [(4, 8), (8, 4), (1, 0), (2, 16)])
def test_slab_field_cycles_match_oracle(gpu_lib, precision, tol, n_slabs, guard):
    """Three field cycles (gp_fft_fwd, gp_galilean_psatd_update, gp_fft_inv)
    from written E, B, J, rho against the oracle's slab solve."""
    real = np.float64 if precision == gp.GP_FP64 else np.float32
    rng = np.random.default_rng(70 + n_slabs)
    ctx = _ctx(precision)
    E = _held_free(rng, 3, real)
    B = _held_free(rng, 3, real)
    rho0 = (rng.standard_normal(SHAPE) + 2.0).astype(real).astype(np.float64)
    for name, f in zip(("EX", "EY", "EZ", "BX", "BY", "BZ", "RHO"), E + B + [rho0]):
        ctx.write_field(0, name, f)
    ctx.set_local_slabs(n_slabs, guard)
    slab = olc.SlabSolver(SHAPE, SPACING, DT, VGAL, STENCIL, n_slabs, guard)
    slab.start(rho0)
    Es, Bs = tuple(E), tuple(B)
    for cycle in range(3):
        J = [(rng.standard_normal(SHAPE) + m).astype(real).astype(np.float64)
             for m in (0.3, -0.1, 0.8)]
        rho1 = (rng.standard_normal(SHAPE) + 2.0).astype(real).astype(np.float64)
        for name, f in zip(("JX", "JY", "JZ", "RHO"), J + [rho1]):
            ctx.write_field(0, name, f)
        ctx.fft_fwd()
        ctx.galilean_psatd_update()
        ctx.fft_inv()
        Es, Bs = slab.step(Es, Bs, J, rho1)
        for a, c in enumerate("XYZ"):
            assert rel_l2(ctx.read_field(0, "E" + c), Es[a]) <= tol, (cycle, "E" + c)
            assert rel_l2(ctx.read_field(0, "B" + c), Bs[a]) <= tol, (cycle, "B" + c)
    ctx.close()


def test_full_window_slab_solve_equals_global_solve(gpu_lib):
    """Windows as long as the grid (2 slabs, 16 guard planes on 64): the
    slab solve is the global solve, on the GPU as in the oracle."""
    rng = np.random.default_rng(80)
    ctxs = [_ctx(gp.GP_FP64), _ctx(gp.GP_FP64)]
    E = _held_free(rng, 3, np.float64)
    B = _held_free(rng, 3, np.float64)
    rho0 = rng.standard_normal(SHAPE) + 2.0
    for ctx in ctxs:
        for name, f in zip(("EX", "EY", "EZ", "BX", "BY", "BZ", "RHO"), E + B + [rho0]):
            ctx.write_field(0, name, f)
    # the global context's rho^n and spectral E, B from the same fields
    ctxs[0].write_field(0, "RHO_HAT_OLD", _global_spec(rho0))
    for name, f in zip(("EX", "EY", "EZ", "BX", "BY", "BZ"), E + B):
        ctxs[0].write_field(0, name + "_HAT", _global_spec(f))
    ctxs[1].set_local_slabs(2, 16)
    for cycle in range(3):
        J = [rng.standard_normal(SHAPE) + m for m in (0.3, -0.1, 0.8)]
        rho1 = rng.standard_normal(SHAPE) + 2.0
        for ctx in ctxs:
            for name, f in zip(("JX", "JY", "JZ", "RHO"), J + [rho1]):
                ctx.write_field(0, name, f)
            ctx.fft_fwd()
            ctx.galilean_psatd_update()
            ctx.fft_inv()
        for c in ("EX", "EY", "EZ", "BX", "BY", "BZ"):
            assert rel_l2(ctxs[1].read_field(0, c), ctxs[0].read_field(0, c)) <= 1e-12, (cycle, c)
    for ctx in ctxs:
        ctx.close()


def _global_spec(f):
    h = osp.forward(f)
    h[osp.held_zero_mask(SHAPE)] = 0
    return h[:, :, : SHAPE[2] // 2 + 1]


def _plasma_cfg():
    return get_config("c2_lite").with_(shape=(16, 16, 32), u_th=0.2, stencil=(8, 8, 8))


@pytest.mark.parametrize("precision,tol_f,tol_x", [(gp.GP_FP64, 1e-10, 1e-9),
                                                   (gp.GP_MIXED, 2e-5, 5e-6)])
def test_slab_steps_with_particles(gpu_lib, precision, tol_f, tol_x):
    """A hot cubic plasma, 4 slabs of 8 planes with 4 guard planes: three
    whole steps (deposit, slab field cycle, fused gather-push + deposit)
    against the oracle's step with its slab solve."""
    cfg = _plasma_cfg()
    inp = particles_for(cfg)
    ctx = gp.Context([gp.grid_from_config(cfg, precision)])
    ctx.set_v_gal(0, cfg.v_gal())
    parts = gp.particles_from_inputs(inp, cfg, precision)
    ctx.bind_particles([parts])
    ctx.set_local_slabs(4, 4)
    g = oracle_sim(cfg).grid
    from oracle import pic as opic

    sim = opic.Simulation(g, opic.Species(cfg.q, cfg.m, cfg.w), cfg.v_gal(),
                          stencil=cfg.stencil, slabs=(4, 4))
    st = sim.initial_state(inp["x"], inp["u"])
    ctx.run(3)
    for _ in range(3):
        st = sim.step(st)
    compare_state(ctx, parts, st, cfg, tol_f, tol_x)
    ctx.close()


def test_slab_graph_replay_and_switching_back(gpu_lib):
    """Graph replays of slab steps equal eager ones (with eager work between
    replays), and turning the slabs off continues with the global solve
    from the current real fields."""
    cfg = _plasma_cfg()
    inp = particles_for(cfg)
    ctxs, parts = [], []
    for _ in range(2):
        ctx = gp.Context([gp.grid_from_config(cfg, gp.GP_FP64)])
        ctx.set_v_gal(0, cfg.v_gal())
        p = gp.particles_from_inputs(inp, cfg, gp.GP_FP64)
        ctx.bind_particles([p])
        ctx.set_local_slabs(4, 4)
        ctxs.append(ctx)
        parts.append(p)
    for rep in range(2):
        ctxs[0].step_graph(2)
        ctxs[0].synchronize()
        ctxs[1].run(2)
        ctxs[1].field_energy(0)
        for c in ("EX", "EY", "EZ", "BX", "BY", "BZ"):
            assert rel_l2(ctxs[0].read_field(0, c), ctxs[1].read_field(0, c)) <= 1e-12, (rep, c)
    for ctx in ctxs:
        ctx.set_local_slabs(0, 0)
        ctx.run(2)
    for c in ("EX", "EY", "EZ", "BX", "BY", "BZ"):
        assert rel_l2(ctxs[0].read_field(0, c), ctxs[1].read_field(0, c)) <= 1e-12, c
    u0 = parts[0].momenta()[np.argsort(parts[0].id_array())]
    u1 = parts[1].momenta()[np.argsort(parts[1].id_array())]
    assert rel_l2(u0, u1) <= 1e-12
    for ctx in ctxs:
        ctx.close()


def test_slab_solve_refusals(gpu_lib):
    ctx = _ctx(gp.GP_FP64, stencil=(4, 4, 0))
    with pytest.raises(gp.GalpicError) as e:
        ctx.set_local_slabs(4, 8)     # exact k along z
    assert e.value.status == gp.GP_ERR_ARG
    ctx.close()
    ctx = _ctx(gp.GP_FP64)
    for n, g in ((3, 4), (4, 6), (4, 32), (-1, 0)):
        with pytest.raises(gp.GalpicError) as e:
            ctx.set_local_slabs(n, g)
        assert e.value.status == gp.GP_ERR_ARG, (n, g)
    ctx.set_current_correction(True)
    with pytest.raises(gp.GalpicError) as e:
        ctx.set_local_slabs(4, 8)
    assert e.value.status == gp.GP_ERR_STATE
    ctx.set_current_correction(False)
    ctx.set_local_slabs(4, 8)
    with pytest.raises(gp.GalpicError) as e:
        ctx.set_current_correction(True)
    assert e.value.status == gp.GP_ERR_STATE
    ctx.close()
