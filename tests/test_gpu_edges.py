"""GPU parity at the edges of the supported sizes: the shortest (8) and
longest (1024) transform lines on every axis, whole steps on such grids,
and runs without particles (alone, and next to a run with particles)."""

import numpy as np
import pytest

from oracle import spectral as osp
from paper_1608_00215_amd import galpic as gp
from workload import get_config, laser_fields, particles_for
from tests.gpu_common import half, oracle_half_coefficients, oracle_sim, rel_l2, seeded_real
from tests.test_gpu_step import compare_state, setup

pytestmark = pytest.mark.gpu

# (shape, spacing, dt): the smallest grid, a 1024-long line on each axis,
# and the line lengths of the benchmarked grids that no other case reaches:
# 64-point x and y lines (the batched runs), 256-point x and y lines and
# 512-point z lines (the boosted run)
EDGE_GRIDS = [
    ((8, 8, 8), (1.0, 1.0, 1.0), 1.0),
    ((1024, 8, 16), (0.5, 1.0, 1.0), 0.5),
    ((8, 1024, 16), (1.0, 0.5, 1.0), 0.5),
    ((16, 8, 1024), (1.0, 1.0, 0.5), 0.5),
    ((64, 8, 16), (1.0, 1.0, 1.0), 1.0),
    ((8, 64, 16), (1.0, 1.0, 1.0), 1.0),
    ((256, 8, 16), (1.0, 1.0, 1.0), 1.0),
    ((8, 256, 16), (1.0, 1.0, 1.0), 1.0),
    ((16, 8, 512), (1.0, 1.0, 1.0), 1.0),
]


def _ctx(shape, spacing, dt, precision, order=1):
    g = {"nx": shape[0], "ny": shape[1], "nz": shape[2], "dx": spacing[0], "dy": spacing[1],
         "dz": spacing[2], "dt": dt, "order": order, "precision": precision}
    return gp.Context([g])


@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
@pytest.mark.parametrize("shape,spacing,dt", EDGE_GRIDS)
def test_transforms_and_coefficients_at_edge_sizes(gpu_lib, precision, shape, spacing, dt):
    ctx = _ctx(shape, spacing, dt, precision)
    v = (0.05, -0.1, -0.9)
    ctx.set_v_gal(0, v)
    live = ~osp.held_zero_mask(shape)[:, :, : shape[2] // 2 + 1]
    coef, _ = oracle_half_coefficients(shape, spacing, v, dt)
    ctol = 1e-13 if precision == gp.GP_FP64 else 2e-7
    for i, key in enumerate(("c_EE", "s", "c_BJ", "c_EJ", "c_R1", "c_R0")):
        assert rel_l2(ctx.read_field(0, f"COEF{i}")[live], coef[key][live]) <= ctol, key
    fields = seeded_real(shape, 141, n=4)
    if precision == gp.GP_MIXED:
        fields = [f.astype(np.float32).astype(np.float64) for f in fields]
    for name, f in zip(("JX", "JY", "JZ", "RHO"), fields):
        ctx.write_field(0, name, f)
    ctx.fft_fwd()
    tol = 1e-13 if precision == gp.GP_FP64 else 2e-6
    mask = osp.held_zero_mask(shape)
    for name, f in zip(("JX_HAT", "JY_HAT", "JZ_HAT", "RHO_HAT_NEW"), fields):
        ref = osp.forward(f)
        ref[mask] = 0
        assert rel_l2(ctx.read_field(0, name), half(ref, shape[2])) <= tol, name
    # inverse of held-mode-free spectra through the E and B slots
    specs = []
    for q, name in enumerate(("EX", "EY", "EZ", "BX", "BY", "BZ")):
        spec = osp.forward(seeded_real(shape, 150 + q)[0])
        spec[mask] = 0
        ctx.write_field(0, name + "_HAT", half(spec, shape[2]))
        specs.append(spec)
    ctx.fft_inv()
    for q, name in enumerate(("EX", "EY", "EZ", "BX", "BY", "BZ")):
        assert rel_l2(ctx.read_field(0, name), osp.inverse(specs[q])) <= tol, name
    ctx.close()


@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 8, 1024), (1024, 8, 16)])
def test_steps_at_edge_sizes_fp64(gpu_lib, shape):
    """Five whole steps of a hot CIC plasma on the smallest grid and on
    grids with a 1024-long line (tiles of one cell-row across the short
    axes): fields and particles match the oracle."""
    cfg = get_config("c1_cic_fp64").with_(shape=shape, ppc=2, u_th=0.4)
    ctx, parts, inp = setup(cfg, gp.GP_FP64)
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    for _ in range(5):
        ctx.step()
        st = sim.step(st)
    compare_state(ctx, parts, st, cfg, 1e-10, 1e-9)
    ctx.close()


def _empty_inputs(cfg):
    inp = particles_for(cfg.with_(shape=(8, 8, 8), ppc=1))
    return {k: (v[:0] if isinstance(v, np.ndarray) else (0 if k == "n" else v))
            for k, v in inp.items()}


@pytest.mark.parametrize("precision,tol", [(gp.GP_FP64, 1e-12), (gp.GP_MIXED, 1e-5)])
def test_run_without_particles(gpu_lib, precision, tol):
    """A laser in vacuum: no particles at all; every stage runs on empty
    particle arrays and the fields match the oracle."""
    cfg = get_config("c3_lite")
    inp = _empty_inputs(cfg)
    ctx, parts, _ = setup(cfg, precision, inp)
    lf = laser_fields(cfg)
    E0 = tuple(a.astype(np.float32).astype(np.float64) for a in lf[0])
    B0 = tuple(a.astype(np.float32).astype(np.float64) for a in lf[1])
    ctx.set_fields(0, E0, B0, project_transverse=True)
    sim = oracle_sim(cfg)
    st = sim.initial_state(np.zeros((0, 3)), np.zeros((0, 3)), E0, B0, project_transverse=True)
    ctx.run(4)
    ctx.step_graph(2)
    for _ in range(6):
        st = sim.step(st)
    ctx.synchronize()
    for a, c in enumerate("XYZ"):
        assert rel_l2(ctx.read_field(0, "E" + c), st.E[a]) <= tol, c
        assert rel_l2(ctx.read_field(0, "B" + c), st.B[a]) <= tol, c
    assert not np.any(ctx.read_field(0, "RHO"))
    ctx.close()


def test_empty_run_next_to_a_full_one(gpu_lib):
    """In one context, a run without particles beside a run with them: the
    full run steps exactly as alone (FP64)."""
    cfg = get_config("c2_lite").with_(u_th=0.3)
    inp = particles_for(cfg)
    empty = _empty_inputs(cfg)
    ctx = gp.Context([gp.grid_from_config(cfg, gp.GP_FP64)] * 2)
    for r in range(2):
        ctx.set_v_gal(r, cfg.v_gal())
    parts = [gp.particles_from_inputs(empty, cfg, gp.GP_FP64),
             gp.particles_from_inputs(inp, cfg, gp.GP_FP64)]
    ctx.bind_particles(parts)
    ctx.run(5)
    single, sparts, _ = setup(cfg, gp.GP_FP64, inp)
    single.run(5)
    for c in ("EX", "EY", "EZ", "BX", "BY", "BZ"):
        assert rel_l2(ctx.read_field(1, c), single.read_field(0, c)) <= 1e-12, c
        assert not np.any(ctx.read_field(0, c)), c
    u1 = parts[1].momenta()[np.argsort(parts[1].id_array())]
    u2 = sparts.momenta()[np.argsort(sparts.id_array())]
    assert rel_l2(u1, u2) <= 1e-12
    ctx.close()
    single.close()


@pytest.mark.parametrize("flush", [1, 2])
@pytest.mark.parametrize("shape,tile", [((8, 8, 8), (0, 0, 0)), ((16, 16, 32), (8, 2, 4)),
                                        ((32, 16, 64), (8, 8, 8)), ((8, 32, 16), (1, 4, 2)),
                                        ((32, 32, 32), (8, 8, 8))])
def test_mixed_cubic_steps_small_grid_and_tiles(gpu_lib, shape, tile, flush):
    """Mixed precision, cubic shape, drift margin: on a grid smaller than a
    tile's node region (every region holds some nodes twice), with thin
    tiles (up to four tiles' regions hold a node along an axis; one-cell
    tiles: six), and with the usual 8^3 tiles (at 32^3 at least three tiles
    per axis, the per-tile path of the region sum), three steps match the FP64
    oracle, with the tile regions added by atomics (flush 1) and through the
    region buffer and its per-node sum (flush 2)."""
    cfg = get_config("c2_lite").with_(shape=shape, u_th=0.2)
    inp = particles_for(cfg)
    ctx = gp.Context([gp.grid_from_config(cfg, gp.GP_MIXED, tile=tile, flush=flush)])
    ctx.set_v_gal(0, cfg.v_gal())
    parts = gp.particles_from_inputs(inp, cfg, gp.GP_MIXED)
    ctx.bind_particles([parts])
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    for _ in range(3):
        ctx.step()
        st = sim.step(st)
    compare_state(ctx, parts, st, cfg, 2e-5, 5e-6)
    ctx.close()


@pytest.mark.parametrize("precision,ppc,shape,tol_f,tol_p", [
    (gp.GP_MIXED, 10, (16, 16, 16), 2e-5, 5e-6),
    (gp.GP_MIXED, 16, (16, 16, 16), 2e-5, 5e-6),
    (gp.GP_FP64, 10, (16, 16, 16), 1e-10, 1e-9),
    (gp.GP_FP64, 32, (8, 8, 16), 1e-10, 1e-9),
])
def test_dense_tiles_fused_steps(gpu_lib, precision, ppc, shape, tol_f, tol_p):
    """Tiles denser than the bucket passes' one round or the tile lists'
    capacity, through the fused pass (three steps of gp_run: deposit, two
    fused launches, push) against three oracle steps.  Mixed: 5,120 particles
    per 8^3 tile (two rounds of six per thread; the buckets are read again
    for the placement) and 8,192 (past the list capacity: jobs in memory
    order).  FP64: 5,120 (three rounds of four) and 16,384 (past its
    capacity)."""
    cfg = get_config("c2_lite").with_(shape=shape, ppc=ppc, u_th=0.2)
    ctx, parts, inp = setup(cfg, precision)
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    ctx.run(3)
    for _ in range(3):
        st = sim.step(st)
    compare_state(ctx, parts, st, cfg, tol_f, tol_p)
    ctx.close()


@pytest.mark.parametrize("precision,tol_f,tol_p", [(gp.GP_MIXED, 2e-5, 5e-6),
                                                   (gp.GP_FP64, 1e-10, 1e-9)])
def test_half_filled_grid_fused_steps(gpu_lib, precision, tol_f, tol_p):
    """Particles in the lower half of x only (32x16x32 grid, 8 per cell):
    tiles without particles beside full ones, and tiles whose region holds
    the particles of a neighbour only, through the fused pass (three steps
    of gp_run) against three oracle steps."""
    cfg = get_config("c2_lite").with_(shape=(32, 16, 32), u_th=0.2)
    full = particles_for(cfg)
    keep = full["x"][:, 0] < 0.5 * cfg.shape[0] * cfg.spacing[0]
    inp = {k: (v[keep] if isinstance(v, np.ndarray) else v) for k, v in full.items()}
    inp["n"] = int(np.count_nonzero(keep))
    ctx, parts, inp = setup(cfg, precision, inp)
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    ctx.run(3)
    for _ in range(3):
        st = sim.step(st)
    compare_state(ctx, parts, st, cfg, tol_f, tol_p)
    ctx.close()
