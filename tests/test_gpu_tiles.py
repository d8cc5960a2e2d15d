"""The tuning knobs (tile shape, re-sort threshold) change nothing but the
order of float sums: FP64 histories with other tile shapes and an eager
re-sort match the oracle as the default does."""

import numpy as np
import pytest

from oracle import diagnostics as odg
from paper_1608_00215_amd import galpic as gp
from workload import get_config, particles_for
from tests.gpu_common import oracle_sim, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tile,resort_div", [((4, 8, 4), 4), ((4, 4, 4), 64), ((8, 2, 8), 1)])
def test_fp64_history_with_tiles(gpu_lib, tile, resort_div):
    cfg = get_config("c2_lite").with_(u_th=0.3, galilean=False)
    inp = particles_for(cfg)
    ctx = gp.Context([gp.grid_from_config(cfg, gp.GP_FP64, tile=tile, resort_div=resort_div)])
    ctx.set_v_gal(0, cfg.v_gal())
    parts = gp.particles_from_inputs(inp, cfg, gp.GP_FP64)
    ctx.bind_particles([parts])
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    for n in range(8):
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
    if resort_div == 1:
        assert ctx.sort_count(0) > 1   # hot plasma, eager threshold: re-sorted on the way
    ctx.close()


def test_bad_tile_rejected(gpu_lib):
    cfg = get_config("c2_lite")
    with pytest.raises(gp.GalpicError):
        gp.Context([gp.grid_from_config(cfg, gp.GP_MIXED, tile=(3, 8, 8))])


@pytest.mark.parametrize("tile", [(4, 4, 8), (8, 4, 4), (4, 4, 4)])
def test_mixed_steps_with_small_tiles(gpu_lib, tile):
    """Small tiles in mixed precision (smaller regions, bucket blocks and
    lists than the default): three steps of a hot cubic plasma against the
    oracle, to the same bars as the default tiles."""
    from tests.test_gpu_step import compare_state

    cfg = get_config("c2_lite").with_(u_th=0.2)
    inp = particles_for(cfg)
    ctx = gp.Context([gp.grid_from_config(cfg, gp.GP_MIXED, tile=tile)])
    ctx.set_v_gal(0, cfg.v_gal())
    parts = gp.particles_from_inputs(inp, cfg, gp.GP_MIXED)
    ctx.bind_particles([parts])
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    ctx.run(3)
    for _ in range(3):
        st = sim.step(st)
    compare_state(ctx, parts, st, cfg, 2e-5, 5e-6)
    ctx.close()
