"""GPU parity of whole steps and step histories against the oracle, graph
replay against eager steps, and the NCI pair on the GPU."""

import numpy as np
import pytest

from oracle import diagnostics as odg
from paper_1608_00215_amd import galpic as gp
from workload import get_config, particles_for
from tests.gpu_common import oracle_sim, rel_l2

pytestmark = pytest.mark.gpu


def setup(cfg, precision, inp=None, flush=0):
    inp = particles_for(cfg) if inp is None else inp
    ctx = gp.Context([gp.grid_from_config(cfg, precision, flush=flush)])
    ctx.set_v_gal(0, cfg.v_gal())
    parts = gp.particles_from_inputs(inp, cfg, precision)
    ctx.bind_particles([parts])
    return ctx, parts, inp


def compare_state(ctx, parts, st, cfg, tol_f, tol_p):
    errs = {}
    for a, c in enumerate("XYZ"):
        errs["E" + c] = rel_l2(ctx.read_field(0, "E" + c), st.E[a])
        errs["B" + c] = rel_l2(ctx.read_field(0, "B" + c), st.B[a])
    ids = parts.id_array()
    errs["u"] = rel_l2(parts.momenta(), st.u[ids])
    L = np.array(cfg.shape) * np.array(cfg.spacing)
    d = np.abs(parts.positions(cfg.shape, cfg.spacing) - st.x[ids])
    d = np.minimum(d, L[None, :] - d)
    errs["x"] = float(d.max())
    for k, v in errs.items():
        tol = tol_p if k == "x" else tol_f
        assert v <= tol, (k, v, errs)
    return errs


@pytest.mark.parametrize("galilean,steps,tol,flush", [(True, 50, 1e-10, 0), (False, 20, 1e-8, 0),
                                                     (False, 20, 1e-8, 2)])
def test_c1_history_fp64(gpu_lib, galilean, steps, tol, flush):
    """16x16x64 FP64 CIC drifting plasma: every step's field energy and the
    final fields and particles match the oracle (the standard run also with
    the tile regions summed through the region buffer, flush 2)."""
    cfg = get_config("c1_cic_fp64").with_(galilean=galilean)
    ctx, parts, inp = setup(cfg, gp.GP_FP64, flush=flush)
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    for n in range(steps):
        ctx.step()
        st = sim.step(st)
        we, wb = ctx.field_energy(0)
        ow, ob = odg.field_energy(st.E, st.B, 1.0)
        assert abs((we + wb) - (ow + ob)) <= tol * (ow + ob), (n, we + wb, ow + ob)
    compare_state(ctx, parts, st, cfg, tol, 1e-9)
    if not galilean:
        # particles cross a cell per step: the tiles were re-sorted on the way
        assert ctx.sort_count(0) > 1
    ctx.close()


@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_run_equals_steps(gpu_lib, precision):
    """gp_run(n) (gather-push fused with the next deposit) equals n gp_step
    calls (separate kernels), for a hot plasma that crosses tiles."""
    cfg = get_config("c2_lite").with_(u_th=0.5, galilean=False)
    ctx1, p1, inp = setup(cfg, precision)
    ctx2, p2, _ = setup(cfg, precision, inp)
    for _ in range(6):
        ctx1.step()
    ctx2.run(6)
    tol = 1e-12 if precision == gp.GP_FP64 else 2e-5
    for c in ("EX", "EY", "EZ", "BX", "BY", "BZ"):
        assert rel_l2(ctx2.read_field(0, c), ctx1.read_field(0, c)) <= tol, c
    u1 = p1.momenta()[np.argsort(p1.id_array())]
    u2 = p2.momenta()[np.argsort(p2.id_array())]
    assert rel_l2(u2, u1) <= tol
    ctx1.close()
    ctx2.close()


def test_step_calls_equal_gp_step(gpu_lib):
    """The five ABI calls in order do exactly what gp_step does."""
    cfg = get_config("c1_cic_fp64").with_(u_th=0.3)
    ctx1, p1, inp = setup(cfg, gp.GP_FP64)
    ctx2, p2, _ = setup(cfg, gp.GP_FP64, inp)
    for _ in range(3):
        ctx1.deposit()
        ctx1.fft_fwd()
        ctx1.galilean_psatd_update()
        ctx1.fft_inv()
        ctx1.gather_push()
        ctx2.step()
    for c in ("EX", "EY", "EZ", "BX", "BY", "BZ"):
        assert rel_l2(ctx1.read_field(0, c), ctx2.read_field(0, c)) <= 1e-13
    u1 = p1.momenta()[np.argsort(p1.id_array())]
    u2 = p2.momenta()[np.argsort(p2.id_array())]
    assert rel_l2(u1, u2) <= 1e-13
    ctx1.close()
    ctx2.close()


@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_graph_replay_matches_eager(gpu_lib, precision):
    """Graph replays (several, with eager work and synchronisation between
    them) give the same state as eager steps."""
    cfg = get_config("c2_lite").with_(u_th=0.2)
    ctx1, p1, inp = setup(cfg, precision)
    ctx2, p2, _ = setup(cfg, precision, inp)
    tol = 1e-12 if precision == gp.GP_FP64 else 2e-5
    for rep in range(3):
        ctx2.step_graph(3)
        ctx2.synchronize()
        for _ in range(3):
            ctx1.step()
        ctx1.field_energy(0)     # eager work between replays
        for c in ("EX", "EZ", "BY"):
            assert rel_l2(ctx2.read_field(0, c), ctx1.read_field(0, c)) <= tol, (rep, c)
        u1 = p1.momenta()[np.argsort(p1.id_array())]
        u2 = p2.momenta()[np.argsort(p2.id_array())]
        assert rel_l2(u2, u1) <= tol
    assert ctx2.last_graph_ms() > 0
    ctx1.close()
    ctx2.close()


@pytest.mark.parametrize("name", ["c2_lite", "c3_lite"])
def test_mixed_one_step(gpu_lib, name):
    """Mixed precision, cubic: one step from an identical state matches the
    FP64 oracle to the mixed tolerance."""
    from workload import laser_fields

    cfg = get_config(name)
    ctx, parts, inp = setup(cfg, gp.GP_MIXED)
    sim = oracle_sim(cfg)
    lf = laser_fields(cfg)
    if lf is not None:
        E0 = tuple(a.astype(np.float32).astype(np.float64) for a in lf[0])
        B0 = tuple(a.astype(np.float32).astype(np.float64) for a in lf[1])
        ctx.set_fields(0, E0, B0, project_transverse=True)
        st = sim.initial_state(inp["x"], inp["u"], E0, B0, project_transverse=True)
    else:
        st = sim.initial_state(inp["x"], inp["u"])
    ctx.step()
    st = sim.step(st)
    compare_state(ctx, parts, st, cfg, 1e-5, 2e-6)
    ctx.close()


def test_mixed_history_c2_lite(gpu_lib):
    """Mixed precision over 20 steps: per-field error and energy drift vs the
    FP64 oracle stay small (reported growth, stated bound)."""
    cfg = get_config("c2_lite")
    ctx, parts, inp = setup(cfg, gp.GP_MIXED)
    sim = oracle_sim(cfg)
    st = sim.initial_state(inp["x"], inp["u"])
    for n in range(cfg.steps):
        ctx.step()
        st = sim.step(st)
        we, wb = ctx.field_energy(0)
        ow, ob = odg.field_energy(st.E, st.B, 1.0)
        assert abs((we + wb) - (ow + ob)) <= 1e-4 * (ow + ob), n
    compare_state(ctx, parts, st, cfg, 1e-4, 1e-5)
    ctx.close()


def test_nci_pair_gpu(gpu_lib):
    """Galilean (v_gal = v0) stays quiet, standard PSATD (v_gal = 0) grows;
    same thresholds as the oracle's calibrated pair."""
    cfg = get_config("c1_cic_fp64")
    hist = {}
    for galilean in (True, False):
        c = cfg.with_(galilean=galilean)
        ctx, parts, _ = setup(c, gp.GP_FP64)
        W = []
        for _ in range(50):
            ctx.step()
            we, wb = ctx.field_energy(0)
            W.append(we + wb)
        hist[galilean] = np.array(W)
        ctx.close()
    Wg, Ws = hist[True], hist[False]
    assert np.max(Wg) <= 6.0 * Wg[0]
    assert Ws[-1] >= 30.0 * Ws[0]
    assert Ws[-1] >= 10.0 * Wg[-1]


@pytest.mark.parametrize("precision,tol_u,tol_f", [(gp.GP_FP64, 1e-12, 1e-12),
                                                   (gp.GP_MIXED, 1e-6, 1e-5)])
def test_laser_start_half_push_c3_lite(gpu_lib, precision, tol_u, tol_f):
    """The laser start as the boosted run uses it: fields set and projected,
    then the Boris half push u^0 -> u^{1/2} (gp_half_push) against the
    oracle's half push, then two whole steps from there."""
    from workload import laser_fields

    cfg = get_config("c3_lite")
    ctx, parts, inp = setup(cfg, precision)
    sim = oracle_sim(cfg)
    lf = laser_fields(cfg)
    E0 = tuple(a.astype(np.float32).astype(np.float64) for a in lf[0])
    B0 = tuple(a.astype(np.float32).astype(np.float64) for a in lf[1])
    ctx.set_fields(0, E0, B0, project_transverse=True)
    st = sim.initial_state(inp["x"], inp["u"], E0, B0, project_transverse=True)
    ctx.half_push()
    st = sim.half_push(st)
    from tests.sampled import momentum_bar

    ids = parts.id_array()
    assert np.max(np.abs(st.u - inp["u"])) > 1e-2      # the pulse kicks the particles
    # per particle: a rounding of the stored momentum plus that of the kick
    bars = (1e-13, 1e-10) if precision == gp.GP_FP64 else (2e-6, 1e-5)
    assert momentum_bar(parts.momenta(), st.u[ids], inp["u"][ids], *bars) <= 1.0
    assert rel_l2(parts.momenta(), st.u[ids]) <= tol_u
    ctx.run(2)
    for _ in range(2):
        st = sim.step(st)
    compare_state(ctx, parts, st, cfg, tol_f * 2, 1e-9 if precision == gp.GP_FP64 else 5e-6)
    ctx.close()


@pytest.mark.parametrize("precision", [gp.GP_FP64, gp.GP_MIXED])
def test_field_pointer_views_the_library_arrays(gpu_lib, precision):
    """gp_field_ptr: a torch view of a real array and of a spectrum reads
    what gp_read_field copies, a write through the view is what the library
    then reads, and the rho^ roles swap at the update."""
    import torch

    cfg = get_config("c2_lite").with_(u_th=0.2)
    ctx, parts, _ = setup(cfg, precision)
    ctx.run(2)
    ctx.synchronize()
    for name in ("EX", "BZ", "RHO", "EY_HAT", "RHO_HAT_OLD", "COEF3"):
        t = ctx.field_tensor(0, name)
        assert np.array_equal(t.cpu().numpy(), ctx.read_field(0, name)), name
    ex = ctx.field_tensor(0, "EX")
    ex.mul_(2.0)
    torch.cuda.synchronize()
    assert np.array_equal(ctx.read_field(0, "EX"), ex.cpu().numpy())
    old = ctx.field_ptr(0, "RHO_HAT_OLD")
    new = ctx.field_ptr(0, "RHO_HAT_NEW")
    assert old != new
    ctx.deposit()
    ctx.fft_fwd()
    ctx.galilean_psatd_update()
    assert ctx.field_ptr(0, "RHO_HAT_OLD") == new
    assert ctx.field_ptr(0, "RHO_HAT_NEW") == old
    with pytest.raises(gp.GalpicError):
        ctx.field_ptr(1, "EX")
    ctx.close()
