"""The batched form against the oracle, stage by stage.  The 64-run
workload (grids {32, 64}^2 x {64, 128, 256}, gamma in [5, 50], density
scale in [0.5, 2], 4 cubic particles per cell) sits in one context, so
every stage is one launch for all runs (one per grid shape for transforms
and update).  After two whole steps, each stage call of the third step is
checked, for three runs (the largest grid, the smallest, and one with
64-point x lines and 128-point z lines), against the oracle applied to the
library's own input of that stage: the deposit, the forward transform, the
update at sampled modes, the inverse transform and the fused
gather-push + deposit."""

import numpy as np
import pytest

from oracle import particles as opt
from oracle import spectral as osp
from paper_1608_00215_amd import galpic as gp
from workload import batched_runs, particles_for
from tests import sampled as sm
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu

RUNS = batched_runs()
# (64, 64, 256), (32, 32, 64), (64, 32, 128)
PICK = [6, 4, 13]
BARS = {gp.GP_MIXED: (2e-6, 1e-5), gp.GP_FP64: (1e-13, 1e-10)}
FTOL = {gp.GP_MIXED: 1e-5, gp.GP_FP64: 1e-12}
TTOL = {gp.GP_MIXED: 2e-6, gp.GP_FP64: 1e-13}   # transforms
# the forward transform of the sources: float rounding of the whole field,
# mean charge and current included, against the k != 0 spectrum that is
# left (the mean is held at zero), ~15 % of it at 4 particles per cell
STOL = {gp.GP_MIXED: 1e-5, gp.GP_FP64: 1e-12}


@pytest.fixture(scope="module")
def c5_inputs():
    return [particles_for(c) for c in RUNS]


def test_picked_runs_cover_the_shapes():
    assert [RUNS[r].shape for r in PICK] == [(64, 64, 256), (32, 32, 64), (64, 32, 128)]


def _full_deposit(cfg, xh, v, xn):
    qw = cfg.q * cfg.w / np.prod(cfg.spacing)
    J = opt.deposit(xh, v, cfg.shape, cfg.spacing, cfg.order) * qw
    rho = opt.deposit(xn, np.ones(len(xn)), cfg.shape, cfg.spacing, cfg.order)[0] * qw
    return J, rho


def _check_sources(ctx, r, cfg, before, tol):
    """J, rho of run r after a deposit against the oracle, from `before`:
    ('full', x, u_dep) or ('windows', {corner: (x, u_dep)})."""
    J = [ctx.read_field(r, "J" + c) for c in "XYZ"]
    rho = ctx.read_field(r, "RHO")
    if before[0] == "full":
        _, x, u = before
        v, xh, xn = sm.oracle_moves(cfg, x, u)
        Jr, rr = _full_deposit(cfg, xh, v, xn)
        for a in range(3):
            assert rel_l2(J[a], Jr[a]) <= tol, (r, a)
        assert rel_l2(rho, rr) <= tol, r
        return
    for corner, (x, u) in before[1].items():
        v, xh, xn = sm.oracle_moves(cfg, x, u)
        Jr, rr = sm.window_reference(cfg, corner, xh, v, xn)
        win = sm.window_index(cfg, corner)
        for a in range(3):
            assert rel_l2(J[a][win], Jr[a]) <= tol, (r, corner, a)
        assert rel_l2(rho[win], rr) <= tol, (r, corner)


def _before(parts, cfg, pushed_fields=None):
    """The state the next particle pass starts from, for the source check:
    every particle of a small run, or the particles near four windows of a
    large one; with pushed_fields the pass first pushes them (oracle)."""
    def prep(x, u):
        if pushed_fields is None:
            return x, u
        un, _, _, _ = sm.oracle_pass(cfg, x, u, pushed_fields)
        return x, un

    if cfg.n_particles <= (1 << 20):
        x, u = sm.state_of(parts, cfg, np.arange(cfg.n_particles))
        return ("full",) + prep(x, u)
    nx, ny, nz = cfg.shape
    corners = [(0, 0, 0), (nx // 2 - 1, 3, nz // 2), (nx - 1, ny - 1, nz - 1), (5, ny // 2, 60)]
    out = {}
    for corner in corners:
        lo, hi = sm.window_sources(cfg, corner)
        ids = sm.ids_near(parts, cfg, lo, hi)
        out[corner] = prep(*sm.state_of(parts, cfg, ids))
    return ("windows", out)


@pytest.mark.parametrize("precision", [gp.GP_MIXED, gp.GP_FP64])
def test_batched_stages_match_oracle(gpu_lib, c5_inputs, precision):
    ctx = gp.Context([gp.grid_from_config(c, precision) for c in RUNS])
    for r, c in enumerate(RUNS):
        ctx.set_v_gal(r, c.v_gal())
    parts = [gp.particles_from_inputs(i, c, precision, with_ids=True)
             for c, i in zip(RUNS, c5_inputs)]
    ctx.bind_particles(parts)
    ctx.run(2)
    ctx.synchronize()
    # deposit
    before = {r: _before(parts[r], RUNS[r]) for r in PICK}
    ctx.deposit()
    ctx.synchronize()
    for r in PICK:
        _check_sources(ctx, r, RUNS[r], before[r], FTOL[precision])
    # forward transform of the library's J, rho
    ctx.fft_fwd()
    ctx.synchronize()
    spectra = {}
    for r in PICK:
        cfg = RUNS[r]
        nzh = cfg.shape[2] // 2 + 1
        mask = osp.held_zero_mask(cfg.shape)
        for src, dst in (("JX", "JX_HAT"), ("JY", "JY_HAT"), ("JZ", "JZ_HAT"),
                         ("RHO", "RHO_HAT_NEW")):
            ref = osp.forward(ctx.read_field(r, src).astype(np.float64))
            ref[mask] = 0
            assert rel_l2(ctx.read_field(r, dst), ref[:, :, :nzh]) <= STOL[precision], (r, dst)
        spectra[r] = {n: ctx.read_field(r, n) for n in sm.SPECTRA}
    # update at sampled modes
    ctx.galilean_psatd_update()
    ctx.synchronize()
    # against the update's term scale: float inputs and complex64 coefficients
    # carry 6e-8 of each term, and the result can be far smaller than its
    # terms (B_z of a drifting plasma)
    utol = 1e-6 if precision == gp.GP_MIXED else 1e-13
    for r in PICK:
        cfg = RUNS[r]
        idx = sm.sample_modes(cfg.shape, 6000, 60 + r)
        sm.check_update(ctx, r, cfg, spectra[r], idx, utol)
    # inverse transform of the library's E^, B^
    ctx.fft_inv()
    ctx.synchronize()
    fields = {}
    for r in PICK:
        cfg = RUNS[r]
        for c in sm.FIELDS6:
            ref = osp.inverse(sm.full_from_half(ctx.read_field(r, c + "_HAT"), cfg.shape))
            assert rel_l2(ctx.read_field(r, c), ref) <= TTOL[precision], (r, c)
        fields[r] = sm.read_fields(ctx, r)
    # the fused gather-push + deposit
    rng = np.random.Generator(np.random.PCG64(61))
    picks = {r: rng.choice(RUNS[r].n_particles, min(20000, RUNS[r].n_particles), replace=False)
             for r in PICK}
    pstate = {r: sm.state_of(parts[r], RUNS[r], picks[r]) for r in PICK}
    before = {r: _before(parts[r], RUNS[r], fields[r]) for r in PICK}
    ctx.gather_push_deposit()
    ctx.synchronize()
    for r in PICK:
        cfg = RUNS[r]
        x0, u0 = pstate[r]
        x1, u1 = sm.state_of(parts[r], cfg, picks[r])
        un, _, _, xn = sm.oracle_pass(cfg, x0, u0, fields[r])
        assert sm.momentum_bar(u1, un, u0, *BARS[precision]) <= 1.0, r
        assert sm.periodic_max_diff(x1, xn, cfg) <= (2e-5 if precision == gp.GP_MIXED
                                                     else 1e-11), r
        _check_sources(ctx, r, cfg, before[r], FTOL[precision])
    ctx.close()
