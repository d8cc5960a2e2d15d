"""Helpers shared by the GPU parity tests (not collected by pytest)."""

import numpy as np

from oracle import coefficients as oco
from oracle import pic as opic
from oracle import spectral as osp

#: per-field relative L2 tolerances of one call from an identical state
TOL_FP64 = 1e-12
TOL_MIXED = 1e-5


def rel_l2(got, ref, floor=1e-30):
    got = np.asarray(got)
    ref = np.asarray(ref)
    den = max(float(np.linalg.norm(ref.ravel())), floor)
    return float(np.linalg.norm((got - ref).ravel())) / den


def half(spec, nz):
    """Half spectrum [x][y][nz/2+1] of a full C2C spectrum."""
    return np.asarray(spec)[:, :, : nz // 2 + 1]


def half_k(shape, spacing, stencil=(0, 0, 0)):
    k = osp.wavevectors(shape, spacing, stencil)
    nzh = shape[2] // 2 + 1
    kk = tuple(np.array(a[:, :, :nzh]) for a in k)
    # the z-Nyquist index is +nz/2 in the half spectrum (held at zero anyway)
    return kk


def half_mask(shape):
    return osp.held_zero_mask(shape)[:, :, : shape[2] // 2 + 1]


def oracle_sim(cfg, v_gal=None):
    g = opic.Grid(cfg.shape, cfg.spacing, cfg.dt, cfg.order)
    sim = opic.Simulation(g, opic.Species(cfg.q, cfg.m, cfg.w),
                          cfg.v_gal() if v_gal is None else v_gal, stencil=cfg.stencil)
    return sim


def oracle_half_coefficients(shape, spacing, v_gal, dt, stencil=(0, 0, 0)):
    k = half_k(shape, spacing, stencil)
    return oco.galilean_psatd_coefficients(k, v_gal, dt), k


def seeded_real(shape, seed, n=1, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [scale * rng.standard_normal(shape) for _ in range(n)]


def tol_for(precision):
    from paper_1608_00215_amd.galpic import GP_FP64

    return TOL_FP64 if precision == GP_FP64 else TOL_MIXED
