"""CPU check of the full-size test helpers: the oracle's deposit on a local
box around a window of nodes equals its deposit on the whole periodic grid,
at windows across the periodic seams, for both shapes."""

import numpy as np
import pytest

from oracle import particles as opt
from workload import get_config
from tests import sampled


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("corner", [(0, 0, 0), (30, 3, 46), (7, 29, 12)])
def test_window_reference_equals_full_deposit(order, corner):
    cfg = get_config("c2_lite").with_(shape=(32, 32, 48), order=order,
                                      spacing=(1.0, 0.5, 2.0))
    rng = np.random.default_rng(3)
    n = 40000
    L = np.array(cfg.shape) * np.array(cfg.spacing)
    x = rng.random((n, 3)) * L
    u = rng.standard_normal((n, 3)) * 2.0
    v, xh, xn = sampled.oracle_moves(cfg, x, u)
    Jw, rw = sampled.window_reference(cfg, corner, xh, v, xn)
    qw = cfg.q * cfg.w / np.prod(cfg.spacing)
    J = opt.deposit(xh, v, cfg.shape, cfg.spacing, order) * qw
    rho = opt.deposit(xn, np.ones(n), cfg.shape, cfg.spacing, order)[0] * qw
    win = sampled.window_index(cfg, corner)
    for a in range(3):
        np.testing.assert_allclose(Jw[a], J[a][win], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rw, rho[win], rtol=1e-12, atol=1e-14)
    # and the particles the source box keeps are enough
    lo, hi = sampled.window_sources(cfg, corner)
    s = x / np.array(cfg.spacing)
    rel = np.mod(s - lo, np.array(cfg.shape))
    near = np.all(rel < (hi - lo), axis=1)
    Jn, rn = sampled.window_reference(cfg, corner, xh[near], v[near], xn[near])
    for a in range(3):
        np.testing.assert_allclose(Jn[a], J[a][win], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rn, rho[win], rtol=1e-12, atol=1e-14)
