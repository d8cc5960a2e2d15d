"""Pins of the oracle's slab field solve (local transforms with guard
cells).  Pinned against the global finite-order solve: a window as long as
the grid is a cyclic shift of it, so the slab solve must reproduce the
global one to rounding, over several steps, whatever the slab count; with
shorter windows its difference from the global solve must shrink as the
guard planes grow, and faster for a more local stencil."""

import numpy as np
import pytest

from oracle import local as olc
from oracle import spectral as sp
from oracle.coefficients import galilean_psatd_coefficients


def _held_free(rng, shape, n):
    """Real fields whose spectra vanish on the globally held modes (states
    of the global solve)."""
    mask = sp.held_zero_mask(shape)
    out = []
    for _ in range(n):
        h = sp.forward(rng.standard_normal(shape))
        h[mask] = 0
        out.append(sp.inverse(h))
    return out


class GlobalSolver:
    """The global finite-order solve, carried spectrally as the step does."""

    def __init__(self, shape, spacing, dt, v_gal, stencil):
        self.k = sp.wavevectors(shape, spacing, stencil)
        self.mask = sp.held_zero_mask(shape)
        self.coef = galilean_psatd_coefficients(self.k, v_gal, dt)

    def src(self, f):
        h = sp.forward(f)
        h[self.mask] = 0
        return h

    def start(self, E, B, rho):
        self.E = tuple(self.src(a) for a in E)
        self.B = tuple(self.src(a) for a in B)
        self.rho = self.src(rho)

    def step(self, J, rho_new):
        rn = self.src(rho_new)
        self.E, self.B = sp.galilean_psatd_update(self.E, self.B,
                                                  tuple(self.src(a) for a in J), self.rho,
                                                  rn, self.k, self.coef, self.mask)
        self.rho = rn
        return tuple(sp.inverse(a) for a in self.E), tuple(sp.inverse(a) for a in self.B)


@pytest.mark.parametrize("n_slabs,guard", [(1, 0), (2, 8), (4, 12), (8, 14)])
def test_full_window_equals_global_solve(n_slabs, guard):
    shape, spacing, dt = (8, 8, 32), (1.0, 1.0, 0.5), 0.5
    v_gal, stencil = (0.0, 0.0, -0.99), (4, 4, 8)
    assert shape[2] // n_slabs + 2 * guard == shape[2]
    rng = np.random.default_rng(21)
    E = _held_free(rng, shape, 3)
    B = _held_free(rng, shape, 3)
    rho0 = rng.standard_normal(shape) + 3.0
    glob = GlobalSolver(shape, spacing, dt, v_gal, stencil)
    glob.start(E, B, rho0)
    slab = olc.SlabSolver(shape, spacing, dt, v_gal, stencil, n_slabs, guard)
    slab.start(rho0)
    Es, Bs = E, B
    for step in range(3):
        J = [rng.standard_normal(shape) + m for m in (0.5, -0.2, 1.0)]
        rho1 = rng.standard_normal(shape) + 3.0
        Eg, Bg = glob.step(J, rho1)
        Es, Bs = slab.step(Es, Bs, J, rho1)
        scale = max(np.abs(a).max() for a in Eg + Bg)
        for a in range(3):
            np.testing.assert_allclose(Es[a], Eg[a], rtol=0, atol=1e-12 * scale)
            np.testing.assert_allclose(Bs[a], Bg[a], rtol=0, atol=1e-12 * scale)


def _pulse(shape, z0, width, k0):
    """A transverse pulse along z: E_x = B_y = exp(-(z - z0)^2 / w^2) cos(k0 z)
    times a transverse Gaussian (vacuum, no sources)."""
    x = np.arange(shape[0]) - shape[0] / 2
    y = np.arange(shape[1]) - shape[1] / 2
    z = np.arange(shape[2], dtype=float)
    tr = np.exp(-(x[:, None] ** 2 + y[None, :] ** 2) / 9.0)
    lon = np.exp(-((z - z0) / width) ** 2) * np.cos(k0 * (z - z0))
    ex = tr[:, :, None] * lon[None, None, :]
    zero = np.zeros(shape)
    return (ex, zero, zero.copy()), (zero.copy(), ex.copy(), zero.copy())


def _slab_error(stencil_z, guard, steps=8):
    shape, spacing, dt = (8, 8, 128), (1.0, 1.0, 1.0), 1.0
    v_gal = (0.0, 0.0, -0.995)
    stencil = (4, 4, stencil_z)
    E, B = _pulse(shape, 40.0, 6.0, 2 * np.pi / 10)
    glob = GlobalSolver(shape, spacing, dt, v_gal, stencil)
    glob.start(E, B, np.zeros(shape))
    E = tuple(sp.inverse(a) for a in glob.E)
    B = tuple(sp.inverse(a) for a in glob.B)
    slab = olc.SlabSolver(shape, spacing, dt, v_gal, stencil, 8, guard)
    slab.start(np.zeros(shape))
    zero = [np.zeros(shape)] * 3
    Es, Bs = E, B
    for _ in range(steps):
        Eg, Bg = glob.step(zero, np.zeros(shape))
        Es, Bs = slab.step(Es, Bs, zero, np.zeros(shape))
    num = np.sqrt(sum(np.sum((Es[a] - Eg[a]) ** 2 + (Bs[a] - Bg[a]) ** 2) for a in range(3)))
    den = np.sqrt(sum(np.sum(Eg[a] ** 2 + Bg[a] ** 2) for a in range(3)))
    return num / den


def test_slab_error_shrinks_with_guard_and_locality():
    """A vacuum pulse crossing slab edges (8 slabs of 16 planes, v_gal near
    -c so it moves on the grid): the slab solve's distance from the global
    solve falls as the guard planes grow (here from 0.28 at 2 planes to 1e-5
    at 16), and a more local stencil (order 8 against order 32 along z) is
    an order of magnitude closer at 8 guard planes."""
    errs8 = [_slab_error(8, g) for g in (2, 4, 8, 16)]
    assert all(b < a for a, b in zip(errs8, errs8[1:])), errs8
    assert errs8[-1] < 1e-2 * errs8[0], errs8
    assert _slab_error(8, 56) < 1e-12
    # at 8 guard planes: order 8 ~1e-2, order 32 ~2e-1
    assert errs8[2] < 0.2 * _slab_error(32, 8), errs8


def test_slab_windows_and_owned_planes():
    planes = olc.slab_planes(16, 4, 2)
    assert [list(p) for p in planes[:2]] == [[14, 15, 0, 1, 2, 3, 4, 5],
                                            [2, 3, 4, 5, 6, 7, 8, 9]]
    with pytest.raises(ValueError):
        olc.slab_planes(16, 3, 1)
