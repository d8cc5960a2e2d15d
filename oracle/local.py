"""Field solve on z-slabs with local transforms and guard cells (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's closing paragraph names, as future work, the parallelisation of
the Galilean scheme by domain decomposition with arbitrary-order (finite
stencil) solvers, where each subdomain transforms only its own cells plus
guard cells.  It does not print the procedure; this module is one reading
of it, taken on a single periodic grid split along z (no data moves between
processes, so the guard exchange is a copy from the global arrays):

* The grid is cut into S slabs of n_s = nz / S planes.  Slab s owns planes
  s n_s .. s n_s + n_s - 1; its window adds g guard planes on each side,
  planes s n_s - g .. s n_s + n_s + g - 1 (periodic), n_w = n_s + 2 g.
* The state is the real-space E, B on the global grid.  Each step, for
  each slab: the windows of E, B and of the sources J^{n+1/2}, rho^{n+1}
  are transformed on the window's own periodic grid (n_x x n_y x n_w).  The
  sources first lose their global means (the co-moving neutralising ions
  of the global solve, which there hold the k = 0 mode at zero: here a
  global sum, not a transform).  The window's Nyquist planes of the
  sources are held at zero, as the global solve holds its own; nothing
  else is held: the window's k = 0 mode is a regular mode ([k] = 0 gives
  E' = E - dt J, B' = B).
* The update is the Galilean-PSATD update with the finite-order symbol [k]
  of the window's grid (the same stencil orders as the global solve).
  rho^n is the slab's rho^{n+1} window of the previous step, which is the
  window of the same global rho array (at start-up: of rho^0).
* The inverse transform gives E, B on the window; its n_s owned planes are
  written back into the global E, B; the guard planes are discarded (the
  next step reads them again from the neighbours' owned planes).

With a window as long as the grid (n_w = nz, e.g. S = 1, g = 0) every slab
sees a cyclic shift of the whole grid and the slab solve is the global
solve.  Otherwise it differs from it by the part of the one-step propagator
that reaches beyond g planes, which shrinks with g the faster the more
local the stencil is.
"""

import numpy as np

from . import spectral as sp
from .coefficients import galilean_psatd_coefficients


def slab_planes(nz, n_slabs, guard):
    """Global z indices of each slab's window (list of arrays of n_w)."""
    if nz % n_slabs:
        raise ValueError("nz must be a multiple of the slab count")
    ns = nz // n_slabs
    return [np.mod(np.arange(s * ns - guard, s * ns + ns + guard), nz) for s in range(n_slabs)]


def source_mask(shape):
    """Held modes of a window's sources: its Nyquist planes (not k = 0)."""
    mask = np.zeros(shape, dtype=bool)
    for axis, n in enumerate(shape):
        if n % 2 == 0:
            index = [slice(None)] * 3
            index[axis] = n // 2
            mask[tuple(index)] = True
    return mask


class SlabSolver:
    """The slab field solve of one periodic grid (see the module text)."""

    def __init__(self, shape, spacing, dt, v_gal, stencil, n_slabs, guard,
                 c=sp.C_LIGHT, eps0=sp.EPS0):
        self.shape = tuple(shape)
        self.n_slabs = int(n_slabs)
        self.guard = int(guard)
        self.planes = slab_planes(shape[2], n_slabs, guard)
        self.ns = shape[2] // n_slabs
        self.wshape = (shape[0], shape[1], self.ns + 2 * self.guard)
        self.c = c
        self.k = sp.wavevectors(self.wshape, spacing, stencil)
        self.coef = galilean_psatd_coefficients(self.k, v_gal, dt, c, eps0)
        self.smask = source_mask(self.wshape)
        self.nomask = np.zeros(self.wshape, dtype=bool)
        self.rho_old = None

    def _window(self, field, s, mean=0.0):
        return np.asarray(field, dtype=np.float64)[:, :, self.planes[s]] - mean

    def _source(self, field, s, mean):
        spec = sp.forward(self._window(field, s, mean))
        spec[self.smask] = 0.0
        return spec

    def start(self, rho):
        """rho^n of every slab from the global rho (at start-up)."""
        m = float(np.mean(rho))
        self.rho_old = [self._source(rho, s, m) for s in range(self.n_slabs)]

    def step(self, E, B, J, rho_new):
        """One update of the global real-space E, B (3-tuples) with the
        global sources J (3-tuple) and rho^{n+1}; returns the new (E, B)."""
        if self.rho_old is None:
            raise RuntimeError("start() first")
        mJ = [float(np.mean(a)) for a in J]
        mr = float(np.mean(rho_new))
        E_out = [np.empty(self.shape) for _ in range(3)]
        B_out = [np.empty(self.shape) for _ in range(3)]
        g, ns = self.guard, self.ns
        for s in range(self.n_slabs):
            Eh = tuple(sp.forward(self._window(E[a], s)) for a in range(3))
            Bh = tuple(sp.forward(self._window(B[a], s)) for a in range(3))
            Jh = tuple(self._source(J[a], s, mJ[a]) for a in range(3))
            rh = self._source(rho_new, s, mr)
            En, Bn = sp.galilean_psatd_update(Eh, Bh, Jh, self.rho_old[s], rh, self.k,
                                              self.coef, self.nomask, self.c)
            own = slice(s * ns, s * ns + ns)
            for a in range(3):
                E_out[a][:, :, own] = sp.inverse(En[a])[:, :, g:g + ns]
                B_out[a][:, :, own] = sp.inverse(Bn[a])[:, :, g:g + ns]
            self.rho_old[s] = rh
        return tuple(E_out), tuple(B_out)
