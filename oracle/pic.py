"""One full Galilean-PSATD particle-in-cell step (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The order is the one the paper states after the update equations: deposit
J at (n + 1/2) dt and rho at (n + 1) dt on the grid nodes, transform them to
Fourier space, advance the spectral E and B, transform the fields back, and
interpolate them to the particles, which then advance with the
Galilean-transformed equations of motion.

State at the start of step n: positions x'^n (absolute, in [0, L)),
momenta u^{n+1/2} = p / (m c), spectral E^n, B^n, rho^n, and the real-space
E^n, B^n.  One step:

  v      = c u / gamma                          (lab velocity at n + 1/2)
  x_h    = x'^n + (v - v_gal) dt / 2           (wrapped)
  x'^n+1 = x_h  + (v - v_gal) dt / 2           (wrapped)
  J      = sum q w v S(x_node - x_h) / dV       (lab current)
  rho^n+1= sum q w S(x_node - x'^n+1) / dV
  J^, rho^n+1^ = FFT, with k = 0 and Nyquist planes set to zero
  E^, B^ = Galilean-PSATD update; rho^n^ <- rho^n+1^
  E, B   = inverse FFT
  u      = Boris(u, gather(E, B at x'^n+1), dt)   -> u^{n+3/2}
"""

from dataclasses import dataclass, field

import numpy as np

from . import particles as pt
from . import spectral as sp
from .coefficients import galilean_psatd_coefficients
from .local import SlabSolver


@dataclass
class Grid:
    shape: tuple
    spacing: tuple
    dt: float
    order: int

    @property
    def length(self):
        return np.array([n * d for n, d in zip(self.shape, self.spacing)])

    @property
    def cell_volume(self):
        return self.spacing[0] * self.spacing[1] * self.spacing[2]


@dataclass
class Species:
    q: float
    m: float
    w: float


@dataclass
class State:
    x: np.ndarray            # (n, 3) absolute positions in [0, L)
    u: np.ndarray            # (n, 3) momenta p / (m c) at n + 1/2
    E_hat: tuple             # spectral E^n (3 complex arrays)
    B_hat: tuple             # spectral B^n
    rho_hat: np.ndarray      # spectral rho^n
    E: tuple = field(default=None)   # real-space E^n
    B: tuple = field(default=None)
    J_hat: tuple = field(default=None)      # last deposited current (diagnostic)
    rho_new_hat: np.ndarray = field(default=None)
    step: int = 0


class Simulation:
    """Holds the grid, species, v_gal and the per-mode coefficients."""

    def __init__(self, grid, species, v_gal, c=sp.C_LIGHT, eps0=sp.EPS0,
                 current_correction=False, stencil=(0, 0, 0), slabs=None):
        self.grid = grid
        self.species = species
        self.v_gal = np.asarray(v_gal, dtype=np.float64)
        # optional: J made to satisfy the Galilean continuity equation
        # exactly before the update (spectral.galilean_current_correction)
        self.current_correction = current_correction
        self.c = c
        self.eps0 = eps0
        # per-axis stencil order of the field update (0: exact spectral k);
        # the wavevector then is the stencil's symbol [k]
        self.stencil = tuple(int(p) for p in stencil)
        self.k = sp.wavevectors(grid.shape, grid.spacing, self.stencil)
        self.mask = sp.held_zero_mask(grid.shape)
        self.coef = galilean_psatd_coefficients(self.k, self.v_gal, grid.dt, c, eps0)
        # optional: the field solve on z-slabs with local transforms and
        # guard cells, slabs = (n_slabs, guard) (see ``local``); the state
        # is then the real-space E, B
        self.slab = None
        if slabs is not None:
            self.slab = SlabSolver(grid.shape, grid.spacing, grid.dt, self.v_gal, self.stencil,
                                   slabs[0], slabs[1], c, eps0)

    # -- grid sources -----------------------------------------------------
    def deposit_charge(self, x):
        g, s = self.grid, self.species
        rho = pt.deposit(x, np.ones(x.shape[0]), g.shape, g.spacing, g.order)[0]
        return rho * (s.q * s.w / g.cell_volume)

    def deposit_current(self, x, v):
        g, s = self.grid, self.species
        J = pt.deposit(x, v, g.shape, g.spacing, g.order)
        return J * (s.q * s.w / g.cell_volume)

    def to_spectral_source(self, real):
        spec = sp.forward(real)
        spec[self.mask] = 0.0
        return spec

    # -- set-up -----------------------------------------------------------
    def initial_state(self, x, u, E=None, B=None, project_transverse=False):
        """State from positions, momenta u^{1/2}, and real-space E^0, B^0.

        E^0 and B^0 (default zero) are transformed, with the k = 0 mode and
        Nyquist planes set to zero; with ``project_transverse`` their
        component along k is removed (F <- F - k (k.F) / k^2), which makes
        a sampled laser pulse divergence-free.  rho^0 is deposited at x.
        """
        shape = self.grid.shape
        zeros = np.zeros(shape)
        E = tuple(np.asarray(a, dtype=np.float64) for a in (E if E is not None else (zeros,) * 3))
        B = tuple(np.asarray(a, dtype=np.float64) for a in (B if B is not None else (zeros,) * 3))
        E_hat = tuple(self.to_spectral_source(a) for a in E)
        B_hat = tuple(self.to_spectral_source(a) for a in B)
        if project_transverse:
            E_hat = self._transverse(E_hat)
            B_hat = self._transverse(B_hat)
        rho0 = self.deposit_charge(x)
        rho_hat = self.to_spectral_source(rho0)
        if self.slab is not None:
            self.slab.start(rho0)
        E_real = tuple(sp.inverse(a) for a in E_hat)
        B_real = tuple(sp.inverse(a) for a in B_hat)
        return State(x=np.array(x, dtype=np.float64), u=np.array(u, dtype=np.float64),
                     E_hat=E_hat, B_hat=B_hat, rho_hat=rho_hat, E=E_real, B=B_real)

    def _transverse(self, F):
        k = self.k
        k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2]
        k2 = np.where(k2 == 0.0, 1.0, k2)
        kdotF = (k[0] * F[0] + k[1] * F[1] + k[2] * F[2]) / k2
        return tuple(F[a] - k[a] * kdotF for a in range(3))

    def half_push(self, state):
        """u^0 -> u^{1/2}: Boris push through dt/2 with E^0, B^0 at x'^0."""
        g, s = self.grid, self.species
        F = pt.gather(list(state.E) + list(state.B), state.x, g.shape, g.spacing, g.order)
        state.u = pt.boris_push(state.u, F[:3].T, F[3:].T, s.q, s.m, 0.5 * g.dt, self.c)
        return state

    # -- the step ---------------------------------------------------------
    def step(self, state):
        g, s = self.grid, self.species
        L = g.length
        v = pt.lab_velocity(state.u, self.c)
        x_half = pt.half_move(state.x, v, self.v_gal, g.dt, L)
        x_new = pt.half_move(x_half, v, self.v_gal, g.dt, L)
        J = self.deposit_current(x_half, v)
        rho_new = self.deposit_charge(x_new)
        J_hat = tuple(self.to_spectral_source(J[a]) for a in range(3))
        rho_new_hat = self.to_spectral_source(rho_new)
        if self.slab is not None:
            E, B = self.slab.step(state.E, state.B, J, rho_new)
            F = pt.gather(list(E) + list(B), x_new, g.shape, g.spacing, g.order)
            u_new = pt.boris_push(state.u, F[:3].T, F[3:].T, s.q, s.m, g.dt, self.c)
            return State(x=x_new, u=u_new, E_hat=None, B_hat=None, rho_hat=rho_new_hat,
                         E=E, B=B, J_hat=J_hat, rho_new_hat=rho_new_hat, step=state.step + 1)
        if self.current_correction:
            J_hat = sp.galilean_current_correction(J_hat, state.rho_hat, rho_new_hat, self.k,
                                                   self.v_gal, g.dt, self.mask)
        E_hat, B_hat = sp.galilean_psatd_update(
            state.E_hat, state.B_hat, J_hat, state.rho_hat, rho_new_hat,
            self.k, self.coef, self.mask, self.c)
        E = tuple(sp.inverse(a) for a in E_hat)
        B = tuple(sp.inverse(a) for a in B_hat)
        F = pt.gather(list(E) + list(B), x_new, g.shape, g.spacing, g.order)
        u_new = pt.boris_push(state.u, F[:3].T, F[3:].T, s.q, s.m, g.dt, self.c)
        return State(x=x_new, u=u_new, E_hat=E_hat, B_hat=B_hat, rho_hat=rho_new_hat,
                     E=E, B=B, J_hat=J_hat, rho_new_hat=rho_new_hat, step=state.step + 1)
