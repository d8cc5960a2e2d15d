"""Field energy, Gauss and continuity residuals (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Field energy W = 1/2 sum (|E|^2 + |B|^2) dV in normalised units
  (eps0 = c = 1).
* Gauss residual i k.E - rho / eps0 per mode.
* Continuity residual of the Galilean continuity equation
  (d_t - v_gal.grad') rho + div' j = 0 integrated over one step with j held
  constant in the Galilean coordinates (the co-moving current assumption):
      rho^{n+1} - theta^2 rho^n - (1 - theta^2) (k.J) / (k.v_gal),
  whose k.v_gal -> 0 limit is rho^{n+1} - rho^n + i dt k.J.
"""

import numpy as np

from . import spectral as sp


def field_energy(E, B, cell_volume):
    """(W_E, W_B) for real-space fields."""
    we = 0.5 * cell_volume * sum(float(np.sum(a * a)) for a in E)
    wb = 0.5 * cell_volume * sum(float(np.sum(a * a)) for a in B)
    return we, wb


def gauss_residual(E_hat, rho_hat, k, eps0=sp.EPS0):
    return 1j * (k[0] * E_hat[0] + k[1] * E_hat[1] + k[2] * E_hat[2]) - rho_hat / eps0


def divergence_b(B_hat, k):
    return 1j * (k[0] * B_hat[0] + k[1] * B_hat[1] + k[2] * B_hat[2])


def continuity_residual(rho_old, rho_new, J_hat, k, v_gal, dt):
    kdotv = k[0] * v_gal[0] + k[1] * v_gal[1] + k[2] * v_gal[2]
    kdotJ = k[0] * J_hat[0] + k[1] * J_hat[1] + k[2] * J_hat[2]
    theta2 = np.exp(1j * kdotv * dt)
    small = np.abs(kdotv * dt) < 1e-300
    safe = np.where(small, 1.0, kdotv)
    # (1 - theta^2) / (k.v) evaluated without cancellation:
    # 1 - e^{i a} = -2 i sin(a/2) e^{i a/2}, a = k.v dt.
    half = 0.5 * kdotv * dt
    factor = np.where(small, -1j * dt,
                      -2j * np.sin(half) * np.exp(1j * half) / safe)
    return rho_new - theta2 * rho_old - factor * kdotJ
