"""Galilean-PSATD coefficients C, S, nu, theta, chi_1, chi_2, chi_3 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper prints closed forms (coefficient block under the update equations):

  C = cos(c k dt), S = sin(c k dt), nu = k.v_gal / (c k),
  theta = exp(i k.v_gal dt / 2),
  chi_1 = (theta* - C theta + i nu theta S) / (1 - nu^2),
  chi_2 = (chi_1 - theta (1 - C)) / (theta* - theta),
  chi_3 = (chi_1 - theta* (1 - C)) / (theta* - theta).

As printed they are 0/0 on every mode with k.v_gal = 0 and lose most of
their digits when k is nearly parallel to a relativistic v_gal (1 - nu^2 ~
1/gamma^2) or when c k dt is small.  The oracle therefore evaluates the same
quantities through the Duhamel integrals that the closed forms are the
antiderivatives of.  With phi = c k dt and the substitution y = c k tau
(tau in [0, dt] the time since the start of the step):

  A1 = int_0^phi sin(y) e^{i nu y} dy                         = theta chi_1
  A2 = int_0^phi cos(y) e^{i nu y} dy                         = theta^2 S - i nu theta chi_1
  A3 = int_0^phi 2 sin^2(y/2) e^{i nu y} dy                   = chi_2 D
  A4 = int_0^phi 2 sin((phi+y)/2) sin((phi-y)/2) e^{i nu y} dy = -chi_3 D
  D  = int_0^phi e^{i nu y} dy                                = (theta^2 - 1) / (i nu)

(The identities follow by integrating by parts; the tests check each one
against the printed closed forms evaluated in 50-digit arithmetic.)  Every
integrand is a product of bounded factors with no cancelling difference, so
composite Gauss-Legendre quadrature evaluates them to full FP64 accuracy.
A1 and A2 are the B- and E-responses to a current that is constant in the
Galilean coordinates (the co-moving current assumption).

The update then uses, per mode with k != 0:

  c_EE = theta^2 C                      (multiplies E and B)
  s    = theta^2 S / (c k)              (B gets -s ik x E, E gets +c^2 s ik x B)
  c_BJ = theta chi_1 / (eps0 c^2 k^2)   = A1 / (eps0 c^2 k^2)
  c_EJ = (i nu theta chi_1 - theta^2 S) / (eps0 c k) = -A2 / (eps0 c k)
  c_R1 = -chi_2 / (eps0 k^2)            (multiplies rho^{n+1} i k)
  c_R0 = +theta^2 chi_3 / (eps0 k^2)    (multiplies rho^n i k)

At k = 0 the finite limits are stored (c_EE = 1, s = dt, c_BJ = dt^2 /
(2 eps0), c_EJ = -dt / eps0, c_R1 = -c^2 dt^2 / (6 eps0), c_R0 = -c^2 dt^2 /
(3 eps0)); that mode is held at zero by the update anyway.

The printed form is singular where theta* = theta with k.v_gal != 0, i.e.
|k.v_gal| dt = 2 pi m; there D = 0 and the rho-form has no solution.
``max_galilean_phase`` reports the largest |k.v_gal| dt of a grid so callers
can reject such grids.
"""

import numpy as np

from .spectral import C_LIGHT, EPS0

#: Gauss-Legendre points per panel; panels are at most PANEL_LENGTH long in y.
GL_POINTS = 16
PANEL_LENGTH = 1.0


def _gauss_legendre_unit(n):
    """Gauss-Legendre nodes and weights on [0, 1] (numpy's leggauss)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def duhamel_integrals(phi, nu, points=GL_POINTS, panel_length=PANEL_LENGTH):
    """Return (A1, A2, A3, A4, D) for arrays phi >= 0 and nu (same shape).

    Composite Gauss-Legendre: [0, phi] is split into P equal panels with
    P = ceil(max(phi) / panel_length), so each panel is at most
    ``panel_length`` long, and each panel gets ``points`` nodes.
    """
    phi = np.asarray(phi, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    shape = np.broadcast(phi, nu).shape
    phi = np.broadcast_to(phi, shape).ravel()
    nu = np.broadcast_to(nu, shape).ravel()
    t, w = _gauss_legendre_unit(points)
    n_panels = max(1, int(np.ceil(phi.max(initial=0.0) / panel_length)))
    out = [np.zeros(phi.shape, dtype=np.complex128) for _ in range(5)]
    chunk = 1 << 15
    for lo in range(0, phi.size, chunk):
        p = phi[lo:lo + chunk, None]
        v = nu[lo:lo + chunk, None]
        h = p / n_panels
        acc = [np.zeros(p.shape[0], dtype=np.complex128) for _ in range(5)]
        for panel in range(n_panels):
            y = h * (panel + t[None, :])
            phase = np.exp(1j * v * y)
            wh = h * w[None, :]
            sin_half = np.sin(0.5 * y)
            f1 = np.sin(y)
            f2 = np.cos(y)
            f3 = 2.0 * sin_half * sin_half
            f4 = 2.0 * np.sin(0.5 * (p + y)) * np.sin(0.5 * (p - y))
            for i, f in enumerate((f1, f2, f3, f4, np.ones_like(y))):
                acc[i] += np.sum(wh * f * phase, axis=1)
        for i in range(5):
            out[i][lo:lo + chunk] = acc[i]
    return tuple(o.reshape(shape) for o in out)


def galilean_psatd_coefficients(k, v_gal, dt, c=C_LIGHT, eps0=EPS0):
    """Per-mode update coefficients (dict of complex128 arrays).

    ``k`` is a 3-tuple of wavevector component arrays, ``v_gal`` a 3-vector.
    Keys: c_EE, s, c_BJ, c_EJ, c_R1, c_R0 (see module docstring), plus the
    intermediate theta, C, S, nu, chi1, chi2, chi3 for tests.
    """
    kx, ky, kz = (np.asarray(a, dtype=np.float64) for a in k)
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    kdotv = kx * v_gal[0] + ky * v_gal[1] + kz * v_gal[2]
    zero = kmag == 0.0
    ksafe = np.where(zero, 1.0, kmag)
    phi = c * kmag * dt
    nu = np.where(zero, 0.0, kdotv / (c * ksafe))
    A1, A2, A3, A4, D = duhamel_integrals(phi, nu)
    theta = np.exp(0.5j * kdotv * dt)
    theta2 = theta * theta
    C = np.cos(phi)
    S = np.sin(phi)
    Dsafe = np.where(zero, 1.0, D)
    chi2 = A3 / Dsafe
    chi3 = -A4 / Dsafe
    chi1 = A1 / theta
    k2 = ksafe * ksafe
    coef = {
        "c_EE": theta2 * C,
        "s": np.where(zero, dt, theta2 * S / (c * ksafe)),
        "c_BJ": np.where(zero, 0.5 * dt * dt / eps0, A1 / (eps0 * c * c * k2)),
        "c_EJ": np.where(zero, -dt / eps0, -A2 / (eps0 * c * ksafe)),
        "c_R1": np.where(zero, -c * c * dt * dt / (6.0 * eps0), -chi2 / (eps0 * k2)),
        "c_R0": np.where(zero, -c * c * dt * dt / (3.0 * eps0), theta2 * chi3 / (eps0 * k2)),
        "theta": theta, "C": C, "S": S, "nu": nu,
        "chi1": np.where(zero, 0.0, chi1),
        "chi2": np.where(zero, 0.0, chi2),
        "chi3": np.where(zero, 0.0, chi3),
    }
    for key in ("c_EE", "s", "c_BJ", "c_EJ", "c_R1", "c_R0"):
        coef[key] = np.asarray(coef[key], dtype=np.complex128)
    return coef


def max_galilean_phase(shape, spacing, v_gal, dt):
    """Largest |k.v_gal| dt over the non-Nyquist modes of a grid."""
    total = 0.0
    for n, d, v in zip(shape, spacing, v_gal):
        m = n // 2 - 1 if n % 2 == 0 else (n - 1) // 2
        total += abs(v) * 2.0 * np.pi * m / (n * d)
    return total * dt
