"""Spectral grid, transforms and the Galilean-PSATD field update (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (readings of points the paper leaves silent):

* Fourier convention: forward transform with kernel exp(-i k.x), inverse
  normalised by 1/N (``numpy.fft.fftn`` / ``ifftn``).  With it the spatial
  derivative with respect to the Galilean coordinates becomes +i k, which is
  the convention under which the printed theta = exp(i k.v_gal dt / 2) is
  consistent with the transformed Maxwell equations.
* k is the exact spectral wavevector 2 pi m / L per axis (pseudo-spectral)
  unless a finite stencil order is asked for: then every spatial derivative
  of the update, the curls, the divergences in the charge terms and the
  Galilean advection v_gal.grad in theta alike, uses the symbol [k] of the
  centered difference of that order on the colocated grid (the paper names
  arbitrary-order spectral solvers only as future work; this reading
  replaces k by [k] everywhere in the field update and nowhere else).
* Grid quantities are colocated on the nodes x_i = i * d (no staggering).
* The k = 0 mode and every Nyquist plane (index N_a / 2 on any axis) of the
  sources and of the fields are held at zero.  On Nyquist planes the update
  does not map a Hermitian spectrum to a Hermitian spectrum, and the k = 0
  mode carries the mean current of the electrons, which the co-moving
  neutralising ion background cancels.
"""

from fractions import Fraction
from math import factorial

import numpy as np

C_LIGHT = 1.0
EPS0 = 1.0


def axis_wavenumbers(n, d):
    """k values of one axis in FFT index order: 2 pi * fftfreq(n, d)."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d)


def centered_difference_weights(half_width):
    """Weights a_1 .. a_M (M = half_width) of the centered first-derivative
    stencil of order 2M on a colocated grid,

        (D f)_i = (1 / d) sum_{l=1}^{M} a_l (f_{i+l} - f_{i-l}),

    the unique one exact for polynomials of degree 2M:
    a_l = (-1)^(l+1) (M!)^2 / (l (M - l)! (M + l)!), computed exactly."""
    M = int(half_width)
    return [float(Fraction((-1) ** (l + 1) * factorial(M) ** 2,
                           l * factorial(M - l) * factorial(M + l)))
            for l in range(1, M + 1)]


def modified_wavenumbers(n, d, order):
    """Symbol [k] of one axis in FFT index order: D exp(i k x) = i [k]
    exp(i k x) for the centered stencil of even ``order`` 2M,
    [k] = (2 / d) sum_l a_l sin(l k d).  ``order`` 0 is the exact k."""
    k = axis_wavenumbers(n, d)
    if order == 0:
        return k
    if order < 2 or order % 2:
        raise ValueError("stencil order must be 0 or even and >= 2")
    a = centered_difference_weights(order // 2)
    return (2.0 / d) * sum(al * np.sin(l * k * d) for l, al in enumerate(a, start=1))


def wavevectors(shape, spacing, stencil=(0, 0, 0)):
    """Full (C2C) wavevector grid, each component shaped like the grid;
    ``stencil`` gives each axis's stencil order (0: exact k)."""
    ks = [modified_wavenumbers(n, d, p) for n, d, p in zip(shape, spacing, stencil)]
    return np.meshgrid(*ks, indexing="ij")


def held_zero_mask(shape):
    """True on the k = 0 mode and on every Nyquist plane."""
    mask = np.zeros(shape, dtype=bool)
    mask[0, 0, 0] = True
    for axis, n in enumerate(shape):
        if n % 2 == 0:
            index = [slice(None)] * 3
            index[axis] = n // 2
            mask[tuple(index)] = True
    return mask


def forward(field):
    """Unnormalised forward DFT, kernel exp(-i k.x)."""
    return np.fft.fftn(np.asarray(field, dtype=np.float64))


def inverse(spectrum):
    """Inverse DFT normalised by 1/N; the real part of a Hermitian spectrum."""
    return np.fft.ifftn(spectrum).real


def cross(a, b):
    """Component-wise cross product of two 3-vectors of arrays."""
    return (a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0])


def galilean_psatd_update(E, B, J, rho_old, rho_new, k, coef, mask, c=C_LIGHT):
    """Advance spectral E and B by one step (Galilean-PSATD update).

    Written from the paper's update display for B^{n+1} and E^{n+1}:

      B' = theta^2 C B - (theta^2 S / (c k)) i k x E
           + theta chi_1 / (eps0 c^2 k^2) i k x J
      E' = theta^2 C E + (theta^2 S / k) c i k x B
           + (i nu theta chi_1 - theta^2 S) / (eps0 c k) J
           - (chi_2 rho^{n+1} - theta^2 chi_3 rho^n) i k / (eps0 k^2)

    ``coef`` holds those products per mode under the names
    c_EE (= theta^2 C), s (= theta^2 S / (c k)), c_BJ, c_EJ,
    c_R1 (= -chi_2 / (eps0 k^2)) and c_R0 (= +theta^2 chi_3 / (eps0 k^2)),
    see ``coefficients.galilean_psatd_coefficients``.  J is taken at
    (n + 1/2) dt, rho_old at n dt and rho_new at (n + 1) dt.  Modes in
    ``mask`` are set to zero.  Returns new (E, B) as 3-tuples.
    """
    ik = tuple(1j * ka for ka in k)
    ik_x_E = cross(ik, E)
    ik_x_B = cross(ik, B)
    ik_x_J = cross(ik, J)
    rho_term = coef["c_R1"] * rho_new + coef["c_R0"] * rho_old
    B_new = []
    E_new = []
    for a in range(3):
        b = coef["c_EE"] * B[a] - coef["s"] * ik_x_E[a] + coef["c_BJ"] * ik_x_J[a]
        e = (coef["c_EE"] * E[a] + c * c * coef["s"] * ik_x_B[a]
             + coef["c_EJ"] * J[a] + rho_term * ik[a])
        b = np.where(mask, 0.0, b)
        e = np.where(mask, 0.0, e)
        B_new.append(b)
        E_new.append(e)
    return tuple(E_new), tuple(B_new)


def galilean_current_correction(J, rho_old, rho_new, k, v_gal, dt, mask):
    """Current with its longitudinal part replaced so that the Galilean
    continuity equation holds exactly over the step.

    The transformed equations carry the continuity equation
    (d_t - v_gal.grad') rho + div' j = 0; in k-space (grad' -> +i k) with J
    held constant over the step it integrates to

        rho^{n+1} = theta^2 rho^n + F (k.J),   F = (1 - theta^2) / (k.v_gal),

    theta^2 = exp(i k.v_gal dt), with F -> -i dt as k.v_gal -> 0.  The
    deposited J need not satisfy it; the corrected current keeps the
    transverse part of J and takes the longitudinal component k.J_c =
    (rho^{n+1} - theta^2 rho^n) / F:  J_c = J + k (k.J_c - k.J) / k^2.
    F is written as -i dt theta sinc(k.v_gal dt / 2), theta = exp(i k.v_gal
    dt / 2), which has no 0/0.  Modes in ``mask`` (k = 0, Nyquist planes)
    are returned as zero.  Not part of the printed update: an option.
    """
    kdotv = k[0] * v_gal[0] + k[1] * v_gal[1] + k[2] * v_gal[2]
    half = 0.5 * kdotv * dt
    theta = np.exp(1j * half)
    sinc = np.sinc(half / np.pi)              # sin(half) / half, 1 at 0
    F = -1j * dt * theta * sinc
    k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2]
    safe_k2 = np.where(mask, 1.0, k2)
    safe_F = np.where(mask, 1.0, F)
    kdotJ = k[0] * J[0] + k[1] * J[1] + k[2] * J[2]
    target = (rho_new - theta * theta * rho_old) / safe_F
    alpha = (target - kdotJ) / safe_k2
    return tuple(np.where(mask, 0.0, J[a] + alpha * k[a]) for a in range(3))
