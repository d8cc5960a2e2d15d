"""Quasi-cylindrical (azimuthal-mode) Galilean-PSATD field solve (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's own runs use a quasi-3D spectral code: fields are expanded in
azimuthal modes, and discrete Hankel transforms along r take the place of
the transverse Fourier transforms; it states that the Galilean scheme does
not depend on the geometry.  It does not write the cylindrical algorithm
down.  Readings taken here:

* A mode m field is F(r, theta, z) = F_m(r, z) exp(i m theta) (complex
  profiles; the physical field is the real part of the sum over modes).
  Its components combine as G_+ = (F_r + i F_theta) / 2 and G_- = (F_r -
  i F_theta) / 2, since F_x + i F_y = 2 G_+ exp(i (m+1) theta) and
  F_x - i F_y = 2 G_- exp(i (m-1) theta): G_+ is a Hankel field of order
  m+1, G_- of order m-1, F_z and scalars of order m.
* Grid: periodic in z (nodes z_k = k dz, forward kernel exp(-i k_z z)),
  radial nodes r_j = (j + 1/2) dr, j < N_r, R = N_r dr.  One spectral
  grid per mode for all three orders: k_i = alpha_{m,i} / R, the positive
  zeros of J_m.  Backward (spectral -> radial) transform of order p:
  F(r_j) = sum_i F^_i J_p(k_i r_j); the forward transform is its matrix
  inverse.
* The update: the 2D Fourier transform of f(r) exp(i p theta) is
  2 pi (-i)^p exp(i p phi) times the Hankel transform of order p.  At
  azimuth phi = 0 of the wavevector k = (k_r, 0, k_z) the Cartesian
  spectral field of a mode-m state is therefore, up to the factor
  2 pi (-i)^m common to every component and scalar,
      F^_x = i (G^_- - G^_+),  F^_y = -(G^_+ + G^_-),  F^_z = G^_z,
  and the Galilean-PSATD update, covariant under rotations about z for
  v_gal along z, advances the mode as the Cartesian update does at that
  wavevector.  The k_z Nyquist plane is held at zero; k_r > 0 always.
* Particles (deposition and gather in azimuthal modes) are not part of
  this option.
"""

import numpy as np
from scipy import special

from . import spectral as sp
from .coefficients import galilean_psatd_coefficients


def radial_grid(nr, dr):
    return (np.arange(nr) + 0.5) * dr


def spectral_kr(m, nr, dr):
    """k_i = alpha_{m,i} / R, the first nr positive zeros of J_m."""
    return special.jn_zeros(m, nr) / (nr * dr)


def backward_matrix(p, m, nr, dr):
    """M[j, i] = J_p(k_i r_j) on mode m's spectral grid."""
    r = radial_grid(nr, dr)
    k = spectral_kr(m, nr, dr)
    return special.jv(p, np.outer(r, k))


def forward_matrix(p, m, nr, dr):
    return np.linalg.inv(backward_matrix(p, m, nr, dr))


def axis_kz(nz, dz):
    return sp.axis_wavenumbers(nz, dz)


def to_spectral(F, m, dr, dz):
    """Spectral (G^_+, G^_-, G^_z) of a mode-m vector field given as
    (F_r, F_theta, F_z), each complex [z][r]; arrays [k_z][k_r]."""
    nz, nr = F[0].shape
    Fz = [np.fft.fft(a, axis=0) for a in F]
    gp = 0.5 * (Fz[0] + 1j * Fz[1])
    gm = 0.5 * (Fz[0] - 1j * Fz[1])
    H = lambda p, a: a @ forward_matrix(p, m, nr, dr).T
    return H(m + 1, gp), H(m - 1, gm), H(m, Fz[2])


def from_spectral(G, m, dr, dz):
    """(F_r, F_theta, F_z) [z][r] of spectral (G^_+, G^_-, G^_z)."""
    nz, nr = G[0].shape
    B = lambda p, a: a @ backward_matrix(p, m, nr, dr).T
    gp, gm, fz = B(m + 1, G[0]), B(m - 1, G[1]), B(m, G[2])
    Fr = gp + gm
    Ft = -1j * (gp - gm)
    return tuple(np.fft.ifft(a, axis=0) for a in (Fr, Ft, fz))


def scalar_to_spectral(f, m, dr, dz):
    nz, nr = f.shape
    return np.fft.fft(f, axis=0) @ forward_matrix(m, m, nr, dr).T


def scalar_from_spectral(g, m, dr, dz):
    nz, nr = g.shape
    return np.fft.ifft(g @ backward_matrix(m, m, nr, dr).T, axis=0)


def to_cartesian(G):
    """Cartesian spectral vector at azimuth 0 of (G^_+, G^_-, G^_z)."""
    gp, gm, gz = G
    return (1j * (gm - gp), -(gp + gm), gz)


def from_cartesian(F):
    fx, fy, fz = F
    return (0.5j * (fx + 1j * fy), -0.5j * (fx - 1j * fy), fz)


def held_mask(nz, nr):
    mask = np.zeros((nz, nr), dtype=bool)
    mask[nz // 2, :] = True
    return mask


def mode_update(E, B, J, rho_old, rho_new, m, nr, dr, nz, dz, v_gal_z, dt):
    """Advance the spectral (G^_+, G^_-, G^_z) of E and B of mode m by one
    Galilean-PSATD step ([k_z][k_r] arrays), through the Cartesian update
    at k = (k_r, 0, k_z)."""
    kz = axis_kz(nz, dz)[:, None] * np.ones((1, nr))
    kr = np.ones((nz, 1)) * spectral_kr(m, nr, dr)[None, :]
    k = (kr, np.zeros_like(kr), kz)
    v = (0.0, 0.0, v_gal_z)
    coef = galilean_psatd_coefficients(k, v, dt)
    mask = held_mask(nz, nr)
    En, Bn = sp.galilean_psatd_update(to_cartesian(E), to_cartesian(B), to_cartesian(J),
                                      rho_old, rho_new, k, coef, mask)
    return from_cartesian(En), from_cartesian(Bn)
