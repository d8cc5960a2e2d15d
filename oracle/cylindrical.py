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
* Completing the order m - 1 set (m >= 1): on the zeros of J_m the
  functions J_{m-1}(k_i r) form a Dini series (x J'_{m-1} - (m-1) J_{m-1} =
  0 there), which is complete only with the extra eigenfunction r^{m-1}
  (k_r = 0).  Without it a G_- that does not vanish on average (for m = 1
  a transverse field or current uniform across the axis) is carried by
  large high-k_r coefficients with a wrong divergence, and a particle
  column moving sideways runs away.  So for m >= 1 the last G_- function is
  (r / R)^{m-1} at k_r = 0, and the last k_r column of G_+, G_z and the
  scalars (order m + 1 and m, k = alpha_{m,N_r} / R) is held at zero, like
  a Nyquist plane; at k_r = 0 the Cartesian update keeps G_+ at zero by
  itself (F^_x = i G^_-, F^_y = -G^_-).  The orders m and m + 1 on these
  zeros, and order -1 for m = 0, are complete already.
* The update: the 2D Fourier transform of f(r) exp(i p theta) is
  2 pi (-i)^p exp(i p phi) times the Hankel transform of order p.  At
  azimuth phi = 0 of the wavevector k = (k_r, 0, k_z) the Cartesian
  spectral field of a mode-m state is therefore, up to the factor
  2 pi (-i)^m common to every component and scalar,
      F^_x = i (G^_- - G^_+),  F^_y = -(G^_+ + G^_-),  F^_z = G^_z,
  and the Galilean-PSATD update, covariant under rotations about z for
  v_gal along z, advances the mode as the Cartesian update does at that
  wavevector.  The k_z Nyquist plane is held at zero; k_r > 0 always.
* Particles (deposition and gather by azimuthal mode), a reading of the
  standard azimuthal decomposition with B-spline shapes (linear or cubic)
  in r and z:
  - a stored mode-m field is g_m = c_m f_m, with c_0 = 1 and c_m = 2 for
    m >= 1, where f = sum over all integer m of f_m exp(i m theta); the
    physical field is then Re sum_{m >= 0} g_m exp(i m theta);
  - a particle at (r, theta, z) deposits c_m q w W_j(r) W_k(z)
    exp(-i m theta) s / V_j to node (j, k), with the B-spline weights
    (order 1 or 3) of the radial nodes (j + 1/2) dr and of the z nodes k dz
    (periodic);
  - a node j < 0 (at r = (j + 1/2) dr < 0) is node -j-1 seen across the
    axis (the point at angle theta + pi): its weight goes there with
    s = (-1)^m for scalars and z components and s = (-1)^(m+1) for r and
    theta components (whose unit vectors flip there);
  - V_j = 2 pi dz times the integral of node j's (folded, m = 0) weight
    against r dr: (j + 1/2) dr^2 where the support stays off the axis; for
    linear weights (13/24) dr^2 at j = 0, for cubic ones the integral over
    the folded kernel; so a uniform density deposits uniformly up to the
    axis;
  - a weight reaching past the last node (j >= nr) is dropped;
  - at r = 0 the angle is taken as 0;
  - gather is the transpose: F(x_p) = Re sum_m (sum of W s g_m over the
    nodes) exp(i m theta_p), then the r and theta components are rotated to
    x and y.
  The particle cycle (moves, time-centring, push) is the Cartesian one,
  with z periodic and x, y open.
"""

import functools

import numpy as np
from scipy import special

from . import spectral as sp
from .coefficients import galilean_psatd_coefficients


def radial_grid(nr, dr):
    return (np.arange(nr) + 0.5) * dr


def spectral_kr(m, nr, dr):
    """k_i = alpha_{m,i} / R, the first nr positive zeros of J_m."""
    return special.jn_zeros(m, nr) / (nr * dr)


def held_column(m):
    """True if mode m holds its last k_r column (of G_+, G_z and scalars)
    at zero and carries the k_r = 0 function of G_- there."""
    return m >= 1


def update_kr(m, nr, dr):
    """k_r of each spectral column in the update: the zeros of J_m, with 0
    in the last column of modes that hold it."""
    k = spectral_kr(m, nr, dr)
    if held_column(m):
        k[-1] = 0.0
    return k


def backward_matrix(p, m, nr, dr):
    """M[j, i] = J_p(k_i r_j) on mode m's spectral grid; for p = m - 1 of a
    mode that holds its last column, that column is (r_j / R)^{m-1}."""
    r = radial_grid(nr, dr)
    k = spectral_kr(m, nr, dr)
    M = special.jv(p, np.outer(r, k))
    if held_column(m) and p == m - 1:
        M[:, -1] = (r / (nr * dr)) ** (m - 1)
    return M


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


@functools.lru_cache(maxsize=64)
def _mode_tables(m, nr, dr, nz, dz, v_gal_z, dt):
    kz = axis_kz(nz, dz)[:, None] * np.ones((1, nr))
    kr = np.ones((nz, 1)) * update_kr(m, nr, dr)[None, :]
    k = (kr, np.zeros_like(kr), kz)
    coef = galilean_psatd_coefficients(k, (0.0, 0.0, v_gal_z), dt)
    return k, coef, held_mask(nz, nr)


def hold(G, m):
    """(G_+, G_-, G_z) with the held column of G_+ and G_z zeroed."""
    G = tuple(np.array(a, dtype=complex) for a in G)
    if held_column(m):
        G[0][:, -1] = 0.0
        G[2][:, -1] = 0.0
    return G


def hold_scalar(f, m):
    f = np.array(f, dtype=complex)
    if held_column(m):
        f[:, -1] = 0.0
    return f


def mode_update(E, B, J, rho_old, rho_new, m, nr, dr, nz, dz, v_gal_z, dt):
    """Advance the spectral (G^_+, G^_-, G^_z) of E and B of mode m by one
    Galilean-PSATD step ([k_z][k_r] arrays), through the Cartesian update
    at k = (k_r, 0, k_z) (k_r = 0 in a held column, whose G_+, G_z and
    scalar entries are taken as zero and stay zero)."""
    k, coef, mask = _mode_tables(m, nr, dr, nz, dz, v_gal_z, dt)
    En, Bn = sp.galilean_psatd_update(to_cartesian(hold(E, m)), to_cartesian(hold(B, m)),
                                      to_cartesian(hold(J, m)), hold_scalar(rho_old, m),
                                      hold_scalar(rho_new, m), k, coef, mask)
    return hold(from_cartesian(En), m), hold(from_cartesian(Bn), m)


# ---- particles: deposition and gather by azimuthal mode ----------------------

def mode_factor(m):
    """c_m: 1 for m = 0, 2 for m >= 1 (the stored field is c_m f_m)."""
    return 1.0 if m == 0 else 2.0


def shape_kernel(x, order):
    """The centred B-spline of the given order (1: tent, 3: cubic) at x, in
    units of the node spacing."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    if order == 1:
        return np.maximum(0.0, 1.0 - a)
    if order == 3:
        return np.where(a < 1.0, (4.0 - 6.0 * a * a + 3.0 * a ** 3) / 6.0,
                        np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))
    raise ValueError("shape order must be 1 or 3")


def folded_weight(r, j, dr, order):
    """Node j's weight at radius r >= 0 with the axis fold of m = 0: its
    own kernel plus that of the mirrored node -j-1 (at -(j + 1/2) dr)."""
    return (shape_kernel(r / dr - (j + 0.5), order)
            + shape_kernel(r / dr + (j + 0.5), order))


def node_volumes(nr, dr, dz, order=1):
    """V_j = 2 pi dz * int W_j(r) r dr with the axis fold of m = 0.  Nodes
    whose support stays off the axis give (j + 1/2) dr^2; the others are
    integrated exactly (the folded weight times r is a polynomial between the
    breakpoints (n + 1/2) dr, so 3-point Gauss-Legendre per interval)."""
    v = (np.arange(nr) + 0.5) * dr * dr
    t, wq = np.polynomial.legendre.leggauss(3)
    reach = (order + 1) // 2          # support half-width in nodes
    for j in range(min(reach, nr)):
        edges = np.concatenate([[0.0], (np.arange(j + reach + 1) + 0.5) * dr])
        tot = 0.0
        for a, b in zip(edges[:-1], edges[1:]):
            rr = 0.5 * (b - a) * t + 0.5 * (a + b)
            tot += 0.5 * (b - a) * np.sum(wq * folded_weight(rr, j, dr, order) * rr)
        v[j] = tot
    return 2.0 * np.pi * dz * v


def _angle(x, y):
    """(r, cos theta, sin theta), with theta = 0 at r = 0."""
    r = np.hypot(x, y)
    safe = np.where(r > 0, r, 1.0)
    c = np.where(r > 0, x / safe, 1.0)
    s = np.where(r > 0, y / safe, 0.0)
    return r, c, s


def _nodes(r, z, nr, dr, nz, dz, order=1):
    """Radial nodes (j, may be negative: folded) with weights, and the z
    nodes (periodic), of the B-spline shape of the given order."""
    from .particles import bspline_weights
    sr = r / dr - 0.5
    j0 = np.floor(sr).astype(np.int64)
    wr, rel = bspline_weights(sr - j0, order)
    sz = z / dz
    k0 = np.floor(sz).astype(np.int64)
    wz, relz = bspline_weights(sz - k0, order)
    rad = tuple((j0 + d, wr[:, i]) for i, d in enumerate(rel))
    ax = tuple(((k0 + d) % nz, wz[:, i]) for i, d in enumerate(relz))
    return rad, ax


def deposit_mode(x, y, z, values, m, kind, nr, dr, nz, dz, order=1):
    """c_m sum_p values_p W_j W_k exp(-i m theta_p) s / V_j on the [nz][nr]
    grid of mode m.  kind is "scalar" (scalars and z components) or
    "transverse" (r and theta components), which sets the axis-fold sign;
    a node j < 0 is node -j-1 seen across the axis."""
    r, c, s = _angle(x, y)
    rot = (c - 1j * s) ** m
    vol = node_volumes(nr, dr, dz, order)
    fold = (-1.0) ** m if kind == "scalar" else (-1.0) ** (m + 1)
    out = np.zeros((nz, nr), dtype=complex)
    rad, ax = _nodes(r, z, nr, dr, nz, dz, order)
    for j, wr in rad:
        sign = np.where(j < 0, fold, 1.0)
        jj = np.where(j < 0, -j - 1, j)
        live = jj < nr
        for k, wz in ax:
            val = mode_factor(m) * values * wr * wz * sign * rot
            np.add.at(out, (k[live], jj[live]), val[live])
    return out / vol[None, :]


def gather_mode(g, x, y, z, m, kind, nr, dr, nz, dz, order=1):
    """The complex sum over nodes of W_j W_k s g[k][j] at each particle
    (before the factor exp(i m theta) and the real part)."""
    r, _, _ = _angle(x, y)
    fold = (-1.0) ** m if kind == "scalar" else (-1.0) ** (m + 1)
    acc = np.zeros(len(x), dtype=complex)
    rad, ax = _nodes(r, z, nr, dr, nz, dz, order)
    for j, wr in rad:
        sign = np.where(j < 0, fold, 1.0)
        jj = np.where(j < 0, -j - 1, j)
        live = jj < nr
        jc = np.where(live, jj, 0)
        for k, wz in ax:
            acc += np.where(live, wr * wz * sign * g[k, jc], 0.0)
    return acc


def gather_vector(G, x, y, z, nr, dr, nz, dz, order=1):
    """Cartesian (n, 3) field at the particles from the mode fields
    G[m] = (F_r, F_theta, F_z), each [nz][nr]."""
    r, c, s = _angle(x, y)
    Fr = np.zeros(len(x))
    Ft = np.zeros(len(x))
    Fz = np.zeros(len(x))
    for m, comps in enumerate(G):
        e = (c + 1j * s) ** m
        Fr += np.real(gather_mode(comps[0], x, y, z, m, "transverse", nr, dr, nz, dz, order) * e)
        Ft += np.real(gather_mode(comps[1], x, y, z, m, "transverse", nr, dr, nz, dz, order) * e)
        Fz += np.real(gather_mode(comps[2], x, y, z, m, "scalar", nr, dr, nz, dz, order) * e)
    return np.stack([Fr * c - Ft * s, Fr * s + Ft * c, Fz], axis=1)


def deposit_current(x, y, z, v, qw, nmodes, nr, dr, nz, dz, order=1):
    """Per mode (J_r, J_theta, J_z) [nz][nr] of currents qw v at the points."""
    _, c, s = _angle(x, y)
    vr = v[:, 0] * c + v[:, 1] * s
    vt = -v[:, 0] * s + v[:, 1] * c
    return [(deposit_mode(x, y, z, qw * vr, m, "transverse", nr, dr, nz, dz, order),
             deposit_mode(x, y, z, qw * vt, m, "transverse", nr, dr, nz, dz, order),
             deposit_mode(x, y, z, qw * v[:, 2], m, "scalar", nr, dr, nz, dz, order))
            for m in range(nmodes)]


def deposit_charge(x, y, z, qw, nmodes, nr, dr, nz, dz, order=1):
    return [deposit_mode(x, y, z, qw * np.ones(len(x)), m, "scalar", nr, dr, nz, dz, order)
            for m in range(nmodes)]


def _folded_moment(j, dr, order, upper=np.inf):
    """int_0^upper of node j's folded weight times r.  Between the breakpoints
    (n + 1/2) dr (and the cut at upper) the integrand is a polynomial of
    degree order + 1 <= 4, so 3-point Gauss-Legendre on each piece is exact."""
    reach = (order + 1) // 2
    lo = max(0.0, (j + 0.5 - reach) * dr)
    hi = (j + 0.5 + reach) * dr
    cuts = [(i + 0.5) * dr for i in range(j + reach)] + [upper]
    edges = np.unique([lo, hi] + [c for c in cuts if lo < c < hi])
    t, wq = np.polynomial.legendre.leggauss(3)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        if 0.5 * (a + b) >= upper:
            break
        rr = 0.5 * (b - a) * t + 0.5 * (a + b)
        tot += 0.5 * (b - a) * np.sum(wq * folded_weight(rr, j, dr, order) * rr)
    return tot


def uniform_cylinder_background(density, rp, v_z, nmodes, nr, dr, nz, dz, order=1):
    """Charge and current of a neutralising ion column: charge density
    +density for r < rp, uniform in z and theta, drifting at v_z along z
    (it does not depend on time in either frame).  Node j takes the share of
    its (folded) shape volume inside rp, so that it cancels the deposit of a
    uniform electron column up to the particles' noise.  Returns per mode
    (rho, (J_r, J_theta, J_z)) real-space [nz][nr] arrays (modes >= 1
    zero)."""
    prof = np.array([_folded_moment(j, dr, order, rp) / _folded_moment(j, dr, order)
                     for j in range(nr)])
    rho0 = density * np.ones((nz, 1)) * prof[None, :] + 0j
    zero = np.zeros((nz, nr), dtype=complex)
    out = []
    for m in range(nmodes):
        if m == 0:
            out.append((rho0, (zero, zero, v_z * rho0)))
        else:
            out.append((zero, (zero, zero, zero)))
    return out


class CylindricalPIC:
    """The Galilean-PSATD particle cycle in azimuthal modes, in the order of
    the Cartesian cycle: with u at n - 1/2, move x half a step with
    v - v_gal, deposit J there with v, move the second half, deposit rho^{n+1},
    transform, update every mode, transform back, gather at x^{n+1} and push
    (relativistic Boris).  z is periodic; x and y are open."""

    def __init__(self, nz, nr, nmodes, dz, dr, dt, q, mass, w, v_gal_z, background=None,
                 order=1):
        """background: optional per-mode (rho, (J_r, J_theta, J_z)) added to
        the deposits every step (e.g. a neutralising ion column); order: the
        particle shape (1 linear, 3 cubic) in r and z."""
        self.order = order
        self.nz, self.nr, self.nmodes = nz, nr, nmodes
        self.dz, self.dr, self.dt = dz, dr, dt
        self.q, self.mass, self.w = q, mass, w
        self.v_gal_z = v_gal_z
        self.background = background

    def _with_background(self, rho, J):
        if self.background is None:
            return rho, J
        bg = self.background
        rho = [rho[m] + bg[m][0] for m in range(self.nmodes)]
        if J is not None:
            J = [tuple(J[m][a] + bg[m][1][a] for a in range(3)) for m in range(self.nmodes)]
        return rho, J

    def _move(self, x, v):
        h = 0.5 * self.dt
        out = x + h * (v - np.array([0.0, 0.0, self.v_gal_z]))
        out[:, 2] = np.mod(out[:, 2], self.nz * self.dz)
        return out

    def electrostatic_field(self, rho_hat, m):
        """Spectral (G^_+, G^_-, G^_z) of the field with i k.E = rho and no
        curl: E^_c = -i k rho^ / |k|^2 at k = (k_r, 0, k_z), through the
        Cartesian map (every mode has k_r > 0; the held k_z row stays 0)."""
        kz = axis_kz(self.nz, self.dz)[:, None] * np.ones((1, self.nr))
        kr = np.ones((self.nz, 1)) * update_kr(m, self.nr, self.dr)[None, :]
        k2 = kr * kr + kz * kz
        rho = hold_scalar(rho_hat, m)
        live = ~held_mask(self.nz, self.nr) & (k2 > 0)
        safe = np.where(k2 > 0, k2, 1.0)
        Ec = tuple(np.where(live, -1j * ka * rho / safe, 0.0)
                   for ka in (kr, np.zeros_like(kr), kz))
        return hold(from_cartesian(Ec), m)

    def initial_state(self, x, u, E=None, B=None, electrostatic=False):
        """x, u (n, 3); optional real mode fields E, B [m] = (r, theta, z);
        electrostatic: E^0 is the field of the initial charge instead."""
        rho = deposit_charge(x[:, 0], x[:, 1], x[:, 2], self.q * self.w, self.nmodes,
                             self.nr, self.dr, self.nz, self.dz, self.order)
        rho, _ = self._with_background(rho, None)
        zero = np.zeros((self.nz, self.nr), dtype=complex)
        Eh, Bh = [], []
        for m in range(self.nmodes):
            e = E[m] if E is not None else (zero, zero, zero)
            b = B[m] if B is not None else (zero, zero, zero)
            Eh.append(to_spectral(e, m, self.dr, self.dz))
            Bh.append(to_spectral(b, m, self.dr, self.dz))
        rh = [scalar_to_spectral(rho[m], m, self.dr, self.dz) for m in range(self.nmodes)]
        if electrostatic:
            Eh = [self.electrostatic_field(rh[m], m) for m in range(self.nmodes)]
        return {"x": x.copy(), "u": u.copy(), "E_hat": Eh, "B_hat": Bh, "rho_hat": rh,
                "E": None, "B": None}

    def step(self, st):
        from .particles import boris_push, lab_velocity
        nz, nr, dz, dr, nm = self.nz, self.nr, self.dz, self.dr, self.nmodes
        qw = self.q * self.w
        v = lab_velocity(st["u"])
        xh = self._move(st["x"], v)
        xn = self._move(xh, v)
        o = self.order
        J = deposit_current(xh[:, 0], xh[:, 1], xh[:, 2], v, qw, nm, nr, dr, nz, dz, o)
        rho = deposit_charge(xn[:, 0], xn[:, 1], xn[:, 2], qw, nm, nr, dr, nz, dz, o)
        rho, J = self._with_background(rho, J)
        Eh, Bh, rh, E, B = [], [], [], [], []
        for m in range(nm):
            Jh = to_spectral(J[m], m, dr, dz)
            r1 = scalar_to_spectral(rho[m], m, dr, dz)
            en, bn = mode_update(st["E_hat"][m], st["B_hat"][m], Jh, st["rho_hat"][m], r1,
                                 m, nr, dr, nz, dz, self.v_gal_z, self.dt)
            Eh.append(en)
            Bh.append(bn)
            rh.append(r1)
            E.append(from_spectral(en, m, dr, dz))
            B.append(from_spectral(bn, m, dr, dz))
        Ep = gather_vector(E, xn[:, 0], xn[:, 1], xn[:, 2], nr, dr, nz, dz, o)
        Bp = gather_vector(B, xn[:, 0], xn[:, 1], xn[:, 2], nr, dr, nz, dz, o)
        un = boris_push(st["u"], Ep, Bp, self.q, self.mass, self.dt)
        return {"x": xn, "u": un, "E_hat": Eh, "B_hat": Bh, "rho_hat": rh, "E": E, "B": B,
                "J": J, "rho": rho}


def field_energy(G, nr, dr, dz, order=1):
    """sum_m sum_nodes V_j |g_m|^2 / c_m over the components of real mode
    fields G[m] = (F_r, F_theta, F_z), with the node volumes of the shape
    order: a norm for growth diagnostics."""
    vol = node_volumes(nr, dr, dz, order)
    return float(sum(np.sum(vol[None, :] * np.abs(a) ** 2) / mode_factor(m)
                     for m, comps in enumerate(G) for a in comps))
