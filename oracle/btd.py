"""Back-transformation of boosted-frame fields to lab-frame snapshots
(oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper obtains its lab-frame results from the boosted-frame run by an
on-the-fly back-transformation and names it the only overhead of the
boosted run, without writing the procedure down.  Readings taken here:

* The boosted frame moves at +beta c along z relative to the lab, and the
  Galilean frame is the one in which the plasma, at rest in the lab, is at
  rest: v_gal = (0, 0, -beta c).  A grid node z'_k = k dz of the Galilean
  grid at boosted time t' sits at z_b = z'_k - beta c t' in the boosted
  frame, so the Lorentz transformation back to the lab gives
      z_lab = gamma (z_b + beta c t') = gamma z'_k       (fixed in time),
      t_lab = gamma (t' + beta z_b / c) = t' / gamma + gamma beta z'_k / c.
  The lab snapshot at time t_j therefore takes, at lab plane z_lab =
  gamma z'_k, the fields of Galilean plane k at boosted time
      t'_jk = gamma t_j - gamma^2 beta z'_k / c.
* The fields at t'_jk are the linear interpolation in time of the two
  stored levels t'_n < t'_jk <= t'_{n+1} (levels t'_n = t'_0 + n dt); a
  plane whose t'_jk lies outside the stored levels is not filled.
* Particles are recorded where their worldline over a step, taken as the
  straight segment of the move with the momentum that made it, crosses a
  snapshot's lab time (``particle_crossings``).
* E and B of the Galilean grid are the boosted-frame fields (a Galilean
  change of coordinates leaves their values alone); the lab fields follow
  from the Lorentz transformation of the field tensor with the lab frame
  moving at -beta c relative to the boosted one:
      E_x = gamma (E'_x + beta c B'_y),   E_y = gamma (E'_y - beta c B'_x),
      B_x = gamma (B'_x - beta E'_y / c), B_y = gamma (B'_y + beta E'_x / c),
      E_z = E'_z, B_z = B'_z.
"""

import numpy as np

from .spectral import C_LIGHT


def lorentz_to_lab(E, B, beta, c=C_LIGHT):
    """Lab-frame (E, B) from boosted-frame (E', B') for a boost +beta c z."""
    g = 1.0 / np.sqrt(1.0 - beta * beta)
    El = (g * (E[0] + beta * c * B[1]), g * (E[1] - beta * c * B[0]), E[2])
    Bl = (g * (B[0] - beta * E[1] / c), g * (B[1] + beta * E[0] / c), B[2])
    return El, Bl


def plane_time(t_lab, k, dz, beta, c=C_LIGHT):
    """Boosted time t'_jk at which Galilean plane k is at lab time t_lab."""
    g = 1.0 / np.sqrt(1.0 - beta * beta)
    return g * t_lab - g * g * beta * (k * dz) / c


def back_transform(levels, t0, dt, t_snap, dz, beta, c=C_LIGHT):
    """Lab-frame snapshots from stored boosted levels.

    ``levels[n]`` = (E, B), six real arrays [x][y][z] at t'_0 + n dt.
    Returns (snap, filled): snap[j] is a tuple of six lab arrays on the
    snapshot's planes (zero where not filled), filled[j][k] tells whether
    plane k of snapshot j lies inside the stored levels."""
    nz = levels[0][0][0].shape[2]
    nlev = len(levels)
    snaps, filled = [], []
    for tj in t_snap:
        out = [np.zeros_like(levels[0][0][0]) for _ in range(6)]
        got = np.zeros(nz, dtype=bool)
        for k in range(nz):
            tp = plane_time(tj, k, dz, beta, c)
            for n in range(nlev - 1):
                lo, hi = t0 + n * dt, t0 + (n + 1) * dt
                if lo < tp <= hi:
                    w = (tp - lo) / dt
                    E = [(1 - w) * levels[n][0][a][:, :, k] + w * levels[n + 1][0][a][:, :, k]
                         for a in range(3)]
                    B = [(1 - w) * levels[n][1][a][:, :, k] + w * levels[n + 1][1][a][:, :, k]
                         for a in range(3)]
                    El, Bl = lorentz_to_lab(E, B, beta, c)
                    for f, v in enumerate(list(El) + list(Bl)):
                        out[f][:, :, k] = v
                    got[k] = True
                    break
        snaps.append(tuple(out))
        filled.append(got)
    return snaps, filled


def particle_crossings(x_new, u_move, dt, t_new, v_gal_z, t_snap, length, c=C_LIGHT,
                       fractions=False):
    """Lab-frame records of the particles whose worldline over one step
    crosses a snapshot's lab time.

    The step ends at boosted time t_new with each particle at x_new
    (Galilean, in the box [0, L)), having moved by (v - v_gal) dt with
    v = c u / gamma_p of the momentum u_move that moved it.  Its worldline
    over the step is the segment ending there,
        x(s) = x_new - (1 - s) (v - v_gal) dt,  t'(s) = t_new - (1 - s) dt,
    0 <= s <= 1 (the copy of the periodic box that holds the end; the lab
    time depends on which copy).  Along it t_lab(s) = t'(s) / gamma +
    gamma beta z(s) / c (beta = -v_gal_z / c) increases strictly (|v| < c);
    snapshot j is crossed when t_lab(0) < t_j <= t_lab(1), at
    s_j = (t_j - t_lab(0)) / (t_lab(1) - t_lab(0)).  The record holds the
    position there (wrapped to the box; z scaled to the lab plane gamma z)
    and the lab momentum u_x, u_y, gamma (u_z + beta gamma_p).  Returns, per
    snapshot, (index, values) with values[:, 0:6] = x, y, z_lab, u_x, u_y,
    u_z; with fractions, (index, values, s_j) (a crossing with s_j near 0 or
    1 lies within rounding of the adjacent step's)."""
    beta = -v_gal_z / c
    g = 1.0 / np.sqrt(1.0 - beta * beta)
    gp = np.sqrt(1.0 + np.sum(u_move * u_move, axis=1))
    v = c * u_move / gp[:, None]
    step = (v - np.array([0.0, 0.0, v_gal_z])[None, :]) * dt
    ta = (t_new - dt) / g + g * beta * (x_new[:, 2] - step[:, 2]) / c
    tb = t_new / g + g * beta * x_new[:, 2] / c
    out = []
    L = np.asarray(length, dtype=np.float64)
    for tj in t_snap:
        hit = np.nonzero((ta < tj) & (tj <= tb))[0]
        s = (tj - ta[hit]) / (tb[hit] - ta[hit])
        pos = x_new[hit] - (1.0 - s)[:, None] * step[hit]
        pos = pos - np.floor(pos / L[None, :]) * L[None, :]
        u = u_move[hit]
        vals = np.stack([pos[:, 0], pos[:, 1], g * pos[:, 2], u[:, 0], u[:, 1],
                         g * (u[:, 2] + beta * gp[hit])], axis=1)
        out.append((hit, vals, s) if fractions else (hit, vals))
    return out
