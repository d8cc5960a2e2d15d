"""Seeded draws: particle positions and momenta, and the laser envelope.

All draws use numpy's PCG64 generator seeded from the run configuration.
Particles are generated cell by cell (ppc per cell, cell-major order, cell
index (ix * ny + iy) * nz + iz) with in-cell offsets drawn uniformly in
[0, 1) as float32 values, so the absolute position (i + offset) * d is exact
in float64 for the unit spacings used.  Momenta u = p / (m c) are the drift
plus a Gaussian spread, rounded to float32.
"""

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def particles_for(cfg, seed=None, max_particles=None):
    """Seeded particles of a run: dict with

    ``cell`` (n,) int32 linear cell index, ``offset`` (n, 3) float32,
    ``x`` (n, 3) float64 absolute positions (same points), ``u`` (n, 3)
    float64 holding float32-representable momenta, and ``n``.
    ``max_particles`` keeps only the first particles (a prefix of whole
    cells), for bounded samples.
    """
    rng = _rng(cfg.seed if seed is None else seed)
    nx, ny, nz = cfg.shape
    n = cfg.n_particles
    if max_particles is not None:
        n = min(n, (max_particles // cfg.ppc) * cfg.ppc)
    cell = np.repeat(np.arange(n // cfg.ppc, dtype=np.int64), cfg.ppc)
    offset = rng.random((n, 3), dtype=np.float32)
    ix = cell // (ny * nz)
    iy = (cell // nz) % ny
    iz = cell % nz
    x = np.empty((n, 3), dtype=np.float64)
    x[:, 0] = (ix + offset[:, 0].astype(np.float64)) * cfg.spacing[0]
    x[:, 1] = (iy + offset[:, 1].astype(np.float64)) * cfg.spacing[1]
    x[:, 2] = (iz + offset[:, 2].astype(np.float64)) * cfg.spacing[2]
    u = np.zeros((n, 3), dtype=np.float64)
    u[:, 2] = cfg.drift_u()
    if cfg.u_th > 0.0:
        u += cfg.u_th * rng.standard_normal((n, 3))
    u = u.astype(np.float32).astype(np.float64)
    return {"cell": cell.astype(np.int32), "offset": offset, "x": x, "u": u, "n": n}


def split_positions(x, shape, spacing):
    """(cell int32, offset float32) of absolute positions given as float64.

    Used only to hand positions that are already float32-exact offsets to
    the mixed layout (no rounding of the method is involved).
    """
    nx, ny, nz = shape
    s = x / np.asarray(spacing)[None, :]
    i = np.floor(s).astype(np.int64)
    off = (s - i).astype(np.float32)
    i[:, 0] %= nx
    i[:, 1] %= ny
    i[:, 2] %= nz
    cell = (i[:, 0] * ny + i[:, 1]) * nz + i[:, 2]
    return cell.astype(np.int32), off


def laser_fields(cfg):
    """Real-space (E, B) tuples of a Gaussian pulse moving +z, or None.

    E_x = E0 exp(-r^2 / w0^2) exp(-(z - z0)^2 / L^2) cos(k0 (z - z0)),
    B_y = E_x / c, E0 = a0 k0 (m = e = c = 1), centred on the transverse
    axis at z0 = nz / 4 cells.
    """
    if cfg.laser is None:
        return None
    p = cfg.laser
    nx, ny, nz = cfg.shape
    dx, dy, dz = cfg.spacing
    x = (np.arange(nx) - nx / 2) * dx
    y = (np.arange(ny) - ny / 2) * dy
    z = (np.arange(nz) - nz / 4) * dz
    k0 = 2.0 * np.pi / (p["wavelength"] * dz)
    e0 = p["a0"] * k0
    r2 = x[:, None] ** 2 + y[None, :] ** 2
    transverse = np.exp(-r2 / (p["waist"] * dx) ** 2)
    longitudinal = np.exp(-(z / (p["length"] * dz)) ** 2) * np.cos(k0 * z)
    ex = e0 * transverse[:, :, None] * longitudinal[None, None, :]
    zero = np.zeros_like(ex)
    return (ex, zero, zero.copy()), (zero.copy(), ex.copy(), zero.copy())
