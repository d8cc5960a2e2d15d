"""Particle shapes, deposition, gather, position advance and push (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings of what the paper leaves open (it says the currents at (n + 1/2) dt
and the charge densities at n dt and (n + 1) dt are deposited to the grid
nodes, the fields are interpolated back to the particles, and the particles
advance with the Galilean-transformed equations of motion):

* Shapes are cardinal B-splines per axis, tensor-multiplied over x, y, z:
  order 1 (cloud-in-cell) or order 3 (the paper's runs use third-order
  shapes).  A particle at node coordinate i + delta (0 <= delta < 1) touches
  nodes i, i+1 (order 1) or i-1 .. i+2 (order 3), periodically wrapped.
* The cell of a position is floor(x / d) wrapped into [0, N); the offset is
  x / d - cell.
* Gather uses the same shape as deposition (so the two are adjoint).
* Positions move with dx'/dt = v - v_gal (v = p / (gamma m) the lab-frame
  velocity), as two half moves of dt/2: J is deposited at the half-way
  position with q w v, rho at the end position with q w.
* Momentum: relativistic Boris rotation with u = p / (m c), using the lab
  E and B interpolated at the new position.
"""

import numpy as np

from .spectral import C_LIGHT


def bspline_weights(delta, order):
    """1D shape weights for in-cell offsets ``delta`` (shape (n,)).

    Returns (weights (n, order+1), node offsets relative to the cell).
    """
    d = np.asarray(delta, dtype=np.float64)
    if order == 1:
        return np.stack([1.0 - d, d], axis=1), np.array([0, 1])
    if order == 3:
        one_minus = 1.0 - d
        d2 = d * d
        d3 = d2 * d
        w = np.stack([
            one_minus * one_minus * one_minus / 6.0,
            (4.0 - 6.0 * d2 + 3.0 * d3) / 6.0,
            (1.0 + 3.0 * d + 3.0 * d2 - 3.0 * d3) / 6.0,
            d3 / 6.0,
        ], axis=1)
        return w, np.array([-1, 0, 1, 2])
    raise ValueError("shape order must be 1 or 3")


def cell_and_offset(x, n, d):
    """Cell index (wrapped to [0, n)) and in-cell offset for positions x."""
    s = np.asarray(x, dtype=np.float64) / d
    cell = np.floor(s)
    offset = s - cell
    return np.mod(cell.astype(np.int64), n), offset


def _node_lists(positions, shape, spacing, order):
    """Per axis: (node indices (n, order+1), weights (n, order+1))."""
    out = []
    for axis in range(3):
        cell, off = cell_and_offset(positions[:, axis], shape[axis], spacing[axis])
        w, rel = bspline_weights(off, order)
        nodes = np.mod(cell[:, None] + rel[None, :], shape[axis])
        out.append((nodes, w))
    return out


def deposit(positions, values, shape, spacing, order):
    """Scatter per-particle ``values`` (n, q) to the nodes: sum of value * S.

    Returns an array (q, *shape).  Division by the cell volume and the charge
    factors are the caller's (``deposit_current`` / ``deposit_charge``).
    """
    values = np.asarray(values, dtype=np.float64)
    if values.ndim == 1:
        values = values[:, None]
    (nx, wx), (ny, wy), (nz, wz) = _node_lists(positions, shape, spacing, order)
    ncell = shape[0] * shape[1] * shape[2]
    out = np.zeros((values.shape[1], ncell), dtype=np.float64)
    m = order + 1
    for a in range(m):
        for b in range(m):
            wab = wx[:, a] * wy[:, b]
            base = (nx[:, a] * shape[1] + ny[:, b]) * shape[2]
            for g in range(m):
                idx = base + nz[:, g]
                w = wab * wz[:, g]
                for q in range(values.shape[1]):
                    out[q] += np.bincount(idx, weights=w * values[:, q], minlength=ncell)
    return out.reshape((values.shape[1],) + tuple(shape))


def gather(fields, positions, shape, spacing, order):
    """Interpolate each grid field in ``fields`` (list of arrays) to positions."""
    (nx, wx), (ny, wy), (nz, wz) = _node_lists(positions, shape, spacing, order)
    flat = [np.asarray(f, dtype=np.float64).ravel() for f in fields]
    out = np.zeros((len(fields), positions.shape[0]), dtype=np.float64)
    m = order + 1
    for a in range(m):
        for b in range(m):
            wab = wx[:, a] * wy[:, b]
            base = (nx[:, a] * shape[1] + ny[:, b]) * shape[2]
            for g in range(m):
                idx = base + nz[:, g]
                w = wab * wz[:, g]
                for i, f in enumerate(flat):
                    out[i] += w * f[idx]
    return out


def lorentz_factor(u):
    """gamma = sqrt(1 + |u|^2) for u = p / (m c), u shaped (n, 3)."""
    return np.sqrt(1.0 + np.sum(u * u, axis=1))


def lab_velocity(u, c=C_LIGHT):
    """v = p / (gamma m) = c u / gamma."""
    return c * u / lorentz_factor(u)[:, None]


def wrap(x, length):
    """Periodic wrap of positions into [0, length) per axis."""
    x = np.mod(x, length)
    return np.where(x >= length, x - length, x)


def half_move(x, v, v_gal, dt, length):
    """x' += (v - v_gal) dt / 2, wrapped: the Galilean equation of motion."""
    return wrap(x + (v - np.asarray(v_gal)[None, :]) * (0.5 * dt), length)


def boris_push(u, E, B, q, m, dt, c=C_LIGHT):
    """Relativistic Boris push of u = p / (m c) through dt with lab E, B.

    E and B are (n, 3).  h = q dt / (2 m c); u- = u + h E; gamma- =
    sqrt(1 + |u-|^2); t = h c B / gamma-; s = 2 t / (1 + |t|^2);
    u' = u- + u- x t; u+ = u- + u' x s; result u+ + h E.
    """
    h = q * dt / (2.0 * m * c)
    u_minus = u + h * E
    gamma = np.sqrt(1.0 + np.sum(u_minus * u_minus, axis=1))
    t = (h * c) * B / gamma[:, None]
    s = 2.0 * t / (1.0 + np.sum(t * t, axis=1))[:, None]
    u_prime = u_minus + np.cross(u_minus, t)
    u_plus = u_minus + np.cross(u_prime, s)
    return u_plus + h * E
