"""Helpers of the GPU parity tests at full size (not collected by pytest):
read a sample of particles by id straight from the device arrays, find the
particles that can reach a window of grid nodes, and the oracle's particle
pass (gather, Boris push, the two half moves, the deposits) for a subset of
particles, with the fields the library holds as input."""

import numpy as np

from oracle import particles as opt

FIELDS6 = ("EX", "EY", "EZ", "BX", "BY", "BZ")


def _positions_dev(parts, cfg, idx=None):
    """Absolute float64 positions (n, 3) of the particles at device indices
    idx (all if None), as a torch tensor on the device."""
    import torch

    take = (lambda t: t) if idx is None else (lambda t: t[idx])
    if parts.off is None:
        return torch.stack([take(t) for t in parts.pos], dim=1)
    nx, ny, nz = cfg.shape
    cell = take(parts.pos[0]).to(torch.int64)
    ijk = torch.stack([cell // (ny * nz), (cell // nz) % ny, cell % nz], dim=1)
    off = torch.stack([take(t).to(torch.float64) for t in parts.off], dim=1)
    d = torch.tensor(cfg.spacing, dtype=torch.float64, device=off.device)
    return (ijk.to(torch.float64) + off) * d[None, :]


def state_of(parts, cfg, ids):
    """(positions, momenta) of the particles with the given ids, float64
    numpy arrays in the order of ids."""
    import torch

    pid = parts.ids
    inv = torch.empty_like(pid)
    inv[pid] = torch.arange(pid.numel(), device=pid.device)
    idx = inv[torch.as_tensor(np.asarray(ids, dtype=np.int64), device=pid.device)]
    x = _positions_dev(parts, cfg, idx).cpu().numpy()
    u = torch.stack([t[idx].to(torch.float64) for t in parts.u], dim=1).cpu().numpy()
    return x, u


def ids_near(parts, cfg, lo, hi):
    """Ids of the particles whose position lies in the periodic box
    [lo, hi) (grid-node units per axis, hi - lo below the box length)."""
    import torch

    x = _positions_dev(parts, cfg)
    d = torch.tensor(cfg.spacing, dtype=torch.float64, device=x.device)
    L = torch.tensor(cfg.shape, dtype=torch.float64, device=x.device)
    s = x / d[None, :]
    lo_t = torch.tensor(lo, dtype=torch.float64, device=x.device)
    width = torch.tensor(np.asarray(hi, float) - np.asarray(lo, float), dtype=torch.float64,
                         device=x.device)
    rel = torch.remainder(s - lo_t[None, :], L[None, :])
    keep = torch.all(rel < width[None, :], dim=1)
    return parts.ids[keep].cpu().numpy()


def read_fields(ctx, run, names=FIELDS6):
    return [ctx.read_field(run, n).astype(np.float64) for n in names]


def oracle_pass(cfg, x, u, F, dt_factor=1.0, v_gal=None):
    """The oracle's particle pass from (x, u) with real fields F (6 arrays):
    u' = Boris(u, gather(F at x), dt), v = c u' / gamma, x_h and x' the two
    half moves.  Returns (u', v, x_h, x')."""
    vg = cfg.v_gal() if v_gal is None else v_gal
    L = np.array(cfg.shape) * np.array(cfg.spacing)
    G = opt.gather(F, x, cfg.shape, cfg.spacing, cfg.order)
    un = opt.boris_push(u, G[:3].T, G[3:].T, cfg.q, cfg.m, dt_factor * cfg.dt)
    v = opt.lab_velocity(un)
    xh = opt.half_move(x, v, vg, cfg.dt, L)
    xn = opt.half_move(xh, v, vg, cfg.dt, L)
    return un, v, xh, xn


def oracle_moves(cfg, x, u, v_gal=None):
    """The deposit's half moves from (x, u): (v, x_h, x')."""
    vg = cfg.v_gal() if v_gal is None else v_gal
    L = np.array(cfg.shape) * np.array(cfg.spacing)
    v = opt.lab_velocity(u)
    xh = opt.half_move(x, v, vg, cfg.dt, L)
    return v, xh, opt.half_move(xh, v, vg, cfg.dt, L)


def window_reference(cfg, corner, xh, v, xn, width=4):
    """J (3 arrays) and rho of the particles (x_h, v, x') on the width^3
    nodes from corner (periodic), deposited one by one by the oracle on a
    local box around the window (the particles farther away cannot reach
    it), so that no full-size grid is needed."""
    lo, hi = window_sources(cfg, corner, width)
    W = int(hi[0] - lo[0]) + 1
    d = np.asarray(cfg.spacing, float)
    Lc = np.asarray(cfg.shape, float)

    reach = float(corner[0] - lo[0])
    # local coordinates in [-reach, L - reach): a particle that moved below
    # the box start (by at most 2 cells) stays just below it
    assert np.all(Lc >= W + reach + 2), "grid too small for a local window box"

    def local(x):
        s = x / d[None, :] - lo[None, :]
        return np.mod(s + reach, Lc[None, :]) - reach

    qw = cfg.q * cfg.w / (cfg.spacing[0] * cfg.spacing[1] * cfg.spacing[2])
    sh, sn = local(xh), local(xn)
    keep_h = np.all((sh >= 0) & (sh < W), axis=1)
    keep_n = np.all((sn >= 0) & (sn < W), axis=1)
    box = (W, W, W)
    J = opt.deposit(sh[keep_h], v[keep_h], box, (1.0, 1.0, 1.0), cfg.order) * qw
    rho = opt.deposit(sn[keep_n], np.ones(int(keep_n.sum())), box, (1.0, 1.0, 1.0),
                      cfg.order)[0] * qw
    off = int(round(corner[0] - lo[0]))
    sl = (slice(off, off + width),) * 3
    return [J[a][sl] for a in range(3)], rho[sl]


def window_index(cfg, corner, width=4):
    nodes = tuple((np.asarray(corner)[:, None] + np.arange(width)[None, :])
                  % np.array(cfg.shape)[:, None])
    return np.ix_(*nodes)


def window_sources(cfg, corner, width=4):
    """The periodic box of particle positions (before a pass that moves them
    at most |v - v_gal| dt <= 2 cells) that can reach the window's nodes:
    the shape's support plus the move, with one cell to spare."""
    reach = (cfg.order + 1) // 2 + 1 + 2 + 1
    lo = np.asarray(corner, float) - reach
    hi = np.asarray(corner, float) + (width - 1) + reach
    return lo, hi


def momentum_bar(u_got, u_ref, u_before, rel_u, rel_du):
    """Per particle |u_got - u_ref| <= rel_u |u_before| + rel_du |u_ref - u_before|
    (the rounding of the stored momentum plus that of the kick); returns the
    largest ratio of the error to its bar."""
    err = np.linalg.norm(u_got - u_ref, axis=1)
    bar = rel_u * np.linalg.norm(u_before, axis=1) + rel_du * np.linalg.norm(u_ref - u_before,
                                                                              axis=1) + 1e-300
    return float(np.max(err / bar)) if len(err) else 0.0


def periodic_max_diff(a, b, cfg):
    L = np.array(cfg.shape) * np.array(cfg.spacing)
    d = np.abs(np.asarray(a) - np.asarray(b))
    d = np.minimum(d, L[None, :] - d)
    return float(d.max()) if d.size else 0.0


def full_from_half(h, shape):
    """The full spectrum [x][y][z] of a real field from its half spectrum
    [x][y][z/2+1] (Hermitian symmetry F(-k) = conj F(k))."""
    nx, ny, nz = shape
    h = np.asarray(h, dtype=np.complex128)
    full = np.empty((nx, ny, nz), dtype=np.complex128)
    full[:, :, : nz // 2 + 1] = h
    ix = (-np.arange(nx)) % nx
    iy = (-np.arange(ny)) % ny
    kz = np.arange(nz // 2 + 1, nz)
    full[:, :, kz] = np.conj(h[np.ix_(ix, iy, nz - kz)])
    return full


def sample_modes(shape, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    nzh = shape[2] // 2 + 1
    return (rng.integers(0, shape[0], n), rng.integers(0, shape[1], n), rng.integers(0, nzh, n))


def half_k_at(idx, shape, spacing):
    from oracle import spectral as osp

    ix, iy, iz = idx
    kx = osp.axis_wavenumbers(shape[0], spacing[0])[ix]
    ky = osp.axis_wavenumbers(shape[1], spacing[1])[iy]
    kz = 2 * np.pi * iz / (shape[2] * spacing[2])
    return kx, ky, kz


def held_at(idx, shape):
    ix, iy, iz = idx
    return ((ix == shape[0] // 2) | (iy == shape[1] // 2) | (iz == shape[2] // 2) |
            ((ix == 0) & (iy == 0) & (iz == 0)))


SPECTRA = ("EX_HAT", "EY_HAT", "EZ_HAT", "BX_HAT", "BY_HAT", "BZ_HAT", "JX_HAT", "JY_HAT",
           "JZ_HAT", "RHO_HAT_OLD", "RHO_HAT_NEW")


def update_reference(cfg, spectra, idx):
    """The oracle's update at the sampled modes idx of the half spectrum,
    from the library's input spectra (dict by selector name)."""
    from oracle import coefficients as oco
    from oracle import spectral as osp

    k = half_k_at(idx, cfg.shape, cfg.spacing)
    coef = oco.galilean_psatd_coefficients(k, cfg.v_gal(), cfg.dt)
    take = lambda n: np.asarray(spectra[n])[idx].astype(np.complex128)
    E = tuple(take("E" + c + "_HAT") for c in "XYZ")
    B = tuple(take("B" + c + "_HAT") for c in "XYZ")
    J = tuple(take("J" + c + "_HAT") for c in "XYZ")
    return osp.galilean_psatd_update(E, B, J, take("RHO_HAT_OLD"), take("RHO_HAT_NEW"), k,
                                     coef, held_at(idx, cfg.shape))


def update_scale(cfg, spectra, idx):
    """Per sampled mode, the sum of the magnitudes of the terms of the
    update (|c||input| over every term, with |k| for the curls and the
    charge terms): the size against which the float rounding of inputs and
    coefficients is measured, since cancellation can make the result far
    smaller than its terms."""
    from oracle import coefficients as oco

    k = half_k_at(idx, cfg.shape, cfg.spacing)
    kmag = np.sqrt(k[0] ** 2 + k[1] ** 2 + k[2] ** 2)
    coef = oco.galilean_psatd_coefficients(k, cfg.v_gal(), cfg.dt)
    take = lambda n: np.abs(np.asarray(spectra[n])[idx].astype(np.complex128))
    E = np.sqrt(sum(take("E" + c + "_HAT") ** 2 for c in "XYZ"))
    B = np.sqrt(sum(take("B" + c + "_HAT") ** 2 for c in "XYZ"))
    J = np.sqrt(sum(take("J" + c + "_HAT") ** 2 for c in "XYZ"))
    a = lambda key: np.abs(coef[key])
    return ((E + B) * (a("c_EE") + a("s") * kmag) + J * (a("c_BJ") * kmag + a("c_EJ"))
            + kmag * (a("c_R1") * take("RHO_HAT_NEW") + a("c_R0") * take("RHO_HAT_OLD")))


def check_update(ctx, run, cfg, spectra, idx, tol):
    """E^, B^ after the update at the sampled modes against the oracle's
    update of the library's inputs, each component within tol of the
    update's term scale (L2 over the modes)."""
    En, Bn = update_reference(cfg, spectra, idx)
    scale = float(np.linalg.norm(update_scale(cfg, spectra, idx)))
    for a, c in enumerate("XYZ"):
        for name, ref in (("E" + c + "_HAT", En[a]), ("B" + c + "_HAT", Bn[a])):
            got = ctx.read_field(run, name)[idx].astype(np.complex128)
            err = float(np.linalg.norm(got - ref))
            assert err <= tol * scale, (run, name, err / scale)
