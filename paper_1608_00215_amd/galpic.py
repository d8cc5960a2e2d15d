"""ctypes binding of ``libgalpic.so`` (argument marshalling only).

Every step of the method runs in the HIP kernels behind the C ABI declared
in ``include/galpic.h``; this module only converts Python arguments to
pointers and sizes.  PyTorch provides device memory for the particle
arrays.  There is no fallback: if the library is missing, ``load()``
raises.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgalpic.so")

GP_OK, GP_ERR_ARG, GP_ERR_STATE, GP_ERR_HIP, GP_ERR_UNSTABLE, GP_ERR_OOM = 0, -1, -2, -3, -4, -5
GP_FP64, GP_MIXED = 0, 1

FIELDS = ["EX", "EY", "EZ", "BX", "BY", "BZ", "JX", "JY", "JZ", "RHO",
          "EX_HAT", "EY_HAT", "EZ_HAT", "BX_HAT", "BY_HAT", "BZ_HAT",
          "JX_HAT", "JY_HAT", "JZ_HAT", "RHO_HAT_OLD", "RHO_HAT_NEW",
          "COEF0", "COEF1", "COEF2", "COEF3", "COEF4", "COEF5"]
FIELD = {name: i for i, name in enumerate(FIELDS)}

#: every symbol the header declares
EXPORTS = ["gp_init_grid", "gp_set_v_gal", "gp_set_current_correction", "gp_set_local_slabs",
           "gp_bind_particles", "gp_deposit", "gp_fft_fwd",
           "gp_galilean_psatd_update", "gp_fft_inv", "gp_gather_push",
           "gp_gather_push_deposit", "gp_step",
           "gp_step_graph", "gp_set_fields", "gp_half_push", "gp_read_field",
           "gp_write_field", "gp_field_ptr", "gp_field_energy", "gp_field_energy_noalloc", "gp_last_graph_ms", "gp_synchronize",
           "gp_stage_timing", "gp_stage_times", "gp_stage_name", "gp_sort_count",
           "gp_run", "gp_destroy", "gp_last_error", "gp_btd_configure", "gp_btd_record",
           "gp_btd_particles", "gp_qc_init", "gp_qc_set_v_gal", "gp_qc_write", "gp_qc_read",
           "gp_qc_fields_fwd", "gp_qc_sources_fwd", "gp_qc_init_rho", "gp_qc_update",
           "gp_qc_fields_inv", "gp_qc_step", "gp_qc_synchronize", "gp_qc_destroy",
           "gp_qc_wavenumbers", "gp_qc_hankel_matrix", "gp_qc_stage_timing",
           "gp_qc_stage_times", "gp_qc_set_background", "gp_qc_bind_particles",
           "gp_qc_electrostatic_fields", "gp_qc_particle_step", "gp_qc_set_resort"]
QC_FIELDS = ["ER", "ET", "EZ", "BR", "BT", "BZ", "JR", "JT", "JZ", "RHO",
             "E_PLUS", "E_MINUS", "E_Z_HAT", "B_PLUS", "B_MINUS", "B_Z_HAT",
             "J_PLUS", "J_MINUS", "J_Z_HAT", "RHO_HAT_OLD", "RHO_HAT_NEW",
             "COEF0", "COEF1", "COEF2", "COEF3", "COEF4", "COEF5"]
QC_FIELD = {name: i for i, name in enumerate(QC_FIELDS)}
QC_STAGES = ["z_fwd", "hankel_fwd", "update", "hankel_bwd", "z_inv", "deposit",
             "gather_push"]
GP_N_STAGES = 16


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("dt", ctypes.c_double), ("shape_order", ctypes.c_int),
                ("precision", ctypes.c_int), ("tile", ctypes.c_int * 3),
                ("resort_div", ctypes.c_int), ("stencil", ctypes.c_int * 3),
                ("flush", ctypes.c_int)]


class QcParticlesC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_double), ("m", ctypes.c_double),
                ("w", ctypes.c_double),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("uz", ctypes.c_void_p)]


class QcDesc(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int), ("nr", ctypes.c_int), ("nmodes", ctypes.c_int),
                ("dz", ctypes.c_double), ("dr", ctypes.c_double), ("dt", ctypes.c_double),
                ("precision", ctypes.c_int), ("shape_order", ctypes.c_int)]


class ParticlesC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_double), ("m", ctypes.c_double),
                ("w", ctypes.c_double),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("off_x", ctypes.c_void_p), ("off_y", ctypes.c_void_p),
                ("off_z", ctypes.c_void_p),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("uz", ctypes.c_void_p),
                ("id", ctypes.c_void_p)]


class GalpicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"galpic status {status}: {msg}")
        self.status = status


_LIB = None


def load(path=LIB_PATH):
    """Load the library (once) and declare argument types."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_1608_00215_amd.build` (no CPU fallback exists)")
    # torch first: its HIP runtime then also serves the library (the same
    # soname), so the process holds one runtime and torch's streams and
    # allocations are the library's
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "gp_init_grid": [ctypes.POINTER(GridDesc), i32, vp, ctypes.POINTER(vp)],
        "gp_set_v_gal": [vp, i32, dbl, dbl, dbl],
        "gp_set_current_correction": [vp, i32],
        "gp_set_local_slabs": [vp, i32, i32],
        "gp_bind_particles": [vp, vp],
        "gp_deposit": [vp, vp],
        "gp_fft_fwd": [vp],
        "gp_galilean_psatd_update": [vp],
        "gp_fft_inv": [vp],
        "gp_gather_push": [vp, vp],
        "gp_gather_push_deposit": [vp, vp],
        "gp_step": [vp, vp],
        "gp_step_graph": [vp, vp, i32],
        "gp_set_fields": [vp, i32, vp, vp, i32],
        "gp_half_push": [vp, vp],
        "gp_read_field": [vp, i32, i32, vp],
        "gp_write_field": [vp, i32, i32, vp],
        "gp_field_ptr": [vp, i32, i32, ctypes.POINTER(vp)],
        "gp_field_energy": [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)],
        "gp_field_energy_noalloc": [vp, i32, vp],
        "gp_last_graph_ms": [vp, ctypes.POINTER(dbl)],
        "gp_synchronize": [vp],
        "gp_stage_timing": [vp, i32],
        "gp_stage_times": [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32)],
        "gp_sort_count": [vp, i32, ctypes.POINTER(i32)],
        "gp_run": [vp, vp, i32],
        "gp_destroy": [vp],
        "gp_btd_configure": [vp, i32, i32, dbl, dbl, dbl, vp],
        "gp_btd_record": [vp],
        "gp_btd_particles": [vp, i32, i32, vp, vp, vp],
        "gp_qc_init": [ctypes.POINTER(QcDesc), vp, ctypes.POINTER(vp)],
        "gp_qc_set_v_gal": [vp, dbl],
        "gp_qc_write": [vp, i32, vp],
        "gp_qc_read": [vp, i32, vp],
        "gp_qc_fields_fwd": [vp],
        "gp_qc_sources_fwd": [vp],
        "gp_qc_init_rho": [vp],
        "gp_qc_update": [vp],
        "gp_qc_fields_inv": [vp],
        "gp_qc_step": [vp, i32],
        "gp_qc_synchronize": [vp],
        "gp_qc_destroy": [vp],
        "gp_qc_wavenumbers": [i32, i32, dbl, vp],
        "gp_qc_stage_timing": [vp, i32],
        "gp_qc_set_background": [vp, vp, vp, vp, vp],
        "gp_qc_bind_particles": [vp, ctypes.POINTER(QcParticlesC)],
        "gp_qc_electrostatic_fields": [vp],
        "gp_qc_particle_step": [vp, i32],
        "gp_qc_set_resort": [vp, i32],
        "gp_qc_stage_times": [vp, vp, vp],
        "gp_qc_hankel_matrix": [i32, i32, i32, dbl, i32, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.gp_last_error.argtypes = []
    lib.gp_last_error.restype = ctypes.c_char_p
    lib.gp_stage_name.argtypes = [i32]
    lib.gp_stage_name.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _init_torch_first():
    """Let PyTorch initialise the HIP runtime before the library touches it,
    so torch tensors and the library share one device context."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def _check(lib, status):
    if status != GP_OK:
        raise GalpicError(status, lib.gp_last_error().decode())


class Particles:
    """Device arrays of one run's particles (torch tensors, caller-owned).

    FP64: x, y, z absolute positions (float64).  Mixed: ``cell`` int32 linear
    index and offsets (float32).  Momenta u (float64 or float32); optional
    int64 ids carried through reorderings.
    """

    def __init__(self, precision, q, m, w, u, x=None, cell=None, offset=None, ids=None,
                 device="cuda"):
        import torch

        self.precision = precision
        self.q, self.m, self.w = float(q), float(m), float(w)
        if precision == GP_FP64:
            dt = torch.float64
            x = np.asarray(x, dtype=np.float64)
            self.pos = [torch.tensor(np.ascontiguousarray(x[:, a]), device=device) for a in range(3)]
            self.off = None
            self.n = x.shape[0]
        else:
            dt = torch.float32
            self.pos = [torch.tensor(np.ascontiguousarray(cell, dtype=np.int32), device=device)]
            off = np.asarray(offset, dtype=np.float32)
            self.off = [torch.tensor(np.ascontiguousarray(off[:, a]), device=device)
                        for a in range(3)]
            self.n = off.shape[0]
        u = np.asarray(u)
        self.u = [torch.tensor(np.ascontiguousarray(u[:, a]), dtype=dt, device=device)
                  for a in range(3)]
        self.ids = None if ids is None else torch.tensor(np.asarray(ids, dtype=np.int64),
                                                         device=device)

    def c_struct(self):
        p = ParticlesC()
        p.n = self.n
        p.q, p.m, p.w = self.q, self.m, self.w
        ptr = lambda t: t.data_ptr() if (t is not None and t.numel() > 0) else None
        if self.precision == GP_FP64:
            p.x, p.y, p.z = (ptr(t) for t in self.pos)
        else:
            p.x = ptr(self.pos[0])
            p.off_x, p.off_y, p.off_z = (ptr(t) for t in self.off)
        p.ux, p.uy, p.uz = (ptr(t) for t in self.u)
        p.id = ptr(self.ids) if self.ids is not None else None
        if self.n == 0:
            # zero-length tensors may have no storage; pass a dummy pointer
            p.x = p.x or 1
        return p

    def positions(self, shape=None, spacing=None):
        """Absolute positions (n, 3) as float64 numpy (host copy)."""
        if self.precision == GP_FP64:
            return np.stack([t.cpu().numpy() for t in self.pos], axis=1)
        nx, ny, nz = shape
        cell = self.pos[0].cpu().numpy().astype(np.int64)
        off = np.stack([t.cpu().numpy().astype(np.float64) for t in self.off], axis=1)
        ix = cell // (ny * nz)
        iy = (cell // nz) % ny
        iz = cell % nz
        d = np.asarray(spacing, dtype=np.float64)
        return (np.stack([ix, iy, iz], axis=1) + off) * d[None, :]

    def momenta(self):
        return np.stack([t.cpu().numpy().astype(np.float64) for t in self.u], axis=1)

    def id_array(self):
        return None if self.ids is None else self.ids.cpu().numpy()


class Context:
    """One gp_ctx: n_runs runs of one precision and shape order."""

    def __init__(self, grids, stream=None):
        """grids: list of dicts with nx, ny, nz, dx, dy, dz, dt, order, precision."""
        self.lib = load()
        _init_torch_first()
        n = len(grids)
        arr = (GridDesc * n)()
        for i, g in enumerate(grids):
            tile = (ctypes.c_int * 3)(*g.get("tile", (0, 0, 0)))
            stencil = (ctypes.c_int * 3)(*g.get("stencil", (0, 0, 0)))
            arr[i] = GridDesc(g["nx"], g["ny"], g["nz"], g.get("dx", 1.0), g.get("dy", 1.0),
                              g.get("dz", 1.0), g["dt"], g["order"], g["precision"], tile,
                              g.get("resort_div", 0), stencil, g.get("flush", 0))
        self.grids = grids
        self.precision = grids[0]["precision"]
        self.real = np.float64 if self.precision == GP_FP64 else np.float32
        self.cplx = np.complex128 if self.precision == GP_FP64 else np.complex64
        handle = ctypes.c_void_p()
        _check(self.lib, self.lib.gp_init_grid(arr, n, stream, ctypes.byref(handle)))
        self.h = handle
        self._parts = None
        self._parts_c = None

    # -- lifecycle -------------------------------------------------------------
    def close(self):
        if self.h:
            self.lib.gp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        _check(self.lib, getattr(self.lib, name)(self.h, *args))

    # -- the C ABI, one method per call ---------------------------------------
    def set_v_gal(self, run, v):
        self._call("gp_set_v_gal", int(run), float(v[0]), float(v[1]), float(v[2]))

    def set_current_correction(self, enable):
        self._call("gp_set_current_correction", 1 if enable else 0)

    def set_local_slabs(self, n_slabs, guard):
        """Field solve on z-slabs with local transforms and guard cells
        (gp_set_local_slabs); n_slabs = 0 returns to the global solve."""
        self._call("gp_set_local_slabs", int(n_slabs), int(guard))

    def bind_particles(self, parts):
        import torch

        torch.cuda.synchronize()
        self._parts = list(parts)
        arr = (ParticlesC * len(parts))()
        for i, p in enumerate(parts):
            arr[i] = p.c_struct()
        self._parts_c = arr
        self._call("gp_bind_particles", arr)

    def deposit(self):
        self._call("gp_deposit", self._parts_c)

    def fft_fwd(self):
        self._call("gp_fft_fwd")

    def galilean_psatd_update(self):
        self._call("gp_galilean_psatd_update")

    def fft_inv(self):
        self._call("gp_fft_inv")

    def gather_push(self):
        self._call("gp_gather_push", self._parts_c)

    def gather_push_deposit(self):
        self._call("gp_gather_push_deposit", self._parts_c)

    def half_push(self):
        self._call("gp_half_push", self._parts_c)

    def step(self):
        self._call("gp_step", self._parts_c)

    def step_graph(self, nsteps):
        self._call("gp_step_graph", self._parts_c, int(nsteps))

    def last_graph_ms(self):
        ms = ctypes.c_double()
        self._call("gp_last_graph_ms", ctypes.byref(ms))
        return ms.value

    def synchronize(self):
        self._call("gp_synchronize")

    def stage_timing(self, enable=True):
        self._call("gp_stage_timing", 1 if enable else 0)

    def stage_times(self):
        """{stage name: (summed ms, launches)} recorded since timing was enabled."""
        ms = (ctypes.c_double * GP_N_STAGES)()
        n = (ctypes.c_int * GP_N_STAGES)()
        self._call("gp_stage_times", ms, n)
        names = [self.lib.gp_stage_name(i).decode() for i in range(GP_N_STAGES)]
        return {nm: (ms[i], n[i]) for i, nm in enumerate(names)}

    def sort_count(self, run=0):
        n = ctypes.c_int()
        self._call("gp_sort_count", int(run), ctypes.byref(n))
        return n.value

    def run(self, nsteps):
        self._call("gp_run", self._parts_c, int(nsteps))

    def btd_configure(self, run, n_snap, t_lab0, dt_lab, t_boost0=0.0):
        """Record lab-frame snapshots of run (gp_btd_configure) into a device
        tensor [n_snap][6][nz][nx][ny] (plane-major) that this object
        allocates, keeps alive while recording, and returns; n_snap = 0
        stops recording."""
        import torch

        if not hasattr(self, "_btd"):
            self._btd = {}
        g = self.grids[run]
        out = None
        ptr = None
        if n_snap > 0:
            dtype = torch.float64 if self.precision == GP_FP64 else torch.float32
            out = torch.empty((n_snap, 6, g["nz"], g["nx"], g["ny"]), dtype=dtype,
                              device="cuda")
            ptr = out.data_ptr()
        self._call("gp_btd_configure", int(run), int(n_snap), float(t_lab0), float(dt_lab),
                   float(t_boost0), ptr)
        if n_snap == 0:
            self._call("gp_synchronize")
        self._btd[run] = out
        return out

    def btd_particles(self, run, cap, with_ids=True):
        """Lab-frame particle records of run (gp_btd_particles): returns
        device tensors (vals [n_snap][6][cap], ids [n_snap][cap] or None,
        counts [n_snap]) that this object keeps alive while recording; cap = 0
        turns the records off."""
        import torch

        if not hasattr(self, "_btdp"):
            self._btdp = {}
        out = self._btd.get(run) if hasattr(self, "_btd") else None
        nsnap = out.shape[0] if out is not None else 0
        vals = ids = counts = None
        if cap > 0:
            dtype = torch.float64 if self.precision == GP_FP64 else torch.float32
            vals = torch.empty((nsnap, 6, cap), dtype=dtype, device="cuda")
            ids = torch.empty((nsnap, cap), dtype=torch.int64, device="cuda") if with_ids else None
            counts = torch.empty((max(nsnap, 1),), dtype=torch.int32, device="cuda")
        ptr = lambda t: None if t is None else t.data_ptr()
        self._call("gp_btd_particles", int(run), int(cap), ptr(vals), ptr(ids), ptr(counts))
        self._btdp[run] = (vals, ids, counts)
        return vals, ids, counts

    def btd_record(self):
        """Record the current real E, B as the next level (gp_btd_record)."""
        self._call("gp_btd_record")

    def set_fields(self, run, E=None, B=None, project_transverse=False):
        """E, B: tuples of three real numpy arrays (host) or None."""
        keep = []

        def ptrs(F):
            if F is None:
                return None
            arr = (ctypes.c_void_p * 3)()
            for a in range(3):
                h = np.ascontiguousarray(F[a], dtype=self.real)
                keep.append(h)
                arr[a] = h.ctypes.data
            return arr

        self._call("gp_set_fields", int(run), ptrs(E), ptrs(B), 1 if project_transverse else 0)

    def _shape(self, run, which):
        g = self.grids[run]
        name = FIELDS[which]
        if name in ("EX", "EY", "EZ", "BX", "BY", "BZ", "JX", "JY", "JZ", "RHO"):
            return (g["nx"], g["ny"], g["nz"]), self.real
        return (g["nx"], g["ny"], g["nz"] // 2 + 1), self.cplx

    def read_field(self, run, name):
        which = FIELD[name]
        shape, dt = self._shape(run, which)
        out = np.empty(shape, dtype=dt)
        self._call("gp_read_field", int(run), which, out.ctypes.data)
        return out

    def write_field(self, run, name, values):
        which = FIELD[name]
        shape, dt = self._shape(run, which)
        arr = np.ascontiguousarray(np.broadcast_to(values, shape), dtype=dt)
        self._call("gp_write_field", int(run), which, arr.ctypes.data)

    def field_ptr(self, run, name):
        """Device address of one grid array of a run (gp_field_ptr)."""
        p = ctypes.c_void_p()
        self._call("gp_field_ptr", int(run), FIELD[name], ctypes.byref(p))
        return p.value

    def field_tensor(self, run, name):
        """A torch tensor viewing one grid array in place (no copy): real
        arrays as [nx][ny][nz] of the run's real type, spectral ones as
        [nx][ny][nz/2+1] complex.  It aliases library memory, so it is valid
        while the context lives (rho^ slots: until the next update)."""
        import torch

        which = FIELD[name]
        shape, dt = self._shape(run, which)
        tdt = {np.float64: torch.float64, np.float32: torch.float32,
               np.complex128: torch.complex128, np.complex64: torch.complex64}[dt]
        n = int(np.prod(shape))
        addr = self.field_ptr(run, name)
        elem = np.dtype(dt).itemsize

        class _Iface:
            __cuda_array_interface__ = {"shape": (n,), "typestr": np.dtype(dt).str,
                                        "data": (addr, False), "version": 2,
                                        "strides": None}

        t = torch.as_tensor(_Iface(), device="cuda")
        assert t.element_size() == elem and t.dtype == tdt
        return t.view(shape)

    def field_energy_noalloc(self, run, out_ptr):
        """gp_field_energy_noalloc: W_E, W_B into the device buffer at
        out_ptr (2 doubles), asynchronously, allocating nothing."""
        self._call("gp_field_energy_noalloc", int(run), out_ptr)

    def field_energy(self, run=0):
        we, wb = ctypes.c_double(), ctypes.c_double()
        self._call("gp_field_energy", int(run), ctypes.byref(we), ctypes.byref(wb))
        return we.value, wb.value


def grid_from_config(cfg, precision=None, tile=(0, 0, 0), resort_div=0, flush=0):
    """Grid descriptor dict of a workload.RunConfig (tile, resort_div,
    flush: the tuning knobs of gp_grid_desc, 0 = default; the stencil orders
    of the field solve come from the config)."""
    prec = precision if precision is not None else (
        GP_FP64 if cfg.precision == "fp64" else GP_MIXED)
    return {"nx": cfg.shape[0], "ny": cfg.shape[1], "nz": cfg.shape[2],
            "dx": cfg.spacing[0], "dy": cfg.spacing[1], "dz": cfg.spacing[2],
            "dt": cfg.dt, "order": cfg.order, "precision": prec,
            "tile": tuple(tile), "resort_div": int(resort_div), "flush": int(flush),
            "stencil": tuple(int(p) for p in cfg.stencil)}


def particles_from_inputs(inputs, cfg, precision, with_ids=True, device="cuda"):
    """Device particles of a run from workload.particles_for output."""
    ids = np.arange(inputs["n"], dtype=np.int64) if with_ids else None
    if precision == GP_FP64:
        return Particles(GP_FP64, cfg.q, cfg.m, cfg.w, inputs["u"], x=inputs["x"], ids=ids,
                         device=device)
    return Particles(GP_MIXED, cfg.q, cfg.m, cfg.w, inputs["u"], cell=inputs["cell"],
                     offset=inputs["offset"], ids=ids, device=device)


def qc_wavenumbers(m, nr, dr):
    """Spectral k_r of azimuthal mode m (host only, no GPU)."""
    lib = load()
    out = np.empty(nr, dtype=np.float64)
    _check(lib, lib.gp_qc_wavenumbers(int(m), int(nr), float(dr), out.ctypes.data))
    return out


def qc_hankel_matrix(p, m, nr, dr, forward=False):
    """Backward matrix M[j][i] = J_p(k_i r_j) of mode m's grid, or its
    inverse (host only, no GPU)."""
    lib = load()
    out = np.empty((nr, nr), dtype=np.float64)
    _check(lib, lib.gp_qc_hankel_matrix(int(p), int(m), int(nr), float(dr), int(bool(forward)),
                                        out.ctypes.data))
    return out


class QcContext:
    """One gp_qc_ctx: the quasi-cylindrical field solve of nmodes azimuthal
    modes on an nz x nr (z, r) grid.  Fields are complex numpy arrays
    [mode][z][r]."""

    def __init__(self, nz, nr, nmodes, dz, dr, dt, precision, stream=None, shape_order=1):
        self.lib = load()
        _init_torch_first()
        d = QcDesc(nz, nr, nmodes, dz, dr, dt, precision, shape_order)
        self.shape = (nmodes, nz, nr)
        self.precision = precision
        self.cplx = np.complex128 if precision == GP_FP64 else np.complex64
        handle = ctypes.c_void_p()
        _check(self.lib, self.lib.gp_qc_init(ctypes.byref(d), stream, ctypes.byref(handle)))
        self.h = handle

    def close(self):
        if self.h:
            self.lib.gp_qc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        _check(self.lib, getattr(self.lib, name)(self.h, *args))

    def set_v_gal(self, vz):
        self._call("gp_qc_set_v_gal", float(vz))

    def write(self, name, arr):
        a = np.ascontiguousarray(np.broadcast_to(arr, self.shape), dtype=self.cplx)
        self._call("gp_qc_write", QC_FIELD[name], a.ctypes.data)

    def read(self, name):
        out = np.empty(self.shape, dtype=self.cplx)
        self._call("gp_qc_read", QC_FIELD[name], out.ctypes.data)
        return out

    def fields_fwd(self):
        self._call("gp_qc_fields_fwd")

    def sources_fwd(self):
        self._call("gp_qc_sources_fwd")

    def init_rho(self):
        self._call("gp_qc_init_rho")

    def update(self):
        self._call("gp_qc_update")

    def fields_inv(self):
        self._call("gp_qc_fields_inv")

    def step(self, nsteps=1):
        self._call("gp_qc_step", int(nsteps))

    def synchronize(self):
        self._call("gp_qc_synchronize")

    def set_background(self, rho=None, j_r=None, j_theta=None, j_z=None):
        """Fixed sources added to every deposit (complex [mode][z][r])."""
        keep = []

        def ptr(a):
            if a is None:
                return None
            b = np.ascontiguousarray(np.broadcast_to(a, self.shape), dtype=self.cplx)
            keep.append(b)
            return b.ctypes.data

        self._call("gp_qc_set_background", ptr(rho), ptr(j_r), ptr(j_theta), ptr(j_z))

    def bind_particles(self, q, m, w, x, y, z, ux, uy, uz):
        """x ... uz: device tensors of the context's real type (kept by the
        caller while bound); deposits rho^n."""
        arrs = (x, y, z, ux, uy, uz)
        n = int(x.numel())
        for a in arrs:
            if a.numel() != n or not a.is_contiguous() or not a.is_cuda:
                raise ValueError("particle arrays must be contiguous device tensors of one size")
            if a.element_size() != (8 if self.precision == GP_FP64 else 4):
                raise ValueError("particle arrays must have the context's real type")
        self._parts = arrs
        pc = QcParticlesC(n, float(q), float(m), float(w), *[a.data_ptr() for a in arrs])
        self._call("gp_qc_bind_particles", ctypes.byref(pc))

    def electrostatic_fields(self):
        self._call("gp_qc_electrostatic_fields")

    def particle_step(self, nsteps=1):
        self._call("gp_qc_particle_step", int(nsteps))

    def set_resort(self, div):
        """Re-sort the particles along z when more than n / div of them had
        a deposit node outside their chunk's window (0: never)."""
        self._call("gp_qc_set_resort", int(div))

    def stage_timing(self, enable=True):
        self._call("gp_qc_stage_timing", int(bool(enable)))

    def stage_times(self):
        """{stage: (summed ms, launches)} of the launches timed so far."""
        ms = np.zeros(len(QC_STAGES), dtype=np.float64)
        cnt = np.zeros(len(QC_STAGES), dtype=np.int32)
        self._call("gp_qc_stage_times", ms.ctypes.data, cnt.ctypes.data)
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(QC_STAGES)}
