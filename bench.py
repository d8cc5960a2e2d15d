"""Benchmark of the Galilean-PSATD PIC step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Runs W untimed steps, then K timed steps (default 200, or the workload's
run if shorter) of the whole hot path (deposit, forward FFT, k-space update,
inverse FFT, gather + Boris push) on the workload's seeded synthetic plasma,
inputs resident in HBM, and prints one JSON line: particle-steps/s (the
whole job), the per-kernel device times measured with HIP events on the
library's stream, the roofline of the dominant kernel, the FP64 GPU path on
the same workload, and the CPU oracle timed on a bounded sample of the
workload on this host.  The default workload is the 256x256x512 boosted
run with its laser (cubic shapes, dt = dz / c, v_gal = -beta c), the
largest single-GPU configuration; the mixed-precision and FP64 GPU paths
run it side by side.  After the timed steps (and their graph replay) the
run continues to step 200 and times 20 more steps there, so that a short
timed window early in the run is reported beside a later one.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32, published (256 CUs, 2.4 GHz)
FP64_PEAK_TFLOPS = 78.6
PARTICLE_STAGES = ("deposit", "fused_push_deposit", "gather_push")
METRIC = "particle-steps/s per Galilean-PSATD PIC step (mixed vs FP64); % HBM peak"


def stage_bytes(cfg, precision_fp64):
    """Algorithmic HBM bytes of one launch of each stage (each array read or
    written once): particles read/write their state once, grids once."""
    rb = 8 if precision_fp64 else 4
    cb = 2 * rb
    pos = 24 if precision_fp64 else 16          # 3 doubles | int32 cell + 3 floats
    nc, nk, npart = cfg.n_cells, cfg.n_modes, cfg.n_particles
    return {
        "zero_sources": 4 * nc * rb,
        "sort": 0,                              # a flag check unless a re-sort is due
        "deposit": npart * (pos + 3 * rb + pos) + 4 * nc * rb,
        # read x, u; write u, x; read E, B (6 grids); write J, rho (4 grids)
        "fused_push_deposit": npart * (pos + 3 * rb + 3 * rb + pos) + 10 * nc * rb,
        "fft_fwd_z": 4 * (nc * rb + nk * cb),
        "fft_fwd_y": 4 * 2 * nk * cb,
        "fft_fwd_x": 4 * 2 * nk * cb,
        "update": nk * cb * (11 + 6 + 6),
        "fft_inv_x": 6 * 2 * nk * cb,
        "fft_inv_y": 6 * 2 * nk * cb,
        "fft_inv_z": 6 * (nk * cb + nc * rb),
        "gather_push": npart * (pos + 3 * rb + 3 * rb) + 6 * nc * rb,
        "btd": 0,                               # a few planes per snapshot and step
        # the slab solve: windows and owned planes (two stamps of unequal
        # size per step) and the windows' E, B transforms; reported as times
        "slab_copy": 0,
        "slab_fft_fwd_eb": 0,
        # region buffer (flush 2): every tile's region of J, rho read once
        # (8^3 tiles, region (8 + shape width - 1 + 2)^3), J and rho read
        # and written
        "region_reduce": (nc // 512) * 4 * (8 + (3 if cfg.order == 3 else 1) + 2) ** 3 * rb
        + 8 * nc * rb,
    }


def stage_flops(cfg):
    """Algorithmic floating-point operations per particle of the particle
    stages (shape weights, node weight products, gather and deposit
    multiply-adds, Boris push, moves)."""
    n = 4 if cfg.order == 3 else 2
    n2, n3 = n * n, n * n * n
    weights = 3 * (10 if n == 4 else 2)      # one position: three axes
    products = n2 + n3                       # w_x w_y, then times w_z
    position = weights + products
    gather = 12 * n3                         # 6 fields, multiply-add
    deposit = 6 * n3 + 2 * n3                # J (3 values) and rho, multiply-add
    push = 70                                # relativistic Boris
    move = 15 + 20                           # v = u / gamma, two half moves
    return {
        "deposit": cfg.n_particles * (2 * position + deposit + move),
        "fused_push_deposit": cfg.n_particles * (3 * position + gather + push + deposit + move),
        "gather_push": cfg.n_particles * (position + gather + push),
    }


def btd_snapshot_times(c, nsnap, t_mid):
    """Lab times of nsnap snapshots whose planes k_j = (j + 1/2) nz / nsnap
    are reached at boosted time t_mid (v_gal = -beta c along z)."""
    beta = -c.v_gal()[2]
    g = 1.0 / np.sqrt(1.0 - beta * beta)
    gap = c.shape[2] / nsnap * c.spacing[2]          # dz between the planes k_j
    t_lab0 = (t_mid + g * g * beta * 0.5 * gap) / g
    return t_lab0, g * beta * gap


def run_gpu(cfg, precision, steps, warmup, inputs, tile=(0, 0, 0), resort_div=0, btd=0,
            btd_cap=0, correction=False, late_at=0, late_n=20, slabs=None, flush=0):
    """Time one run (cfg, inputs) or a batch of runs (lists of both)."""
    import torch

    from paper_1608_00215_amd import galpic as gp
    from workload import laser_fields

    cfgs = cfg if isinstance(cfg, list) else [cfg]
    inps = inputs if isinstance(inputs, list) else [inputs]
    grids = [gp.grid_from_config(c, precision,
                                 tile=tuple(min(tile[a], c.shape[a]) for a in range(3)),
                                 resort_div=resort_div, flush=flush) for c in cfgs]
    ctx = gp.Context(grids)
    for r, c in enumerate(cfgs):
        ctx.set_v_gal(r, c.v_gal())
    if correction:
        ctx.set_current_correction(True)
    parts = [gp.particles_from_inputs(i, c, precision, with_ids=False)
             for c, i in zip(cfgs, inps)]
    ctx.bind_particles(parts)
    for r, c in enumerate(cfgs):
        lf = laser_fields(c)
        if lf is not None:
            ctx.set_fields(r, lf[0], lf[1], project_transverse=True)
    if any(c.laser is not None for c in cfgs):
        ctx.half_push()
    if slabs is not None:
        ctx.set_local_slabs(*slabs)
    if btd > 0:
        # lab-frame snapshots of the first run, recorded on the fly; their
        # planes are reached in the middle of the timed steps
        t_lab0, dt_lab = btd_snapshot_times(cfgs[0], btd, (warmup + 0.5 * steps) * cfgs[0].dt)
        ctx.btd_configure(0, btd, t_lab0, dt_lab, 0.0)
        if btd_cap > 0:
            ctx.btd_particles(0, btd_cap, with_ids=False)
    if warmup > 0:
        ctx.run(warmup)
    ctx.synchronize()
    ctx.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run(steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage = ctx.stage_times()
    ctx.stage_timing(False)
    sorts = sum(ctx.sort_count(r) for r in range(len(cfgs)))
    # the same steps replayed from a captured HIP graph
    ctx.step_graph(1)
    ctx.synchronize()
    ctx.step_graph(steps)
    graph_ms = ctx.last_graph_ms()
    we, wb = ctx.field_energy(0)
    done = warmup + 2 * steps + 1
    late = None
    if late_at > 0:
        # a later window of the same run: advance to step late_at (untimed),
        # then time late_n eager steps
        if done < late_at:
            ctx.run(late_at - done)
            done = late_at
        ctx.synchronize()
        ctx.stage_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run(late_n)
        ctx.synchronize()
        torch.cuda.synchronize()
        late_wall = time.perf_counter() - t0
        lst = ctx.stage_times()
        ctx.stage_timing(False)
        late = {"first_step": done + 1, "steps": late_n,
                "ms_per_step": late_wall / late_n * 1e3,
                "stage_ms": {k: ms / n for k, (ms, n) in lst.items() if n > 0}}
    ctx.close()
    del parts
    torch.cuda.empty_cache()
    return {"wall_s": wall,
            "stage_ms": {k: ms / n for k, (ms, n) in stage.items() if n > 0},
            "stage_launches": {k: n for k, (ms, n) in stage.items() if n > 0},
            "graph_ms_per_step": graph_ms / steps, "field_energy": we + wb, "sorts": sorts,
            "late": late}


def traffic_from_profiles(workload, kernel_stage, fp64):
    """HBM bytes per launch measured with rocprofv3 counters, if a summary for
    this kernel on this workload exists and its source has not changed
    since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        key = f"{workload}:{'fp64' if fp64 else 'mixed'}:{kernel_stage}"
        rec = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("workload") != workload:
        return None
    for rel, want in rec["sources"].items():
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != want:
            return None
    return rec["bytes_per_launch"]


class BatchView:
    """Totals of a batch of runs, shaped like a RunConfig for the report."""

    def __init__(self, runs):
        self.runs = runs
        self.name = "c5_batched"
        self.shape = ("batch of %d runs" % len(runs),)
        self.n_particles = sum(r.n_particles for r in runs)
        self.n_cells = sum(r.n_cells for r in runs)
        self.n_modes = sum(r.n_modes for r in runs)
        self.ppc = runs[0].ppc
        self.order = runs[0].order
        self.gamma = float(np.mean([r.gamma for r in runs]))
        self.u_th = runs[0].u_th
        self.laser = None


def host_cpu():
    """(model name, logical CPUs) of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(cfg):
    """The oracle, as it stands, on a sub-box of the workload: the same
    particles per cell, shape, drift and thermal spread (and laser pulse,
    started the same way), on about two million particles; the coefficient
    set-up, the laser start and the first step are not timed."""
    from threadpoolctl import threadpool_limits

    from oracle import pic
    from workload import laser_fields, particles_for

    nz = max(64, (1 << 21) // (64 * 64 * cfg.ppc))
    sub = cfg.with_(shape=(64, 64, min(nz, cfg.shape[2])))
    inp = particles_for(sub)
    g = pic.Grid(sub.shape, sub.spacing, sub.dt, sub.order)
    sim = pic.Simulation(g, pic.Species(sub.q, sub.m, sub.w), sub.v_gal())
    lf = laser_fields(sub)
    if lf is not None:
        st = sim.initial_state(inp["x"], inp["u"], lf[0], lf[1], project_transverse=True)
        st = sim.half_push(st)
    else:
        st = sim.initial_state(inp["x"], inp["u"])
    steps = 3
    model, ncpu = host_cpu()
    with threadpool_limits(limits=1):     # any BLAS/OpenMP pool: one thread
        st = sim.step(st)
        t0 = time.perf_counter()
        for _ in range(steps):
            st = sim.step(st)
        t = time.perf_counter() - t0
    return {"value": sub.n_particles * steps / t, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle", "host_cpu": model, "host_logical_cpus": ncpu,
            "sample": (f"{steps} oracle steps (numpy FP64, one thread) on a {sub.shape[0]}x"
                       f"{sub.shape[1]}x{sub.shape[2]} sub-box of the workload "
                       f"({sub.n_particles} particles, same ppc/shape/drift"
                       f"{'/laser' if lf is not None else ''}), {t:.1f} s, after one "
                       f"untimed step; host: {model}, {ncpu} logical CPUs")}


def accuracy_run(cfg, steps, inputs, every=10):
    """The mixed-precision path against the FP64 GPU path on the same
    workload: per-field relative L2 of E and B after `steps` steps, and the
    field-energy histories (sampled every `every` steps) of both."""
    import torch

    from paper_1608_00215_amd import galpic as gp
    from workload import laser_fields

    ctxs, parts = {}, {}
    for name, prec in (("mixed", gp.GP_MIXED), ("fp64", gp.GP_FP64)):
        ctx = gp.Context([gp.grid_from_config(cfg, prec)])
        ctx.set_v_gal(0, cfg.v_gal())
        parts[name] = gp.particles_from_inputs(inputs, cfg, prec, with_ids=False)
        ctx.bind_particles([parts[name]])
        lf = laser_fields(cfg)
        if lf is not None:
            ctx.set_fields(0, lf[0], lf[1], project_transverse=True)
            ctx.half_push()
        ctxs[name] = ctx
    hist = {"step": [], "mixed": [], "fp64": []}
    done = 0
    while done < steps:
        k = min(every, steps - done)
        for name, ctx in ctxs.items():
            ctx.run(k)
        done += k
        hist["step"].append(done)
        for name, ctx in ctxs.items():
            we, wb = ctx.field_energy(0)
            hist[name].append(we + wb)
        print(f"[accuracy] step {done}: W mixed {hist['mixed'][-1]:.6g} "
              f"fp64 {hist['fp64'][-1]:.6g}", file=sys.stderr, flush=True)
    errs = {}
    for f in ("EX", "EY", "EZ", "BX", "BY", "BZ"):
        a = ctxs["mixed"].read_field(0, f).astype(np.float64)
        b = ctxs["fp64"].read_field(0, f)
        nb = float(np.sqrt(np.sum(b * b)))
        errs[f] = float(np.sqrt(np.sum((a - b) ** 2)) / nb) if nb > 0 else None
        del a, b
    wm, wf = np.array(hist["mixed"]), np.array(hist["fp64"])
    drift = np.abs(wm - wf) / np.abs(wf)
    for ctx in ctxs.values():
        ctx.close()
    torch.cuda.empty_cache()
    return {"workload": cfg.name, "steps": steps,
            "field_rel_l2_mixed_vs_fp64": errs,
            "energy_rel_diff_final": float(drift[-1]),
            "energy_rel_diff_max": float(drift.max()),
            "energy_fp64_first_last": [float(wf[0]), float(wf[-1])],
            "history_every": every,
            "energy_mixed": [float(x) for x in wm], "energy_fp64": [float(x) for x in wf]}


def workload_text(cfg):
    prec = ("mixed precision (int32 cell + f32 offsets, f32 FFT/update/push, f64 "
            "coefficients, double tile sums)")
    if isinstance(cfg, BatchView):
        return (f"{cfg.name}: {len(cfg.runs)} independent drifting-plasma runs, grids from "
                "{32,64}^2 x {64,128,256}, gamma ~ U[5,50], density ~ U[0.5,2], "
                f"{cfg.ppc} electrons/cell, u_th {cfg.u_th:g}, v_gal = drift, order-{cfg.order} "
                f"shape, {prec}; one context, per-run kernels in one captured graph")
    laser = ""
    if cfg.laser is not None:
        lp = cfg.laser
        laser = (f", Gaussian laser a0 {lp['a0']:g} waist {lp['waist']:g} wavelength "
                 f"{lp['wavelength']:g} length {lp['length']:g} cells moving +z")
    return (f"{cfg.name}: {cfg.shape[0]}x{cfg.shape[1]}x{cfg.shape[2]} periodic grid, "
            f"{cfg.ppc} electrons/cell, gamma {cfg.gamma:g} drift, u_th {cfg.u_th:g}, "
            f"v_gal = drift{laser}, order-{cfg.order} shape, {prec}")


QC_WORKLOADS = {
    # the cylindrical counterpart of the 256x256x512 boosted-laser grid:
    # 512 z nodes, 128 radial nodes (the box half-width), modes 0 (wake) and
    # 1 (linearly polarised laser), gamma_boost 20, dz = dr = 1, dt = dz / c
    "qc_boosted": dict(nz=512, nr=128, nmodes=2, dz=1.0, dr=1.0, dt=1.0, gamma=20.0,
                       steps=1000),
    # the largest grid a context takes, two modes
    "qc_wide": dict(nz=1024, nr=512, nmodes=2, dz=1.0, dr=1.0, dt=1.0, gamma=20.0,
                    steps=200),
    # the particle cycle: an electron column of radius 96 (density 1, 24
    # particles per (r, z) cell, drifting at gamma 20 along -z) on its
    # neutralising ion column, modes 0 and 1, Galilean frame, electrostatic
    # start
    "qc_column": dict(nz=512, nr=128, nmodes=2, dz=1.0, dr=1.0, dt=1.0, gamma=20.0,
                      steps=200, ppc=24, rp=96.0),
    # the same with cubic shapes in r and z (as the paper's runs use)
    "qc_column_cubic": dict(nz=512, nr=128, nmodes=2, dz=1.0, dr=1.0, dt=1.0, gamma=20.0,
                            steps=200, ppc=24, rp=96.0, order=3),
}


def qc_flops(w, stage):
    """Algorithmic flops of one launch of a Hankel-transform stage: a real
    nr x nr matrix times complex rows, 4 flops per (input, output) pair per
    row, over nz rows, nmodes modes and the launch's components (forward: the
    vector launch's 3 plus the scalar launch's 1, summed per step; backward:
    E and B, 6)."""
    comps = {"hankel_fwd": 4, "hankel_bwd": 6}[stage]
    return 4.0 * w["nz"] * w["nr"] ** 2 * w["nmodes"] * comps


def qc_bytes(w, stage, real_size, n_part=0):
    """Algorithmic HBM bytes of one step's launches of a stage (complex
    fields of nmodes * nz * nr values read and written once; the update reads
    E, B, J (9), rho twice and 6 coefficients and writes E, B (6)).  The
    particle stages read positions and momenta (6 values) and write
    positions (deposit) or momenta (gather-push) (3 values); their grid
    accesses (atomics and gathers) resolve in L2 and are not counted."""
    if stage in ("deposit", "gather_push"):
        return n_part * 9 * real_size
    field = w["nmodes"] * w["nz"] * w["nr"] * 2 * real_size
    per = {"z_fwd": 4 * 2, "hankel_fwd": 5 + 4, "update": 9 + 2 + 6 + 6,
           "hankel_bwd": 6 + 6, "z_inv": 6 * 2}[stage]
    return per * field


def run_qc(name, precision, steps, warmup):
    import torch

    from paper_1608_00215_amd import galpic as gp

    w = QC_WORKLOADS[name]
    beta = np.sqrt(1.0 - 1.0 / w["gamma"] ** 2)
    stream = torch.cuda.current_stream()
    ctx = gp.QcContext(w["nz"], w["nr"], w["nmodes"], w["dz"], w["dr"], w["dt"], precision,
                       stream=ctypes_stream(stream), shape_order=w.get("order", 1))
    ctx.set_v_gal(-beta)
    rng = np.random.Generator(np.random.PCG64(7000))
    shp = (w["nmodes"], w["nz"], w["nr"])
    n_part = 0
    if "ppc" in w:
        x, u, qw_w = qc_column_inputs(w)
        n_part = len(x)
        dt_t = torch.float64 if precision == gp.GP_FP64 else torch.float32
        parts = [torch.tensor(np.ascontiguousarray(a), dtype=dt_t, device="cuda")
                 for a in (x[:, 0], x[:, 1], x[:, 2], u[:, 0], u[:, 1], u[:, 2])]
        rho_bg = np.zeros(shp, dtype=complex)
        rho_bg[0] = qc_ion_profile(w)[None, :]
        zero = np.zeros(shp, dtype=complex)
        ctx.set_background(rho_bg, zero, zero, -beta * rho_bg)
        # re-sort along z when more than n/256 particles had a deposit node
        # outside their chunk's window (the binding order decays over a run)
        ctx.set_resort(256)
        ctx.bind_particles(-1.0, 1.0, qw_w, *parts)
        ctx.electrostatic_fields()
        advance = ctx.particle_step
    else:
        for f in ("ER", "ET", "EZ", "BR", "BT", "BZ", "JR", "JT", "JZ", "RHO"):
            ctx.write(f, rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
        ctx.fields_fwd()
        ctx.init_rho()
        advance = ctx.step
    advance(warmup)
    ctx.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-launch kernel times from events, in a separate pass
    ctx.stage_timing(True)
    advance(min(steps, 50))
    times = ctx.stage_times()
    ctx.stage_timing(False)
    ctx.close()
    return {"wall_s": wall, "stages": times, "particles": n_part}


def qc_column_inputs(w):
    """Seeded electron column: w["ppc"] particles per (r, z) cell inside rp, r drawn
    with density proportional to r, angle and z uniform; cold drift at
    gamma along -z.  Returns x, u (n, 3) and the weight of density 1."""
    rng = np.random.Generator(np.random.PCG64(7002))
    n = int(w["ppc"] * w["nz"] * w["rp"] / w["dr"])
    r = w["rp"] * np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    x = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(0.0, w["nz"] * w["dz"], n)], 1)
    u = np.zeros((n, 3))
    u[:, 2] = -np.sqrt(w["gamma"] ** 2 - 1.0)
    weight = np.pi * w["rp"] ** 2 * w["nz"] * w["dz"] / n
    return x, u, weight


def qc_ion_profile(w):
    """Per radial node, the share of the node's shape volume (its B-spline
    of the workload's order plus the mirror image across the axis, times r)
    inside rp: the charge density of a uniform ion column of density 1 as
    the deposit sees it.  In u = r / dr the integrand is a polynomial of
    degree <= 4 between the half-integers, so 4-point Gauss-Legendre on
    each unit piece (and the piece cut at rp) is exact."""
    dr, nr, rp = w["dr"], w["nr"], w["rp"]
    order = w.get("order", 1)

    def spline(t):
        a = np.abs(t)
        if order == 1:
            return np.maximum(0.0, 1.0 - a)
        return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                        np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))

    gx, gw = np.polynomial.legendre.leggauss(4)
    half = (order + 1) // 2
    ucut = rp / dr
    prof = np.zeros(nr)
    for j in range(nr):
        c = j + 0.5
        bounds = sorted({max(0.0, c - half), c + half, *[b + 0.5 for b in range(j + half)],
                         *([ucut] if 0.0 < ucut < c + half else [])})
        bounds = [b for b in bounds if max(0.0, c - half) <= b <= c + half]
        inside = total = 0.0
        for a, b in zip(bounds[:-1], bounds[1:]):
            u = 0.5 * (a + b) + 0.5 * (b - a) * gx
            part = 0.5 * (b - a) * np.sum(gw * (spline(u - c) + spline(u + c)) * u)
            total += part
            if 0.5 * (a + b) < ucut:
                inside += part
        prof[j] = inside / total
    return prof


def ctypes_stream(stream):
    import ctypes

    return ctypes.c_void_p(stream.cuda_stream)


def qc_cpu_baseline(name, budget_s=10.0):
    """The oracle's mode transforms and update, as they stand, on the
    workload's grid, for as many whole steps (all modes) as fit the budget."""
    from threadpoolctl import threadpool_limits

    from oracle import cylindrical as cy

    w = QC_WORKLOADS[name]
    beta = np.sqrt(1.0 - 1.0 / w["gamma"] ** 2)
    rng = np.random.Generator(np.random.PCG64(7001))
    shp = (w["nz"], w["nr"])
    c = lambda: rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    nz, nr, dz, dr, dt = w["nz"], w["nr"], w["dz"], w["dr"], w["dt"]
    state = {m: (cy.to_spectral((c(), c(), c()), m, dr, dz),
                 cy.to_spectral((c(), c(), c()), m, dr, dz)) for m in range(w["nmodes"])}
    J = (c(), c(), c())
    rho = c()
    steps = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s or steps == 0:
            for m in range(w["nmodes"]):
                E, B = state[m]
                Jh = cy.to_spectral(J, m, dr, dz)
                rh = cy.scalar_to_spectral(rho, m, dr, dz)
                E, B = cy.mode_update(E, B, Jh, rh, rh, m, nr, dr, nz, dz, -beta, dt)
                cy.from_spectral(E, m, dr, dz)
                cy.from_spectral(B, m, dr, dz)
                state[m] = (E, B)
            steps += 1
        t = time.perf_counter() - t0
    cells = w["nmodes"] * nz * nr
    return {"value": cells * steps / t, "unit": "mode-cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{steps} whole oracle steps (sources forward, update, fields back, "
                       f"every mode; numpy, single thread) on the full {nz}x{nr} grid, "
                       f"{w['nmodes']} modes, {t:.1f} s; transform matrices rebuilt "
                       f"per call as the oracle does")}


def qc_particle_cpu_baseline(name, budget_s=15.0):
    """The oracle's whole particle cycle (CylindricalPIC: moves, deposits,
    transforms, mode update, gather and push), as it stands, on a sub-box
    of the workload: 64 of its z cells with the same radius, particles per
    cell, drift, modes and shape; single thread, as many steps as fit the
    budget."""
    from threadpoolctl import threadpool_limits

    from oracle import cylindrical as cy

    w = dict(QC_WORKLOADS[name])
    w["nz"] = 64
    beta = np.sqrt(1.0 - 1.0 / w["gamma"] ** 2)
    order = w.get("order", 1)
    x, u, qw_w = qc_column_inputs(w)
    bg = cy.uniform_cylinder_background(1.0, w["rp"], -beta, w["nmodes"], w["nr"], w["dr"],
                                        w["nz"], w["dz"], order)
    sim = cy.CylindricalPIC(w["nz"], w["nr"], w["nmodes"], w["dz"], w["dr"], w["dt"], -1.0, 1.0,
                            qw_w, -beta, background=bg, order=order)
    steps = 0
    with threadpool_limits(limits=1):
        st = sim.initial_state(x, u, electrostatic=True)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s or steps == 0:
            st = sim.step(st)
            steps += 1
        t = time.perf_counter() - t0
    return {"value": len(x) * steps / t, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"{steps} whole oracle steps (numpy, single thread) on a {w['nz']}x"
                       f"{w['nr']} sub-box of the workload ({len(x)} particles, same radius, "
                       f"particles per cell, drift, modes and shape), {t:.1f} s; set-up and "
                       "electrostatic start not timed")}


def qc_main(args):
    from paper_1608_00215_amd import galpic as gp

    w = QC_WORKLOADS[args.qc]
    steps = w["steps"] if args.steps is None else args.steps
    print(f"[bench] {args.qc}: nz {w['nz']} nr {w['nr']} modes {w['nmodes']}, {steps} steps",
          file=sys.stderr, flush=True)
    mixed = run_qc(args.qc, gp.GP_MIXED, steps, args.warmup)
    print(f"[bench] mixed: {mixed['wall_s'] / steps * 1e3:.4f} ms/step", file=sys.stderr,
          flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_qc(args.qc, gp.GP_FP64, steps, args.warmup)
        print(f"[bench] fp64: {fp64['wall_s'] / steps * 1e3:.4f} ms/step", file=sys.stderr,
              flush=True)
    cells = w["nmodes"] * w["nz"] * w["nr"]

    def stages_of(st, res, real_size):
        stages = {}
        for k, v in st.items():
            ms_s = v[0] / st["update"][1]
            d = {"ms_per_step": round(ms_s, 5), "launches_per_step": v[1] // st["update"][1],
                 "gbs": round(qc_bytes(w, k, real_size, res["particles"]) / (ms_s * 1e-3) / 1e9,
                              1)}
            if k in ("deposit", "gather_push"):
                d["ns_per_particle"] = round(ms_s * 1e6 / res["particles"], 3)
            if k.startswith("hankel"):
                d["tflops"] = round(qc_flops(w, k) / (ms_s * 1e-3) / 1e12, 2)
            stages[k] = d
        return stages

    def summary(res, real_size, peak):
        st = {k: v for k, v in res["stages"].items() if v[1] > 0}
        per = {k: v[0] / v[1] for k, v in st.items()}
        if res["particles"]:
            # with particles the move-and-deposit kernel dominates; its
            # algorithmic HBM bytes are the particle arrays (read 6, write 3
            # values) and the four source grids written once; its atomics
            # resolve in L2 and bound it
            ms_launch = per["deposit"]
            byt = qc_bytes(w, "deposit", real_size, res["particles"]) + \
                4 * w["nmodes"] * w["nz"] * w["nr"] * 2 * real_size
            achieved = byt / (ms_launch * 1e-3) / 1e9
            roof = {"kernel": "k_qc_move_deposit", "bound": "hbm", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "ms_per_launch": ms_launch, "traffic": None,
                    "note": "bound by global atomics to the source grids (resolved in L2)"}
        else:
            # the largest single launch of the field step: the backward
            # Hankel transform of E and B (one k_qc_hankel<T, kVecBwd> launch;
            # the forward stage is two different launches); it runs on the
            # matrix cores, so its roof is the dense MFMA peak of its type
            ms_launch = per["hankel_bwd"]
            achieved = qc_flops(w, "hankel_bwd") / (ms_launch * 1e-3) / 1e12
            roof = {"kernel": "k_qc_hankel (backward, E and B)", "bound": "mfma",
                    "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "ms_per_launch": ms_launch, "traffic": None}
        return roof, stages_of(st, res, real_size)

    # dense MFMA peaks of MI355X: fp32 157.3, fp64 78.6 TFLOP/s
    roof, stages = summary(mixed, 4, FP32_PEAK_TFLOPS)
    line = {
        "metric": "mode-cell updates/s of the quasi-cylindrical Galilean-PSATD field solve",
        "value": cells * steps / mixed["wall_s"],
        "unit": "mode-cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["wall_s"] / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.qc}: quasi-cylindrical field solve, nz {w['nz']}, "
                               f"nr {w['nr']}, modes 0..{w['nmodes'] - 1}, gamma_boost "
                               f"{w['gamma']}, v_gal = -beta c, seeded random mode fields "
                               "and sources (kernel cost does not depend on the values)",
                   "precision": "mixed"},
        "stages": stages,
        "roofline": roof,
    }
    if mixed["particles"]:
        line["particles"] = mixed["particles"]
        line["particle_steps_per_s"] = mixed["particles"] * steps / mixed["wall_s"]
        line["config"]["workload"] = (f"{args.qc}: quasi-cylindrical particle cycle, nz "
                                      f"{w['nz']}, nr {w['nr']}, modes 0..{w['nmodes'] - 1}, "
                                      "an electron column of "
                                      f"radius {w['rp']:g} ({w['ppc']} particles per (r, z) "
                                      f"cell, {mixed['particles']} particles) drifting at "
                                      f"gamma {w['gamma']:g} on its ion column, Galilean frame, "
                                      f"{'cubic' if w.get('order', 1) == 3 else 'linear'} "
                                      "shapes")
    if fp64 is not None:
        roof64, stages64 = summary(fp64, 8, FP64_PEAK_TFLOPS)
        line["fp64_gpu"] = {"value": cells * steps / fp64["wall_s"],
                            "ms_per_step": fp64["wall_s"] / steps * 1e3,
                            "stages": stages64, "roofline": roof64}
    if not args.no_cpu:
        line["cpu_baseline"] = (qc_particle_cpu_baseline(args.qc) if mixed["particles"]
                                else qc_cpu_baseline(args.qc))
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200, or the workload's run if shorter)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3_boosted_laser")
    ap.add_argument("--late-at", type=int, default=200, metavar="STEP",
                    help="after the timed steps, continue the run to this step and time 20 "
                         "more steps there (0: skip)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--accuracy", action="store_true",
                    help="instead of timing, run the mixed and FP64 GPU paths side by side "
                         "and report per-field errors and energy histories")
    ap.add_argument("--autotune", action="store_true",
                    help="first time candidate tile shapes and re-sort thresholds on the "
                         "workload (outside the timed steps) and use the fastest")
    ap.add_argument("--btd", type=int, default=0, metavar="N",
                    help="record N lab-frame snapshots of the (first) run on the fly in the "
                         "mixed run and report the back-transformation's share of the step")
    ap.add_argument("--btd-particles", type=int, default=0, metavar="CAP",
                    help="with --btd: also record the particles crossing the snapshots' lab "
                         "times (up to CAP per snapshot)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a plain copy "
                         "kernel of known size for scaling HBM byte counters)")
    ap.add_argument("--stencil", type=int, default=0, metavar="P",
                    help="field solve with the finite-order stencil of even order P on every "
                         "axis (0: spectral, the default)")
    ap.add_argument("--current-correction", action="store_true",
                    help="field solve with the Galilean current correction")
    ap.add_argument("--slabs", type=int, default=0, metavar="S",
                    help="field solve on S z-slabs with local transforms and guard cells "
                         "(needs --stencil; see --guard)")
    ap.add_argument("--guard", type=int, default=0, metavar="G",
                    help="with --slabs: guard planes on each side of a slab")
    ap.add_argument("--flush", type=int, default=0, choices=(0, 1, 2),
                    help="how deposition tiles add their regions: 1 (and 0, the default) "
                         "atomics, 2 region buffer and per-node sum")
    ap.add_argument("--qc", default=None, choices=sorted(QC_WORKLOADS),
                    help="instead, time the quasi-cylindrical (azimuthal-mode) field solve "
                         "on the named grid and print its own line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the "
              "multi-GPU decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.qc:
        qc_main(args)
        return

    from paper_1608_00215_amd import galpic as gp
    from workload import get_config, particles_for

    if args.copy_calibration > 0:
        import torch

        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {args.copy_calibration} MiB x 3", file=sys.stderr,
              flush=True)
        del src, dst

    if args.workload == "c5_batched":
        from workload import batched_runs

        runs = batched_runs()
        cfg = BatchView(runs)
        inputs = [particles_for(c) for c in runs]
        run_arg = runs
    else:
        cfg = get_config(args.workload)
        if args.stencil:
            cfg = cfg.with_(stencil=(args.stencil,) * 3)
        inputs = particles_for(cfg)
        run_arg = cfg
    if args.steps is None:
        args.steps = min(200, cfg.runs[0].steps if isinstance(cfg, BatchView) else cfg.steps)
    print(f"[bench] {cfg.name}: grid {cfg.shape}, {cfg.n_particles} particles, "
          f"{args.steps} steps", file=sys.stderr, flush=True)
    if args.accuracy:
        if isinstance(cfg, BatchView):
            sys.exit("bench.py: --accuracy takes a single-run workload")
        print(json.dumps(accuracy_run(cfg, args.steps, inputs)), flush=True)
        return
    tuning = None
    setting = {"tile": (0, 0, 0), "resort_div": 0}
    if args.autotune:
        from paper_1608_00215_amd import autotune

        t0 = time.perf_counter()
        tcfgs = run_arg if isinstance(run_arg, list) else [run_arg]
        tinps = inputs if isinstance(inputs, list) else [inputs]
        best, res = autotune.tune(tcfgs, tinps, gp.GP_MIXED,
                                  log=lambda m: print(f"[autotune] {m}", file=sys.stderr,
                                                      flush=True))
        setting = {"tile": best[0], "resort_div": best[1]}
        tuning = {"tile": list(best[0]), "resort_div": best[1],
                  "tuning_s": round(time.perf_counter() - t0, 1),
                  "candidates_ms_per_step": {f"{k[0][0]}x{k[0][1]}x{k[0][2]}/n{k[1]}": round(v, 4)
                                             for k, v in res.items()}}
    slabs = (args.slabs, args.guard) if args.slabs > 0 else None
    mixed = run_gpu(run_arg, gp.GP_MIXED, args.steps, args.warmup, inputs, btd=args.btd,
                    btd_cap=args.btd_particles, correction=args.current_correction,
                    late_at=args.late_at, slabs=slabs, flush=args.flush, **setting)
    print(f"[bench] mixed: {mixed['wall_s'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr,
          flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu(run_arg, gp.GP_FP64, args.steps, args.warmup, inputs,
                       correction=args.current_correction, late_at=args.late_at, slabs=slabs,
                       flush=args.flush)
        print(f"[bench] fp64: {fp64['wall_s'] / args.steps * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    del inputs

    ms_step = mixed["wall_s"] / args.steps * 1e3
    value = cfg.n_particles * args.steps / mixed["wall_s"]
    alg = stage_bytes(cfg, False)
    # dominant = the kernel with the largest share of the step
    share = {k: v * mixed["stage_launches"][k] for k, v in mixed["stage_ms"].items()}
    dominant = max(share, key=share.get)
    dom_ms = mixed["stage_ms"][dominant]
    if dominant in PARTICLE_STAGES:
        # the particle kernels are bound by vector ALU work (and LDS), not HBM
        achieved = stage_flops(cfg)[dominant] / (dom_ms * 1e-3) / 1e12
        roof = {"kernel": dominant, "bound": "alu", "achieved": achieved,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                "hbm_gbs": alg[dominant] / (dom_ms * 1e-3) / 1e9,
                "hbm_frac": alg[dominant] / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    else:
        achieved = alg[dominant] / (dom_ms * 1e-3) / 1e9
        roof = {"kernel": dominant, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}
    roof["traffic"] = traffic_from_profiles(cfg.name, dominant, False)
    stages = {k: {"ms_per_launch": round(v, 5), "launches": mixed["stage_launches"][k],
                  "gbs": round(alg[k] / (v * 1e-3) / 1e9, 1) if (v > 0 and alg[k]) else None}
              for k, v in mixed["stage_ms"].items()}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload_text(cfg),
            "grid": list(cfg.shape),
            "particles": cfg.n_particles,
            "cells": cfg.n_cells,
            "precision": "mixed",
            "stencil": list(cfg.stencil) if not isinstance(cfg, BatchView) else None,
            "current_correction": args.current_correction,
            "slabs": None if slabs is None else {"n_slabs": slabs[0], "guard": slabs[1]},
        },
        "grid_updates_per_s": cfg.n_cells * args.steps / mixed["wall_s"],
        "graph_ms_per_step": mixed["graph_ms_per_step"],
        "tile_sorts": mixed["sorts"],
        "late_window": None if mixed["late"] is None else {
            "first_step": mixed["late"]["first_step"], "steps": mixed["late"]["steps"],
            "ms_per_step": mixed["late"]["ms_per_step"],
            "particle_steps_per_s": cfg.n_particles / (mixed["late"]["ms_per_step"] * 1e-3),
            "dominant_ms_per_launch": mixed["late"]["stage_ms"].get(dominant)},
        "stages": stages,
        "roofline": roof,
        "tuning": tuning,
    }
    if args.btd > 0:
        c0 = cfg.runs[0] if isinstance(cfg, BatchView) else cfg
        beta = -c0.v_gal()[2]
        g = 1.0 / np.sqrt(1.0 - beta * beta)
        btd_ms = mixed["stage_ms"].get("btd", 0.0) * mixed["stage_launches"].get("btd", 0)
        line["btd"] = {"snapshots": args.btd, "particle_cap": args.btd_particles,
                       "ms_per_launch": mixed["stage_ms"].get("btd"),
                       "share_of_step": btd_ms / (mixed["wall_s"] * 1e3),
                       "planes_per_snapshot_per_step": c0.dt / (g * g * beta * c0.spacing[2])}
    if fp64 is not None:
        line["fp64_gpu"] = {
            "value": cfg.n_particles * args.steps / fp64["wall_s"],
            "unit": "particle-steps/s",
            "ms_per_step": fp64["wall_s"] / args.steps * 1e3,
            "graph_ms_per_step": fp64["graph_ms_per_step"],
            "stages_ms": {k: round(v, 5) for k, v in fp64["stage_ms"].items()},
            "field_energy_rel_diff_vs_mixed": abs(fp64["field_energy"] - mixed["field_energy"])
            / max(abs(fp64["field_energy"]), 1e-300),
            "late_window_ms_per_step": None if fp64["late"] is None
            else fp64["late"]["ms_per_step"],
        }
    if rank == 0 and not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg.runs[0] if isinstance(cfg, BatchView) else cfg)
    if rank == 0:
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
