/*
 * galpic.h -- C ABI of the Galilean-PSATD particle-in-cell step on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Kirchen, Lehe, Godfrey, Dornmair, Jalas, Peters, Vay, Maier,
 * "Stable discrete representation of relativistically drifting plasmas"
 * (arXiv:1608.00215).  The paper transforms the Maxwell and Newton-Lorentz
 * equations to coordinates x' = x - v_gal t, integrates the transformed
 * Maxwell equations analytically in Fourier space with the current held
 * constant over a step in x' (the Galilean-PSATD update and its
 * coefficient block), deposits J at (n+1/2) dt and rho at n dt and
 * (n+1) dt on the grid nodes, transforms back, interpolates to the
 * particles and advances them with dx'/dt = v - v_gal.
 *
 * Passages of the paper cited below (it numbers no equations):
 *  - "the transformed equations": the equations of motion and Maxwell's
 *    equations written in x' = x - v_gal t, with the continuity equation;
 *  - "the update display": the Galilean-PSATD update of E and B with its
 *    coefficients C, S, nu, theta, chi_1..chi_3;
 *  - "the deposition paragraph": the paragraph after the update display
 *    (J deposited at (n+1/2) dt, rho at n dt and (n+1) dt, on the grid
 *    nodes; transform to Fourier space; update; transform back; interpolate
 *    to the particles; advance them with the transformed equations);
 *  - "the simulation parameters": the boosted laser-plasma run's set-up
 *    (cubic shapes, dt = dz / c).
 *
 * One step is the sequence
 *     gp_deposit -> gp_fft_fwd -> gp_galilean_psatd_update -> gp_fft_inv
 *     -> gp_gather_push
 * or gp_step / gp_run / gp_step_graph, which run the same work (over
 * several steps the gather-push of one step is fused with the deposit of
 * the next).  Options beyond the printed scheme: the Galilean current
 * correction (gp_set_current_correction), finite-order stencils for the
 * field solve (gp_grid_desc.stencil), and lab-frame snapshots of fields
 * and particles recorded on the fly (gp_btd_configure, gp_btd_particles).
 *
 * Conventions
 *  - Normalised units: c = eps0 = 1.  Lengths in c/omega_p, times in
 *    1/omega_p.  Momenta are u = p / (m c).
 *  - Grid: periodic, nx x ny x nz nodes at x_i = i * d (no staggering),
 *    real arrays [x][y][z] row-major (z contiguous); spectral arrays are
 *    the half spectrum [x][y][nz/2+1] of interleaved complex values,
 *    forward kernel exp(-i k.x), unnormalised; the inverse carries 1/N.
 *    k is the exact spectral wavevector 2 pi m / L, or a finite-order
 *    stencil's symbol where gp_grid_desc.stencil asks for one.
 *  - The k = 0 mode and every Nyquist plane of J, rho, E and B are held at
 *    zero (the co-moving ion background cancels the mean current).
 *  - Shapes: B-splines of order 1 (cloud-in-cell) or 3 (cubic), the same
 *    shape for deposit and gather.
 *  - Precision GP_FP64: every quantity is double; positions are absolute
 *    doubles wrapped into [0, L).  GP_MIXED: positions are an int32 linear
 *    cell index (ix * ny + iy) * nz + iz plus three float offsets in
 *    [0, 1); momenta, real and spectral fields, FFT, update and push are
 *    float (complex64 spectra); the update coefficients are computed in
 *    double and rounded once; each deposition tile is summed in double
 *    (LDS) before its one float add into the grid.
 *
 * Ownership and threading
 *  - Particle arrays are owned by the caller (device memory, e.g. torch
 *    tensors); the library reads and writes them in place and may reorder
 *    the particles of a run (all arrays of that run, and the optional id
 *    array, are permuted together).  It never frees them.
 *  - Everything else (fields, spectra, coefficient tables, FFT scratch,
 *    sort buffers) is owned by the context from gp_init_grid to
 *    gp_destroy.
 *  - Every call is asynchronous on the stream given at gp_init_grid unless
 *    documented as synchronising.  A context is not thread-safe.  No C++
 *    exception crosses this boundary; failures return a negative status
 *    and gp_last_error() describes the last one (thread-local string).
 */
#ifndef GALPIC_H
#define GALPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_ctx gp_ctx;
typedef int gp_status;

enum {
  GP_OK = 0,
  GP_ERR_ARG = -1,      /* invalid argument                                   */
  GP_ERR_STATE = -2,    /* call out of order (inputs of the call not ready)    */
  GP_ERR_HIP = -3,      /* a HIP runtime call failed                           */
  GP_ERR_UNSTABLE = -4, /* some mode has |k.v_gal| dt >= 2 pi (1 - 1e-6), where
                           the rho-form of the update is singular             */
  GP_ERR_OOM = -5       /* device allocation failed                            */
};

enum { GP_FP64 = 0, GP_MIXED = 1 };

/* Grid selectors for gp_read_field / gp_write_field.  Real arrays hold
 * nx*ny*nz values of the run's real type; spectral ones nx*ny*(nz/2+1)
 * complex values (two reals each). */
enum {
  GP_EX = 0, GP_EY, GP_EZ, GP_BX, GP_BY, GP_BZ,          /* real E, B      */
  GP_JX, GP_JY, GP_JZ, GP_RHO,                            /* real J, rho    */
  GP_EX_HAT, GP_EY_HAT, GP_EZ_HAT,                        /* spectral E^n   */
  GP_BX_HAT, GP_BY_HAT, GP_BZ_HAT,                        /* spectral B^n   */
  GP_JX_HAT, GP_JY_HAT, GP_JZ_HAT,                        /* spectral J     */
  GP_RHO_HAT_OLD,                                         /* rho^n          */
  GP_RHO_HAT_NEW,                                         /* rho^{n+1}      */
  GP_COEF0, GP_COEF1, GP_COEF2, GP_COEF3, GP_COEF4, GP_COEF5, /* c_EE, s, c_BJ,
                                   c_EJ, c_R1, c_R0 (read only, see below) */
  GP_N_FIELDS
};

/* One run's grid.  nx, ny, nz: powers of two in [8, 1024]; dx, dy, dz > 0;
 * dt > 0; shape_order 1 or 3; precision GP_FP64 or GP_MIXED (all runs of a
 * context use the same precision and shape order).
 * stencil[3]: spatial derivative of the field solve per axis.  0 (the
 * paper's solver): the exact spectral wavenumber k.  An even order p in
 * [2, 64]: the centered difference of order p on the colocated grid, whose
 * symbol [k] = (2/d) sum_{l=1}^{p/2} a_l sin(l k d) replaces k in every
 * part of the field update (curls, charge terms, the Galilean phase
 * theta, the current correction and the transverse projection); a
 * finite-order solve has a local real-space stencil, the prerequisite of
 * domain decomposition with local transforms and guard cells, which the
 * paper names as future work.  Deposition and gather do not change.
 * Tuning knobs (0 = default; results do not depend on them beyond float
 * summation order):
 *   tile[3]     cells per deposition tile and axis: powers of two, at most 8
 *               and at most the grid (default 8, or the grid if smaller);
 *   resort_div  re-sort the particles by tile when more than n / resort_div
 *               of them used the global path since the last decision
 *               (default 64; at least 1);
 *   flush       how a deposition tile adds its node region (the tile, the
 *               shape's support and the drift margin, summed in LDS) into
 *               J and rho: 1 (and 0, the default) float atomics into the
 *               grids; 2 plain stores into a region buffer (tiles x 4 x
 *               region values, allocated at binding), summed node by node
 *               by a second kernel (stage "region_reduce"). */
typedef struct {
  int nx, ny, nz;
  double dx, dy, dz, dt;
  int shape_order;
  int precision;
  int tile[3];
  int resort_div;
  int stencil[3];
  int flush;
} gp_grid_desc;

/* One run's macro-particles (one species, uniform weights).
 *  n       number of particles (>= 0)
 *  q, m, w charge, mass and weight (physical particles per macro-particle);
 *          each deposits q w / (dx dy dz) times its shape
 *  GP_FP64: x, y, z are double* absolute positions in [0, n_a d_a);
 *           off_x, off_y, off_z unused (NULL).
 *  GP_MIXED: x is int32* linear cell index, y and z unused (NULL);
 *           off_x, off_y, off_z are float* offsets in [0, 1).
 *  ux, uy, uz: momenta u = p / (m c) (double* or float*), at the half
 *          step before the next deposit.
 *  id      optional int64* carried along when particles are reordered. */
typedef struct {
  int64_t n;
  double q, m, w;
  void *x, *y, *z;
  void *off_x, *off_y, *off_z;
  void *ux, *uy, *uz;
  int64_t *id;
} gp_particles;

/* Create a context for n_runs independent runs advanced together.
 * Paper: the deposition paragraph (fields and sources on the nodes of a
 * periodic grid, advanced in Fourier space by the pseudo-spectral solver
 * of the update display).
 * hip_stream: a hipStream_t, or NULL for a stream created and owned by
 * the context (default priority; graph capture needs a non-null stream).
 * Allocates all
 * device state; fields start at zero.  v_gal starts at zero (standard
 * PSATD) with coefficients built.  Errors: GP_ERR_ARG for an invalid
 * descriptor, GP_ERR_OOM, GP_ERR_HIP.  Synchronising. */
gp_status gp_init_grid(const gp_grid_desc *runs, int n_runs, void *hip_stream,
                       gp_ctx **out);

/* Set v_gal of one run and rebuild its coefficient table in double
 * precision on the device.  Paper: the update display (C, S, nu, theta,
 * chi_1..chi_3, evaluated here through cancellation-free integral forms).
 * Errors: GP_ERR_ARG if run is out of range or |v_gal| >= c,
 * GP_ERR_UNSTABLE if some non-Nyquist mode has |k.v_gal| dt >=
 * 2 pi (1 - 1e-6). */
gp_status gp_set_v_gal(gp_ctx *ctx, int run, double vx, double vy, double vz);

/* Option, off by default (not with the slab solve of gp_set_local_slabs,
 * GP_ERR_STATE): before each update replace the longitudinal part
 * of J^ of every run so that the Galilean continuity equation of the
 * transformed equations, integrated over the step with J constant
 * (rho^{n+1} = theta^2 rho^n + F k.J, F = (1 - theta^2) / (k.v_gal), -> -i dt
 * as k.v_gal -> 0), holds exactly for the deposited rho^n, rho^{n+1}; the
 * transverse part of J is kept.  Gauss's law then evolves exactly as the
 * update prescribes for any deposition.  Not part of the printed update.
 * enable: 0 or 1.  Takes effect at the next update.  Errors: GP_ERR_ARG. */
gp_status gp_set_current_correction(gp_ctx *ctx, int enable);

/* Register the particle arrays p[0..n_runs-1] with the context, sort them
 * into deposition tiles (reordering them in place), deposit rho at the
 * current positions and transform it into rho^n.  Paper: the deposition
 * paragraph (rho at n dt, the first of the two charge densities).  Must precede
 * gp_deposit / gp_gather_push / gp_step; call again after changing the
 * arrays from outside.  Errors: GP_ERR_ARG (NULL pointers, n < 0,
 * positions outside the layout contract are not checked). */
gp_status gp_bind_particles(gp_ctx *ctx, const gp_particles *p);

/* Deposit J^{n+1/2} and rho^{n+1}: move every particle by (v - v_gal) dt/2,
 * deposit q w v S (lab velocity v = u / gamma) into J, move it by another
 * (v - v_gal) dt/2, deposit q w S into rho.  Paper: the deposition
 * paragraph (currents at (n+1/2) dt, charge at (n+1) dt, on the grid
 * nodes) and the transformed equations (dx'/dt = v - v_gal).  Positions are
 * written back.  p must be the bound arrays (else GP_ERR_STATE). */
gp_status gp_deposit(gp_ctx *ctx, const gp_particles *p);

/* Forward FFT of J (3 components) and rho^{n+1}; k = 0 and Nyquist planes
 * set to zero.  Paper: the deposition paragraph (the deposited sources are
 * transformed to Fourier space before the update).  Requires a deposit (or
 * written J/rho) since the last forward transform. */
gp_status gp_fft_fwd(gp_ctx *ctx);

/* Galilean-PSATD update of spectral E and B from E^n, B^n, J^{n+1/2},
 * rho^n, rho^{n+1}; then rho^{n+1} becomes rho^n.  Paper: the update
 * display.  Requires gp_fft_fwd (or written spectral J and rho^{n+1}). */
gp_status gp_galilean_psatd_update(gp_ctx *ctx);

/* Inverse FFT of spectral E and B into the real E and B used by the
 * gather.  Paper: the deposition paragraph (the updated fields are
 * transformed back to real space and interpolated to the particles).  The
 * spectral state is left unchanged. */
gp_status gp_fft_inv(gp_ctx *ctx);

/* Interpolate E and B to every particle (same shape as the deposit) and
 * advance u by dt with the relativistic Boris scheme.  Paper: the
 * deposition paragraph (interpolation to the particles) and the
 * transformed equations (dp/dt = q (E + v x B), unchanged by the
 * transformation).  Positions are unchanged.
 * Requires real E and B produced by gp_fft_inv or gp_write_field. */
gp_status gp_gather_push(gp_ctx *ctx, const gp_particles *p);

/* gp_gather_push followed by gp_deposit in one particle pass: interpolate
 * E and B at x^n, push u^{n-1/2} -> u^{n+1/2}, then move by (v - v_gal) dt/2,
 * deposit J^{n+1/2}, move again and deposit rho^{n+1}.  This is the pass
 * gp_run makes between two field cycles; callers that drive the stage calls
 * themselves use it in place of the two calls.  Paper: the deposition
 * paragraph (interpolation, push, then the next step's deposition) and the
 * transformed equations.  Requires real E and B as for gp_gather_push. */
gp_status gp_gather_push_deposit(gp_ctx *ctx, const gp_particles *p);

/* One full step for every run (deposit, fft_fwd, update, fft_inv,
 * gather_push), equivalent to the five calls above.  Paper: the deposition
 * paragraph (the order of the cycle). */
gp_status gp_step(gp_ctx *ctx, const gp_particles *p);

/* nsteps full steps, equivalent to nsteps gp_step calls; the gather-push
 * of each step is fused with the deposit of the next into one particle
 * pass.  Paper: the deposition paragraph (the order of the cycle, which
 * the fusion keeps: push with the fields at x^n, then move and deposit). */
gp_status gp_run(gp_ctx *ctx, const gp_particles *p, int nsteps);

/* As gp_run, replayed from HIP graphs captured on first use (recaptured
 * after gp_bind_particles or gp_set_v_gal).  Paper: the deposition
 * paragraph (the same cycle as gp_run).  The context stream must not be
 * the null stream. */
gp_status gp_step_graph(gp_ctx *ctx, const gp_particles *p, int nsteps);

/* Option, off by default: the field solve of every run on z-slabs with
 * local transforms and guard cells.  The paper's closing paragraph names
 * domain decomposition with local transforms over subdomains padded by
 * guard cells, which finite-order solvers make possible, as future work; it
 * does not print the procedure.  Reading taken here (one device; the guard
 * exchange between neighbouring slabs is a copy out of the run's grids):
 *  - the grid is cut into n_slabs slabs of ns = nz / n_slabs planes; slab s
 *    owns planes s ns .. s ns + ns - 1 and transforms the window of planes
 *    s ns - guard .. s ns + ns + guard - 1 (periodic) as its own periodic
 *    grid of nw = ns + 2 guard planes;
 *  - the state is the real E, B; each field cycle takes the windows of E, B
 *    and of J, rho^{n+1} (less their grid means: the co-moving ions that
 *    hold the global solve's k = 0 mode at zero), holds the windows' Nyquist
 *    planes of the sources at zero and nothing else, advances every local
 *    mode with the Galilean-PSATD update on the window's grid (the run's
 *    stencil orders; at [k] = 0 the update is E' = E - dt J, B' = B), with
 *    rho^n the slab's previous rho^{n+1} window, and writes the windows'
 *    owned planes of the new E, B back into the run's E, B (the guard
 *    planes are dropped and read again from the neighbours next cycle);
 *  - gp_fft_fwd, gp_galilean_psatd_update and gp_fft_inv then run these
 *    three parts (windows and forward transforms; the slabs' update; inverse
 *    transforms and owned planes), and the step drivers use them; the run's
 *    own spectral E^, B^, rho^ are not kept up to date (gp_read_field of
 *    them returns old values).
 * A window as long as the grid (nw = nz) reproduces the global solve; a
 * shorter one differs from it by the part of the one-step propagator that
 * reaches past the guard planes.
 *   n_slabs  0: back to the global solve (its spectral state is rebuilt from
 *            the real E, B and rho); else nz must be a multiple of it;
 *   guard    planes on each side: nz / n_slabs + 2 guard must be a power of
 *            two in [8, nz].
 * Every run needs a finite-order stencil along z (gp_grid_desc.stencil[2]
 * in [2, 64]); the current correction must be off (GP_ERR_STATE).  Requires real E, B current; with particles bound, rho^n of
 * the slabs is taken from the runs' current rho (the last deposit).
 * Allocates the slabs' grids (like a context of n_runs * n_slabs runs of
 * nx x ny x nw).  Errors: GP_ERR_ARG, GP_ERR_STATE, GP_ERR_OOM. */
gp_status gp_set_local_slabs(gp_ctx *ctx, int n_slabs, int guard);

/* Lab-frame snapshots of a boosted run (back-transformed diagnostics): the
 * paper reports its boosted-frame results in the lab frame through an
 * on-the-fly back-transformation, named as the boosted run's only
 * overhead (closing results paragraph; the procedure itself is not
 * printed).  The run's v_gal must be (0, 0, -beta c): the boosted frame
 * moves at +beta c along z relative to the lab, where the plasma, at rest
 * on the Galilean grid, is at rest.  Galilean plane k (z'_k = k dz) is
 * then the fixed lab plane z_lab = gamma z'_k, and its event at boosted
 * time t' has lab time t'/gamma + gamma beta z'_k / c.
 *   n_snap   number of snapshots (at most 65535), at lab times
 *            t_lab0 + j dt_lab; 0 turns the recording of this run off (out
 *            may then be NULL);
 *   t_boost0 boosted time of the current real E, B (level 0); every field
 *            cycle of gp_step / gp_run / gp_step_graph, and every
 *            gp_btd_record, adds the next level, dt later;
 *   out      device buffer of 6 * n_snap * nx*ny*nz values of the run's
 *            real type, layout [snapshot][Ex Ey Ez Bx By Bz][z][x][y] (lab
 *            planes contiguous, since they complete one at a time), owned
 *            by the caller and kept valid while recording; cleared here.
 * Plane k of snapshot j receives the Lorentz-transformed fields (lab
 * frame moving at -beta c: E_x = gamma (E'_x + beta c B'_y), E_y =
 * gamma (E'_y - beta c B'_x), B_x = gamma (B'_x - beta E'_y / c), B_y =
 * gamma (B'_y + beta E'_x / c), E_z, B_z unchanged) at boosted time
 * t'_jk = gamma t_j - gamma^2 beta z'_k / c, linearly interpolated
 * between the levels t'_n < t'_jk <= t'_{n+1}.  It is complete once the
 * levels reach t'_jk; before that it holds part of the sum or zero.
 * Records the current real E, B as level 0, so call it after setting the
 * initial fields.  Changing v_gal needs the recording off.  Errors:
 * GP_ERR_ARG (bad run, n_snap outside [0, 65535], NULL out, non-finite
 * times, v_gal not along z), GP_ERR_STATE (real fields not current). */
gp_status gp_btd_configure(gp_ctx *ctx, int run, int n_snap, double t_lab0, double dt_lab,
                           double t_boost0, void *out);

/* Lab-frame particle records of a recording run (the particle side of the
 * back-transformation).  After each particle move (the deposit or fused
 * pass of gp_step / gp_run / gp_step_graph, and gp_deposit) a particle's
 * worldline over the step is the straight segment of its move ending at
 * its position in the box, at boosted time t_boost0 + m dt (m: the run's
 * recorded field levels); along it the lab time t'/gamma + gamma beta z'/c
 * increases strictly.  Each snapshot whose lab time the segment passes
 * (t_lab(start) < t_j <= t_lab(end)) records the particle there: x, y
 * (wrapped to the box), z_lab = gamma z' (z' wrapped to the box), and the
 * lab momentum u_x, u_y, gamma (u_z + beta gamma_p).
 *   cap     records per snapshot; 0 turns particle records off;
 *   vals    device buffer [snapshot][x y z_lab u_x u_y u_z][cap] of the
 *           run's real type;
 *   ids     device int64 [snapshot][cap] for the particles' ids, or NULL
 *           (needs bound particles that carry ids);
 *   counts  device int [snapshot], cleared here: records made; records
 *           past cap are dropped but counted, so counts[j] > cap flags an
 *           overflow.  The order of records within a snapshot is not
 *           fixed.
 * All buffers are the caller's and stay valid while recording.  Requires
 * gp_btd_configure with n_snap > 0 and dt_lab > 0 and bound particles; a
 * new gp_btd_configure turns the records off; re-binding keeps them on
 * (with the new arrays).  Errors: GP_ERR_ARG, GP_ERR_STATE. */
gp_status gp_btd_particles(gp_ctx *ctx, int run, int cap, void *vals, int64_t *ids,
                           int *counts);

/* Record the current real E, B of every recording run as its next level
 * (for callers that drive the stage calls themselves; the step drivers
 * record by themselves).  Errors: GP_ERR_STATE (real fields not current). */
gp_status gp_btd_record(gp_ctx *ctx);

/* Set E^0 and B^0 of one run from real-space arrays (device or host
 * pointers to nx*ny*nz values of the run's real type, or NULL for zero):
 * transformed, held modes set to zero, and with project_transverse != 0
 * the component along k removed.  Also sets the real E and B. */
gp_status gp_set_fields(gp_ctx *ctx, int run, const void *const E[3],
                        const void *const B[3], int project_transverse);

/* Boris half push u^0 -> u^{1/2} through dt/2 with the current real E and
 * B at the current positions (start-up of the leapfrog).  Paper: the
 * transformed equations (the momentum equation over half a step; the
 * start-up itself is not printed). */
gp_status gp_half_push(gp_ctx *ctx, const gp_particles *p);

/* Copy one grid array of one run to dst / from src (host or device
 * pointers; synchronising).  Writing marks the array as a valid input of
 * the next call that consumes it.  Coefficient tables are read-only. */
gp_status gp_read_field(gp_ctx *ctx, int run, int which, void *dst);
gp_status gp_write_field(gp_ctx *ctx, int run, int which, const void *src);

/* Device address of one grid array of one run (the array gp_read_field
 * would copy), for callers that read or write the fields in place (e.g.
 * through torch tensors on the context's stream).  Real arrays hold
 * nx*ny*nz values of the run's real type, spectral ones nx*ny*(nz/2+1)
 * interleaved complex values.  The address of a real array, of E^, B^, J^
 * and of a coefficient table is fixed from gp_init_grid to gp_destroy; the
 * two rho^ buffers swap roles at every update, so the address returned for
 * GP_RHO_HAT_OLD / GP_RHO_HAT_NEW holds that role only until the next
 * update.  Coefficient tables must not be written.  Writing through the
 * address does not mark the array as a fresh input (gp_write_field does);
 * the caller orders its accesses with the context's stream.  Paper: the
 * deposition paragraph (the grids it names: J, rho, E, B and their
 * transforms).  Errors: GP_ERR_ARG (bad run or selector, NULL out). */
gp_status gp_field_ptr(gp_ctx *ctx, int run, int which, void **dev_ptr);

/* Field energy W_E = 1/2 sum |E|^2 dV and W_B = 1/2 sum |B|^2 dV of the
 * real fields, reduced in double on the device (synchronising). */
gp_status gp_field_energy(gp_ctx *ctx, int run, double *we, double *wb);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * quantity of gp_field_energy, out[0] = W_E, out[1] = W_B of one run's real
 * E, B, reduced in double, written to out (device memory, 2 doubles, the
 * caller's) asynchronously on the context's stream (no synchronisation, so
 * it can be captured in a graph).  It allocates nothing: the per-workgroup
 * partial sums go to a file-scope device array of the library (8192 slots
 * of two doubles, 128 KiB per device, held until the process ends); every
 * slot it reads is written by the same call, so nothing needs clearing, and
 * the result does not depend on scheduling.  All calls on one device share
 * that array: calls that may overlap on one device (other streams, other
 * threads) race and must be ordered by the caller.  Errors: GP_ERR_ARG (bad
 * run, NULL out, a run of more than 2^26 = 67,108,864 cells). */
gp_status gp_field_energy_noalloc(gp_ctx *ctx, int run, double *out);

/* Device time of the last gp_step_graph replay in milliseconds (HIP
 * events on the context stream; synchronising). */
gp_status gp_last_graph_ms(gp_ctx *ctx, double *ms);

/* Per-kernel device timing.  While enabled, gp_step, gp_run and the
 * single-call entry points record HIP events on the context stream around
 * each kernel stage (one launch per run each; names from gp_stage_name).
 * gp_stage_times returns, per stage, the summed milliseconds and the number
 * of recorded launches, then clears them (synchronising).  Graph replays
 * are not recorded. */
#define GP_N_STAGES 16
gp_status gp_stage_timing(gp_ctx *ctx, int enable);
gp_status gp_stage_times(gp_ctx *ctx, double ms[GP_N_STAGES], int count[GP_N_STAGES]);
const char *gp_stage_name(int stage);

/* Number of tile sorts performed on run's particles since binding
 * (synchronising). */
gp_status gp_sort_count(gp_ctx *ctx, int run, int *sorts);

/* Wait until all work enqueued on the context's stream has finished. */
gp_status gp_synchronize(gp_ctx *ctx);

/* Release everything the context owns.  NULL is accepted. */
gp_status gp_destroy(gp_ctx *ctx);

/* Message of the last failure on this thread ("" if none). */
const char *gp_last_error(void);

/* ---- Quasi-cylindrical field solve (option) ------------------------------
 * The paper's own runs use a quasi-3D spectral code: fields expanded in
 * azimuthal modes m, discrete Hankel transforms along r in place of the
 * transverse Fourier transforms; the Galilean scheme does not depend on the
 * geometry.  This context advances the fields of nmodes modes with the
 * Galilean-PSATD update for given sources, and (below) particles deposited
 * and gathered by mode.  Readings (the paper does not print the scheme):
 *  - a mode m field is F_m(r, z) exp(i m theta); G_+ = (F_r + i F_theta)/2
 *    carries Hankel order m+1, G_- = (F_r - i F_theta)/2 order m-1, F_z
 *    and rho order m;
 *  - radial nodes r_j = (j + 1/2) dr, j < nr; spectral grid per mode
 *    k_i = alpha_{m,i} / (nr dr) (zeros of J_m) for all three orders;
 *    backward transform F(r_j) = sum_i F^_i J_p(k_i r_j), forward its
 *    matrix inverse; z periodic with the Cartesian Fourier convention, the
 *    k_z Nyquist plane held at zero;
 *  - for m >= 1 the order m-1 functions on the zeros of J_m are a Dini
 *    series that needs r^{m-1} (k_r = 0) to be complete: the last G_-
 *    function is (r / R)^{m-1} at k_r = 0, and the last k_r column of G_+,
 *    G_z and the scalars is held at zero (without this a G_- with nonzero
 *    mean, e.g. a uniform transverse mode-1 field, has a wrong divergence);
 *  - the update is the Cartesian Galilean-PSATD update at k = (k_r, 0, k_z)
 *    applied to F^_x = i (G^_- - G^_+), F^_y = -(G^_+ + G^_-), F^_z = G^_z;
 *    v_gal is along z.
 * Fields are complex [mode][z][r] arrays (r contiguous) of the context's
 * real type (interleaved re, im).  Calls are asynchronous on the context's
 * stream unless noted; errors as for the Cartesian calls. */
typedef struct gp_qc_ctx gp_qc_ctx;
typedef struct {
  int nz;        /* z nodes: power of two in [8, 1024] (periodic)          */
  int nr;        /* radial nodes r_j = (j + 1/2) dr: [4, 512]              */
  int nmodes;    /* azimuthal modes m = 0 .. nmodes-1: [1, 8]              */
  double dz, dr, dt;
  int precision; /* GP_FP64 or GP_MIXED (float fields, FP64-built tables)  */
  int shape_order; /* particle shape in r and z: 0 or 1 linear, 3 cubic    */
} gp_qc_desc;

/* Selectors of gp_qc_read / gp_qc_write: real-space components, spectral
 * G^_+, G^_-, G^_z of E, B, J, rho^n and rho^{n+1}, and (read only) the six
 * update coefficients [mode][k_z][k_r] (as for GP_COEF0..5). */
enum {
  GP_QC_ER = 0, GP_QC_ET, GP_QC_EZ, GP_QC_BR, GP_QC_BT, GP_QC_BZ,
  GP_QC_JR, GP_QC_JT, GP_QC_JZ, GP_QC_RHO,
  GP_QC_E_PLUS, GP_QC_E_MINUS, GP_QC_E_Z_HAT,
  GP_QC_B_PLUS, GP_QC_B_MINUS, GP_QC_B_Z_HAT,
  GP_QC_J_PLUS, GP_QC_J_MINUS, GP_QC_J_Z_HAT,
  GP_QC_RHO_HAT_OLD, GP_QC_RHO_HAT_NEW,
  GP_QC_COEF0, GP_QC_COEF1, GP_QC_COEF2, GP_QC_COEF3, GP_QC_COEF4, GP_QC_COEF5,
  GP_QC_N_FIELDS
};

/* Create a context (fields zero, v_gal 0, transform matrices and k_r built
 * in double on the host).  hip_stream as for gp_init_grid.  Synchronising.
 * Errors: GP_ERR_ARG (sizes), GP_ERR_OOM, GP_ERR_HIP. */
gp_status gp_qc_init(const gp_qc_desc *d, void *hip_stream, gp_qc_ctx **out);
/* v_gal = (0, 0, vz); rebuilds the coefficients in double.  Errors:
 * GP_ERR_ARG (|vz| >= c), GP_ERR_UNSTABLE (|k_z vz| dt >= 2 pi (1 - 1e-6)). */
gp_status gp_qc_set_v_gal(gp_qc_ctx *ctx, double vz);
/* Copy nmodes*nz*nr complex values from or to src / dst (host or device
 * memory).  Synchronising. */
gp_status gp_qc_write(gp_qc_ctx *ctx, int which, const void *src);
gp_status gp_qc_read(gp_qc_ctx *ctx, int which, void *dst);
/* Real E, B -> spectral E^, B^ (initial fields). */
gp_status gp_qc_fields_fwd(gp_qc_ctx *ctx);
/* Real J, rho -> spectral J^ and rho^{n+1}. */
gp_status gp_qc_sources_fwd(gp_qc_ctx *ctx);
/* Real rho -> rho^n (the initial charge). */
gp_status gp_qc_init_rho(gp_qc_ctx *ctx);
/* The Galilean-PSATD update of every mode; then rho^{n+1} becomes rho^n. */
gp_status gp_qc_update(gp_qc_ctx *ctx);
/* Spectral E^, B^ -> real E, B. */
gp_status gp_qc_fields_inv(gp_qc_ctx *ctx);
/* nsteps of (gp_qc_sources_fwd, gp_qc_update, gp_qc_fields_inv) with the
 * real J and rho as they stand. */
gp_status gp_qc_step(gp_qc_ctx *ctx, int nsteps);
gp_status gp_qc_synchronize(gp_qc_ctx *ctx);
/* Particles of a quasi-cylindrical context: caller-owned device arrays of
 * the context's real type (double for GP_FP64, float for GP_MIXED):
 * Cartesian positions x, y (open) and z in [0, nz dz) (periodic), and
 * u = p / (m c).  q, m, w as for gp_particles. */
typedef struct {
  int64_t n;
  double q, m, w;
  void *x, *y, *z;
  void *ux, *uy, *uz;
} gp_qc_particles;

/* Deposition and gather by azimuthal mode (the paper's runs use a
 * quasi-cylindrical code; it does not print the scheme).  B-spline weights
 * of order shape_order (linear or cubic) in r (nodes (j + 1/2) dr) and z; a
 * stored mode-m field is c_m f_m (c_0 = 1, c_m = 2), so the physical field
 * is Re sum_m F_m exp(i m theta); a radial node j < 0 is node -j-1 seen
 * across the axis and takes its weight with (-1)^m (scalars, z components)
 * or (-1)^(m+1) (r, theta components); node j's volume is its folded
 * weight's integral against 2 pi r dr dz; weights past the last node are
 * dropped.
 *
 * gp_qc_set_background: a fixed source added to every deposit (e.g. a
 * neutralising ion column), complex [mode][z][r] host or device arrays of rho,
 * J_r, J_theta, J_z (a NULL one is zero; all NULL clears it).  Synchronising.
 * gp_qc_bind_particles: keeps the pointers (the caller keeps the arrays
 * alive), reorders the particles along z in place (a stable sort of all six
 * arrays together, so that the deposit's chunks of consecutive particles
 * cover few z planes), deposits rho^n (with the background) and makes it
 * the spectral rho^n.  Synchronising.  Errors: GP_ERR_ARG.
 * gp_qc_electrostatic_fields: E^ = the curl-free field with i k.E^ = rho^n
 * (k_z Nyquist row zero), then the real E, B from E^, B^.
 * gp_qc_particle_step: nsteps of the Galilean-PSATD particle cycle (with u
 * at n - 1/2: move half a step with v - v_gal, deposit J with v = u / gamma,
 * move the other half, deposit rho^{n+1}, transform, update every mode,
 * transform back, gather E, B at x^{n+1}, relativistic Boris push).
 * Errors: GP_ERR_STATE (no particles bound). */
gp_status gp_qc_set_background(gp_qc_ctx *ctx, const void *rho, const void *j_r,
                               const void *j_theta, const void *j_z);
gp_status gp_qc_bind_particles(gp_qc_ctx *ctx, const gp_qc_particles *p);
gp_status gp_qc_electrostatic_fields(gp_qc_ctx *ctx);
gp_status gp_qc_particle_step(gp_qc_ctx *ctx, int nsteps);

/* Re-sort of the bound particles along z during gp_qc_particle_step.  The
 * deposit takes chunks of consecutive particles, each with an LDS window of
 * a few z planes; as the particles move the binding order decays and more
 * of their nodes fall outside the window (global atomics instead).  The
 * deposit counts the particles that had such a node; before every 16th
 * deposit, when more than n / div of them were counted since the last
 * decision, the particles are sorted along z again on the device (a
 * counting sort by z cell of all six arrays together, in the caller's
 * arrays; their order within a cell is not kept, and with no particle ids
 * the caller can no longer match particles across steps, hence opt-in).
 * The decision is taken on the device; its time is part of the deposit
 * stage.  div = 0 (the default): never.  Errors: GP_ERR_ARG (div < 0).
 * No passage of the paper defines it: it changes the order in which the
 * deposit visits the particles (the deposited sums up to rounding), not
 * the method. */
gp_status gp_qc_set_resort(gp_qc_ctx *ctx, int div);

/* With timing on, every launch records HIP events on the context stream,
 * by stage: 0 z transforms forward, 1 Hankel transforms forward, 2 mode
 * update, 3 Hankel transforms backward, 4 z transforms inverse, 5 particle
 * moves and deposits, 6 gather and push.  gp_qc_stage_times returns the
 * summed milliseconds and launch counts per stage, then clears them
 * (synchronising). */
#define GP_QC_N_STAGES 7
gp_status gp_qc_stage_timing(gp_qc_ctx *ctx, int enable);
gp_status gp_qc_stage_times(gp_qc_ctx *ctx, double ms[GP_QC_N_STAGES],
                            int count[GP_QC_N_STAGES]);
gp_status gp_qc_destroy(gp_qc_ctx *ctx);
/* Host-only (no GPU, no context): the spectral grid and transform matrices
 * a context builds, for callers that prepare or read spectral fields.
 * gp_qc_wavenumbers writes k_i = alpha_{m,i} / (nr dr), i < nr, the first nr
 * positive zeros of J_m over R (for m >= 1 the update takes k_r = 0 in the
 * last column, see above).  gp_qc_hankel_matrix writes, row-major nr x nr,
 * the backward matrix of Hankel order p on mode m's grid, M[j][i] =
 * J_p(k_i r_j) with r_j = (j + 1/2) dr (radial j <- spectral i), its last
 * column (r_j / R)^{m-1} for p = m - 1, m >= 1; or, with forward != 0, its
 * inverse A[i][j] (spectral i <- radial j).  A
 * context applies these (the backward one divided by nz, in the run's real
 * type) along r.  Errors: GP_ERR_ARG (NULL output, m outside [0, 63], p
 * outside [-64, 64], nr outside [1, 512], dr not positive and finite, a
 * singular matrix). */
gp_status gp_qc_wavenumbers(int m, int nr, double dr, double *kr);
gp_status gp_qc_hankel_matrix(int p, int m, int nr, double dr, int forward, double *out);

#ifdef __cplusplus
}
#endif

#endif /* GALPIC_H */
