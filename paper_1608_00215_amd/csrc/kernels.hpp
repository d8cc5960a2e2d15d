// Host-side launchers of the gfx950 kernels (one translation unit each).
#pragma once

#include <string>

#include "common.hpp"

namespace galpic {

// The message gp_last_error returns (set by entry points outside api.hip).
void set_last_error(const std::string &msg);

// Up to six field arrays of one run.  Launches take a device table of
// FieldSets, one per run: workgroup row blockIdx.y = run * nf + field, so one
// launch covers every run of a grid shape.
struct FieldSet {
  const void *in[6];
  void *out[6];
};

// ---- FFT (fft.hip) ---------------------------------------------------------
// Twiddle table: 1024 values exp(-2 pi i m / 1024) in the run's precision.
template <typename T>
void fill_twiddles(Cx<T> *host1024);

// Forward real-to-complex transform along z of nf real arrays [x][y][z] into
// half spectra [x][y][nz/2+1], for the nsets runs (all of grid shape g) of
// the device table sets.
template <typename T>
void launch_r2c_z(const FieldSet *sets, int nsets, int nf, const RunGeom &g, const Cx<T> *tw,
                  hipStream_t s);
// Complex transform along y (axis 1) or x (axis 0) of nf half spectra.
// mask: kMaskNone; kMaskHeld writes zero on the k = 0 mode and every Nyquist
// plane; kMaskNyquist on the Nyquist planes only.
enum { kMaskNone = 0, kMaskHeld = 1, kMaskNyquist = 2 };
template <typename T>
void launch_c2c(const FieldSet *sets, int nsets, int nf, const RunGeom &g, int axis,
                bool inverse, int mask, const Cx<T> *tw, hipStream_t s);
// Inverse complex-to-real transform along z with the 1/(nx ny nz) scale.
template <typename T>
void launch_c2r_z(const FieldSet *sets, int nsets, int nf, const RunGeom &g, const Cx<T> *tw,
                  hipStream_t s);

// Complex transforms along the lines of arrays of n_outer blocks: line
// element j of column c of block o at o * outer_stride + j * row_stride + c
// (ncols columns, 2^log_len elements per line), no held-mode mask, no
// scaling.
template <typename T>
void launch_c2c_lines(const FieldSet *sets, int nsets, int nf, int log_len, int ncols,
                      int64_t row_stride, int64_t outer_stride, int n_outer, bool inverse,
                      const Cx<T> *tw, hipStream_t s);

// ---- coefficients (coef.hip) ----------------------------------------------
struct CoefPtrs {
  void *c[6];  // c_EE, s, c_BJ, c_EJ, c_R1, c_R0 as Cx<T>
};
// kt: the run's wavenumbers per axis (nx values of x, ny of y, nz/2+1 of
// z, in transform index order), exact or a stencil's symbol.
template <typename T>
void launch_coefficients(const RunGeom &g, const double *kt, const CoefPtrs &cp, hipStream_t s);

// ---- k-space update and reductions (update.hip) ----------------------------
template <typename T>
struct UpdatePtrs {
  Cx<T> *E[3];
  Cx<T> *B[3];
  const Cx<T> *J[3];
  const Cx<T> *rho_old;
  const Cx<T> *rho_new;
  const Cx<T> *coef[6];
  const T *k[3];   // wavenumbers of x (nx), y (ny), z (nz/2+1), index order
  double vgal[3];  // the run's v_gal and dt, for the current correction
  double dt;
  int correct;     // nonzero: correct J before the update (see update.hip)
  int no_hold;     // nonzero: advance every mode (the slab solve's local
                   // grids); zero: k = 0 and the Nyquist planes are written
                   // as zero
};
// The update of the nsets runs (all of grid shape g) of the device table.
template <typename T>
void launch_update(const RunGeom &g, const UpdatePtrs<T> *sets, int nsets, hipStream_t s);
// Transverse projection F <- F - k (k.F)/k^2 of a spectral 3-vector, held
// modes zeroed.
template <typename T>
void launch_project(const RunGeom &g, const T *kt, Cx<T> *F0, Cx<T> *F1, Cx<T> *F2,
                    bool transverse, hipStream_t s);
// Fill nbytes (a multiple of 4) with zeros; a kernel, so it can be captured
// in a graph.
void launch_zero(void *p, size_t nbytes, hipStream_t s);
// Zero every segment of a device table (max_n16: the longest, in 16-byte
// units).
struct ZeroSeg {
  void *p;
  size_t n16;
};
void launch_zero_segments(const ZeroSeg *segs, int nseg, size_t max_n16, hipStream_t s);
// ---- lab-frame snapshots (btd.hip) ------------------------------------------
template <typename T>
struct BtdJob {
  const T *F[6];          // real E, B of the run
  T *out;                 // [snapshot][Ex Ey Ez Bx By Bz][z][x][y]
  int *level;             // level of the fields in F; advanced by each launch
  int nx, ny, nz, nsnap;
  double t_lab0, dt_lab;  // snapshot j at lab time t_lab0 + j dt_lab
  double t0, dt;          // boosted time of level m: t0 + m dt
  double dz, gamma, beta;
  // particle records (off while pcap == 0)
  PartPtrs p;             // the run's particles
  int lx, ly, lz;         // log2 of nx, ny, nz (cell index decoding)
  int pcap;               // records per snapshot
  double dx, dy;
  T *pvals;               // [snapshot][x y z_lab u_x u_y u_z][pcap]
  int64_t *pids;          // [snapshot][pcap], or null
  int *pcount;            // [snapshot]: records made (past pcap: dropped)
};
// Add level m's share to the snapshots of every job, then advance the
// levels (max_snap, max_nxy: the largest snapshot count and nx*ny over the
// jobs).
template <typename T>
void launch_btd(const BtdJob<T> *jobs, int njobs, int max_snap, int64_t max_nxy, hipStream_t s);
// Record the particles whose last move crossed a snapshot's lab time, for
// every job with pcap > 0 (max_n: the largest particle count).
template <typename T>
void launch_btd_particles(const BtdJob<T> *jobs, int njobs, int64_t max_n, hipStream_t s);

// out[0] += sum of squares over n values of each of the three arrays.
template <typename T>
void launch_sum_squares(const T *a, const T *b, const T *c, int64_t n, double *out,
                        hipStream_t s);

// ---- slab field solve (slab.hip) ------------------------------------------
// Sums over the grid of J_x, J_y, J_z and rho of one run.
template <typename T>
struct SlabSum {
  const T *src[4];
  double *out;     // 4 sums, cleared by the caller
  int64_t ncell;
};
// One slab's window of a run's real grids: window plane j of slab run
// (nx x ny x nw) is global plane (first + j) mod nz; owned planes are
// window planes guard .. guard + ns - 1.
template <typename T>
struct SlabCopy {
  T *glob[10];          // the run's real E, B, J, rho
  T *win[10];           // the slab run's real arrays
  const double *sums;   // the run's SlabSum output (J, rho), mean = sum / ncell
  int nxy, nz, nw, first, ns, guard;
  double inv_ncell;
};
template <typename T>
void launch_slab_sums(const SlabSum<T> *sums, int nruns, int64_t max_cells, hipStream_t s);
// Windows of fields f0 .. f0 + nf - 1 (0-5 E, B; 6-8 J; 9 rho) into every
// slab of the table; J and rho lose their means.
template <typename T>
void launch_slab_window(const SlabCopy<T> *jobs, int njobs, int f0, int nf, int64_t max_win,
                        hipStream_t s);
// Owned planes of the slabs' E, B back into the runs' E, B.
template <typename T>
void launch_slab_interior(const SlabCopy<T> *jobs, int njobs, int64_t max_owned,
                          hipStream_t s);

// ---- field energy without allocation (noalloc.hip) ---------------------------
// Look up, once per device (the current one), the device address of the
// file-scope array the no-allocation entry point uses; cells it can take.
hipError_t noalloc_prepare();
double *noalloc_scratch(int device);
int64_t noalloc_max_cells();
// W_E, W_B (times dv / 2) of one run's real E, B into out[0..1] (device),
// through slots (the array above), on stream s; nothing allocated.
template <typename T>
void launch_energy_noalloc(const T *const E[3], const T *const B[3], int64_t ncell, double dv,
                           double *slots, double *out, hipStream_t s);

// ---- particles (particles.hip) ----------------------------------------------
template <typename T>
struct GridPtrs {
  T *E[3];
  T *B[3];
  T *J[3];
  T *rho;
};

// Particles are grouped by tiles of t[a] cells per axis; a tile's node
// region spans e[a] = t[a] + (shape width - 1) nodes per axis.
struct TileGeom {
  int t[3], lt[3], nt[3];
  int e[3];      // node region extents: tile + shape width - 1 + 2 margin
  int ce[3];     // bucket block extents: tile + 2 margin cells
  int margin;    // cells beyond the tile still covered by its node region
  int lcpt;      // log2 of cells per tile
  int n_tiles;
  int sx;        // x stride of the region's node slots: e[1] e[2] + pad
  int region;    // node slots of one region quantity: e[0] sx
  int nb;        // buckets (cells of the bucket block); bucket nb: beyond it
  int cap;       // particles the per-tile bucket list holds
};
// tile[a]: requested cells per tile (0: 8, or the grid if smaller)
TileGeom make_tile_geom(const RunGeom &g, size_t real_size, const int tile[3]);

// Device buffers of the tile sort of one run.
struct SortBufs {
  int *cell_count;  // n_cells: particles per (tile-major) cell
  int *cell_off;    // n_cells: first particle of the cell inside its tile
  int *tile_total;  // n_tiles
  int *start;       // n_tiles + 1: first particle of each tile, then the total
  int *key;         // n particles: tile-major cell index
  int *rank;        // n particles: rank inside the cell
  int *state;       // [0] fallback count, [1] sort flag, [2] sorts done, [3] force
  void *tmp[8];     // scratch columns for the scatter
};

// One run of a batched particle or sort launch: an entry of a device table.
template <typename T>
struct PartJob {
  RunGeom g;
  TileGeom tg;
  PartPtrs p;
  GridPtrs<T> gr;
  SortBufs sb;
  int block0;            // first workgroup of the run in a launch with one workgroup per tile
  int resort_threshold;  // re-sort when more particles than this used the global path
  T *regbuf;             // null: tiles add their regions by atomics; else the deposit
                         // and fused passes store them here ([tile][J_x J_y J_z rho][region])
};

// What the launchers need to know about a table of PartJobs.
struct PartBatch {
  int order;          // shape order (all runs of a context share it)
  int njobs;
  int nblocks;        // tiles of all runs
  int64_t max_n;      // most particles in one run
  int64_t max_cells;  // most cells in one run
  int max_tiles;      // most tiles in one run
  size_t lds[4];      // dynamic LDS of the particle kernel per mode: the most of any run
  int any_regbuf;     // some run stores its tile regions in a region buffer
  int fixed_geom;     // every run has the default cubic tile geometry
};
// True when tg is the default cubic 8x8x8 tile geometry for real_size (the
// particle kernel then has it as compile-time constants).
bool default_cubic_tiles(const TileGeom &tg, size_t real_size);

// Sort the particles of each run by tile when flagged (state[3] forces it;
// otherwise when more than n/64 particles used the global fallback since the
// last decision).  Every kernel checks the flag on the device, so the launch
// sequence is fixed and can be captured in a graph.
template <typename T>
void launch_sort(const PartJob<T> *jobs, const PartBatch &b, hipStream_t s);

enum { kPartRho = 0, kPartDeposit = 1, kPartFused = 2, kPartPush = 3 };
// Tile kernels over every run of the table: rho at the current positions;
// deposit (move, J, move, rho); fused (gather + push through dt_factor * dt,
// then deposit); push (gather + push through dt_factor * dt).  Deposits add
// into the grids, which the caller zeroes first.
template <typename T>
void launch_particles(int mode, const PartJob<T> *jobs, const PartBatch &b, double dt_factor,
                      hipStream_t s);
// After a deposit or fused pass: for every run with a region buffer, add the
// regions that hold each node into J and rho (which hold the global-path
// contributions of the pass).
template <typename T>
void launch_region_reduce(const PartJob<T> *jobs, const PartBatch &b, hipStream_t s);
// Dynamic LDS bytes of the particle kernel of a mode for one run's tiles.
template <typename T>
size_t particle_lds_bytes(int mode, const TileGeom &tg);

}  // namespace galpic
