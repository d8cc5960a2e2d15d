// Particle kernels: tile sort, deposition, gather and relativistic Boris push.
//
// Readings (the paper fixes the order and the equations, not these details):
//  - shape: tensor-product B-spline of order 1 or 3, nodes i..i+1 or
//    i-1..i+2 for a particle at i + delta; gather uses the same shape;
//  - J is deposited at the half-way position x + (v - v_gal) dt/2 with the
//    lab velocity v = u / gamma, rho at x + (v - v_gal) dt (two half moves);
//  - Boris: u- = u + h E, gamma- = sqrt(1 + |u-|^2), t = h B / gamma-,
//    s = 2 t / (1 + |t|^2), u' = u- + u- x t, u+ = u- + u' x s,
//    u_new = u+ + h E with h = q dt / (2 m) (c = 1).
//
// GPU design.  Particles are kept sorted by tile (8x8x8 cells).  One
// workgroup owns one tile: it stages the tile's node region (the tile plus
// the shape's halo and a drift margin) of E and B in LDS for the gather,
// orders its particles by current cell in LDS, accumulates J and rho in
// LDS, and adds the region into the global grid once at the end.  Groups of
// four lanes (quads) take four particles of one cell at a time, pairs of
// lanes a cell's remainder of one or two, and share that cell's node block
// between them (see the section on quads and pairs).  In mixed
// precision the per-tile sums are carried in double (no-return LDS
// atomics): the float roundings of a deposited value are those of the
// contributions of a quad's particles and their sum, and the final
// conversion; the tile sum itself adds no float rounding.  A particle whose shape
// support leaves its tile's region (it drifted since the last sort) uses
// global memory directly and is counted; the next step re-sorts when that
// count passes n/64.
//
// Position layouts: FP64 stores absolute doubles in [0, L); the mixed form
// stores an int32 linear cell index and float offsets in [0, 1), so that a
// particle static on the Galilean grid keeps its position exactly.
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace galpic {
namespace {

constexpr int kNT = 512;          // threads per workgroup of the per-tile sort scan
// per thread and round of the particle kernel's set-up: region nodes staged
// (three cover the 13^3 region of an 8^3 cubic tile, 13 x 172 slots with
// its padded x planes, at 768 threads) and particles bucketed
constexpr int kStageNodes = 3;
constexpr int kListParts = 4;       // particles per thread and round, FP64
constexpr int kListPartsFloat = 6;  // float: one round holds 4608 particles
constexpr size_t kLdsBytes = 160 * 1024;  // LDS of one workgroup on gfx950
// threads per tile workgroup of the particle kernel, one workgroup per CU
// (its LDS): the fused float kernel needs about 160 registers per lane, so
// 768 threads (3 waves per SIMD, at most 168 registers) fit without
// spilling and hide LDS latency better than 512 (5 % faster steps); the
// double one needs ~234 and stays at 512; 1024 threads would cap them at
// 128 and spill
constexpr int quad_threads(size_t real_size) { return real_size == 4 ? 768 : 512; }
// static bucket-scan buffer of that workgroup
constexpr size_t scan_bytes(size_t real_size) { return quad_threads(real_size) * sizeof(int); }

template <int ORDER, typename T>
struct Shape;

template <typename T>
struct Shape<1, T> {
  static constexpr int N = 2;
  static constexpr int FIRST = 0;
  __device__ __forceinline__ static void weights(T d, T *w) {
    w[0] = T(1) - d;
    w[1] = d;
  }
};

template <typename T>
struct Shape<3, T> {
  static constexpr int N = 4;
  static constexpr int FIRST = -1;
  __device__ __forceinline__ static void weights(T d, T *w) {
    const T e = T(1) - d;
    const T d2 = d * d;
    w[0] = e * e * e * T(1.0 / 6.0);
    w[1] = T(2.0 / 3.0) + d2 * (T(0.5) * d - T(1));
    w[2] = T(1.0 / 6.0) + T(0.5) * d * (T(1) + d - d2);
    w[3] = d2 * d * T(1.0 / 6.0);
  }
};

// A position as cell (ix, iy, iz) plus in-cell offset.
template <typename T>
struct CellPos {
  int i[3];
  T o[3];
};

__device__ __forceinline__ void decode_cell(int cell, const RunGeom &g, int i[3]) {
  i[2] = cell & (g.nz - 1);
  i[1] = (cell >> g.lz) & (g.ny - 1);
  i[0] = cell >> (g.lz + g.ly);
}
__device__ __forceinline__ int encode_cell(const int i[3], const RunGeom &g) {
  return (((i[0] << g.ly) | i[1]) << g.lz) | i[2];
}

// ---- FP64 layout: absolute positions ---------------------------------------
struct LayoutAbs {
  using T = double;
  struct State {
    double x[3];
  };
  __device__ __forceinline__ static State load(const PartPtrs &p, int64_t k) {
    State s;
    s.x[0] = static_cast<const double *>(p.x)[k];
    s.x[1] = static_cast<const double *>(p.y)[k];
    s.x[2] = static_cast<const double *>(p.z)[k];
    return s;
  }
  // what the bucket pass reads of a particle (its position) and the cell
  using Key = State;
  __device__ __forceinline__ static Key load_key(const PartPtrs &p, int64_t k) {
    return load(p, k);
  }
  __device__ __forceinline__ static void key_cell(const Key &s, const RunGeom &g, int i[3]) {
    const CellPos<double> c = cell(s, g);
#pragma unroll
    for (int a = 0; a < 3; ++a) i[a] = c.i[a];
  }
  __device__ __forceinline__ static void store(const PartPtrs &p, int64_t k, const State &s) {
    static_cast<double *>(p.x)[k] = s.x[0];
    static_cast<double *>(p.y)[k] = s.x[1];
    static_cast<double *>(p.z)[k] = s.x[2];
  }
  __device__ __forceinline__ static double wrap(double x, double L) {
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
  }
  // x += (v - v_gal) dt / 2, periodic
  __device__ __forceinline__ static void half_move(State &s, const double v[3],
                                                   const RunGeom &g) {
    const double h = 0.5 * g.dt;
    s.x[0] = wrap(s.x[0] + (v[0] - g.vgal[0]) * h, g.nx * g.dx);
    s.x[1] = wrap(s.x[1] + (v[1] - g.vgal[1]) * h, g.ny * g.dy);
    s.x[2] = wrap(s.x[2] + (v[2] - g.vgal[2]) * h, g.nz * g.dz);
  }
  __device__ __forceinline__ static CellPos<double> cell(const State &s, const RunGeom &g) {
    CellPos<double> c;
    const double q[3] = {s.x[0] / g.dx, s.x[1] / g.dy, s.x[2] / g.dz};
    const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double f = floor(q[a]);
      c.o[a] = q[a] - f;
      c.i[a] = int(f) & (n[a] - 1);
    }
    return c;
  }
};

// ---- mixed layout: int32 cell + float offsets ------------------------------
struct LayoutCell {
  using T = float;
  struct State {
    int i[3];
    float o[3];
  };
  __device__ __forceinline__ static State load(const PartPtrs &p, int64_t k, const RunGeom &g) {
    State s;
    decode_cell(static_cast<const int *>(p.x)[k], g, s.i);
    s.o[0] = static_cast<const float *>(p.ox)[k];
    s.o[1] = static_cast<const float *>(p.oy)[k];
    s.o[2] = static_cast<const float *>(p.oz)[k];
    return s;
  }
  // what the bucket pass reads of a particle (its cell word) and the cell
  using Key = int;
  __device__ __forceinline__ static Key load_key(const PartPtrs &p, int64_t k) {
    return static_cast<const int *>(p.x)[k];
  }
  __device__ __forceinline__ static void key_cell(Key w, const RunGeom &g, int i[3]) {
    decode_cell(w, g, i);
  }
  __device__ __forceinline__ static void store(const PartPtrs &p, int64_t k, const State &s,
                                               const RunGeom &g) {
    static_cast<int *>(p.x)[k] = encode_cell(s.i, g);
    static_cast<float *>(p.ox)[k] = s.o[0];
    static_cast<float *>(p.oy)[k] = s.o[1];
    static_cast<float *>(p.oz)[k] = s.o[2];
  }
  // offset += (v - v_gal) dt / (2 d) cells; carry into the cell index
  __device__ __forceinline__ static void half_move(State &s, const float v[3], const RunGeom &g) {
    const float d[3] = {(v[0] - float(g.vgal[0])) * float(0.5 * g.dt / g.dx),
                        (v[1] - float(g.vgal[1])) * float(0.5 * g.dt / g.dy),
                        (v[2] - float(g.vgal[2])) * float(0.5 * g.dt / g.dz)};
    const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float x = s.o[a] + d[a];
      const float f = floorf(x);
      x -= f;
      int carry = int(f);
      if (x >= 1.0f) {  // a tiny negative offset rounded up to 1
        x = 0.0f;
        carry += 1;
      }
      s.o[a] = x;
      s.i[a] = (s.i[a] + carry) & (n[a] - 1);
    }
  }
  __device__ __forceinline__ static CellPos<float> cell(const State &s, const RunGeom &) {
    CellPos<float> c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c.i[a] = s.i[a];
      c.o[a] = s.o[a];
    }
    return c;
  }
};

template <class L>
__device__ __forceinline__ typename L::State load_state(const PartPtrs &p, int64_t k,
                                                        const RunGeom &g) {
  if constexpr (sizeof(typename L::T) == 8)
    return L::load(p, k);
  else
    return L::load(p, k, g);
}
template <class L>
__device__ __forceinline__ void store_state(const PartPtrs &p, int64_t k,
                                            const typename L::State &s, const RunGeom &g) {
  if constexpr (sizeof(typename L::T) == 8)
    L::store(p, k, s);
  else
    L::store(p, k, s, g);
}

template <typename T>
__device__ __forceinline__ void boris(T u[3], const T F[6], T h) {
  T um[3] = {u[0] + h * F[0], u[1] + h * F[1], u[2] + h * F[2]};
  const T gamma = sqrt(T(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const T f = h / gamma;
  const T t[3] = {f * F[3], f * F[4], f * F[5]};
  const T s2 = T(2) / (T(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const T s[3] = {s2 * t[0], s2 * t[1], s2 * t[2]};
  const T up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                   um[2] + (um[0] * t[1] - um[1] * t[0])};
  um[0] += up[1] * s[2] - up[2] * s[1];
  um[1] += up[2] * s[0] - up[0] * s[2];
  um[2] += up[0] * s[1] - up[1] * s[0];
  u[0] = um[0] + h * F[0];
  u[1] = um[1] + h * F[1];
  u[2] = um[2] + h * F[2];
}

// ---- tile geometry ---------------------------------------------------------
// Region of a tile: nodes org[a] .. org[a] + e[a] - 1 (mod n) per axis, with
// org = tile start + FIRST - margin, e = tile + (N - 1) + 2 margin.  A
// particle in cell i touches nodes i + FIRST .. i + FIRST + N - 1; it is
// inside when all of them fall in the region, which holds for particles up
// to `margin` cells outside their tile.  Slots are distinct accumulators even
// if e > n (duplicates add).
struct Region {
  int org[3];
};

// A value of a table that no kernel writes during the launch, read through
// the constant address space (word by word): the loads need not wait behind
// the kernel's own stores and may be hoisted or repeated freely.
template <typename V>
__device__ __forceinline__ V load_const(const V *ptr) {
  static_assert(sizeof(V) % 4 == 0, "whole words");
  using CU = __attribute__((address_space(4))) const unsigned;
  CU *q = (CU *)ptr;
  V v;
  unsigned *d = reinterpret_cast<unsigned *>(&v);
#pragma unroll
  for (size_t i = 0; i < sizeof(V) / 4; ++i) d[i] = q[i];
  return v;
}

// The buffers of a run's table entry as global pointers.
__device__ __forceinline__ void globalize(PartPtrs &p) {
  p.x = global_ptr(p.x);
  p.y = global_ptr(p.y);
  p.z = global_ptr(p.z);
  p.ox = global_ptr(p.ox);
  p.oy = global_ptr(p.oy);
  p.oz = global_ptr(p.oz);
  p.ux = global_ptr(p.ux);
  p.uy = global_ptr(p.uy);
  p.uz = global_ptr(p.uz);
  p.id = global_ptr(p.id);
}
template <typename T>
__device__ __forceinline__ void globalize(GridPtrs<T> &g) {
  for (int a = 0; a < 3; ++a) {
    g.E[a] = global_ptr(g.E[a]);
    g.B[a] = global_ptr(g.B[a]);
    g.J[a] = global_ptr(g.J[a]);
  }
  g.rho = global_ptr(g.rho);
}
__device__ __forceinline__ void globalize(SortBufs &b) {
  b.cell_count = global_ptr(b.cell_count);
  b.cell_off = global_ptr(b.cell_off);
  b.tile_total = global_ptr(b.tile_total);
  b.start = global_ptr(b.start);
  b.key = global_ptr(b.key);
  b.rank = global_ptr(b.rank);
  b.state = global_ptr(b.state);
  for (int c = 0; c < 8; ++c) b.tmp[c] = global_ptr(b.tmp[c]);
}

// Run of a batched launch that owns workgroup b: the last job whose first
// workgroup is at or before b (block0 ascends).
template <typename J>
__device__ __forceinline__ int job_of_block(const J *jobs, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tile of the run's b-th workgroup.  XCD-aware: consecutive workgroups go
// to different XCDs round-robin; give each XCD a contiguous run of tiles so
// neighbours share its L2.
__device__ __forceinline__ int tile_of_block(const TileGeom &tg, int b) {
  if ((tg.n_tiles & 7) != 0) return b;
  const int per = tg.n_tiles >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ Region region_of(int tile, const TileGeom &tg, const RunGeom &g,
                                            int first) {
  Region r;
  const int tz = tile % tg.nt[2];
  const int ty = (tile / tg.nt[2]) % tg.nt[1];
  const int tx = tile / (tg.nt[2] * tg.nt[1]);
  r.org[0] = (tx * tg.t[0] + first - tg.margin) & (g.nx - 1);
  r.org[1] = (ty * tg.t[1] + first - tg.margin) & (g.ny - 1);
  r.org[2] = (tz * tg.t[2] + first - tg.margin) & (g.nz - 1);
  return r;
}

// region-local first support node of cell c; false if the support leaves
// the region
template <int ORDER, typename T>
__device__ __forceinline__ bool region_base(const CellPos<T> &c, const Region &r,
                                            const TileGeom &tg, const RunGeom &g, int hb[3]) {
  using Sh = Shape<ORDER, T>;
  const int n[3] = {g.nx, g.ny, g.nz};
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    hb[a] = (c.i[a] + Sh::FIRST - r.org[a]) & (n[a] - 1);
    in = in && (hb[a] + Sh::N <= tg.e[a]);
  }
  return in;
}

template <int ORDER, typename T>
struct Support {
  using Sh = Shape<ORDER, T>;
  T w[3][Sh::N];
  int base[3];  // region-local index of the first node per axis
  bool inside;
};

template <int ORDER, typename T>
__device__ __forceinline__ void support_of(const CellPos<T> &c, const Region &r,
                                           const TileGeom &tg, const RunGeom &g,
                                           Support<ORDER, T> &s) {
  using Sh = Shape<ORDER, T>;
  const int n[3] = {g.nx, g.ny, g.nz};
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Sh::weights(c.o[a], s.w[a]);
    const int rel = (c.i[a] + Sh::FIRST - r.org[a]) & (n[a] - 1);
    s.base[a] = rel;
    in = in && (rel + Sh::N <= tg.e[a]);
  }
  s.inside = in;
}

// ---- accumulation ----------------------------------------------------------
// Deposit nq values (val[q] * weight) into LDS accumulators q0.. of the
// region (type A: double, also for float contributions) or, outside
// the region, straight into the global grids dst[q].
template <int ORDER, typename T, typename A>
__device__ __forceinline__ void deposit(const CellPos<T> &c, const Support<ORDER, T> &s,
                                        const TileGeom &tg, const RunGeom &g, A *acc, int q0,
                                        int nq, const T *val, T *const *dst, int *fallback) {
  using Sh = Shape<ORDER, T>;
  if (s.inside) {
    const int R = tg.region;
#pragma unroll
    for (int a = 0; a < Sh::N; ++a) {
#pragma unroll
      for (int b = 0; b < Sh::N; ++b) {
        const T wab = s.w[0][a] * s.w[1][b];
        const int row = (s.base[0] + a) * tg.sx + (s.base[1] + b) * tg.e[2] + s.base[2];
#pragma unroll
        for (int e = 0; e < Sh::N; ++e) {
          const T w = wab * s.w[2][e];
          for (int q = 0; q < nq; ++q)
            __hip_atomic_fetch_add(acc + size_t(q0 + q) * R + row + e, A(w * val[q]),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  } else {
    atomicAdd(fallback, 1);
#pragma unroll
    for (int a = 0; a < Sh::N; ++a) {
      const int ix = (c.i[0] + Sh::FIRST + a) & (g.nx - 1);
#pragma unroll
      for (int b = 0; b < Sh::N; ++b) {
        const int iy = (c.i[1] + Sh::FIRST + b) & (g.ny - 1);
        const T wab = s.w[0][a] * s.w[1][b];
        const int64_t row = (int64_t(ix) * g.ny + iy) * g.nz;
#pragma unroll
        for (int e = 0; e < Sh::N; ++e) {
          const int iz = (c.i[2] + Sh::FIRST + e) & (g.nz - 1);
          const T w = wab * s.w[2][e];
          for (int q = 0; q < nq; ++q) unsafeAtomicAdd(dst[q] + row + iz, w * val[q]);
        }
      }
    }
  }
}

template <int ORDER, typename T>
__device__ __forceinline__ void gather(const CellPos<T> &c, const Support<ORDER, T> &s,
                                       const TileGeom &tg, const RunGeom &g, const T *fld,
                                       const GridPtrs<T> &gr, T F[6]) {
  using Sh = Shape<ORDER, T>;
#pragma unroll
  for (int q = 0; q < 6; ++q) F[q] = T(0);
  if (s.inside) {
    const int R = tg.region;
#pragma unroll
    for (int a = 0; a < Sh::N; ++a) {
#pragma unroll
      for (int b = 0; b < Sh::N; ++b) {
        const T wab = s.w[0][a] * s.w[1][b];
        const int row = (s.base[0] + a) * tg.sx + (s.base[1] + b) * tg.e[2] + s.base[2];
#pragma unroll
        for (int e = 0; e < Sh::N; ++e) {
          const T w = wab * s.w[2][e];
#pragma unroll
          for (int q = 0; q < 6; ++q) F[q] += w * fld[q * R + row + e];
        }
      }
    }
  } else {
    const T *src[6] = {gr.E[0], gr.E[1], gr.E[2], gr.B[0], gr.B[1], gr.B[2]};
#pragma unroll
    for (int a = 0; a < Sh::N; ++a) {
      const int ix = (c.i[0] + Sh::FIRST + a) & (g.nx - 1);
#pragma unroll
      for (int b = 0; b < Sh::N; ++b) {
        const int iy = (c.i[1] + Sh::FIRST + b) & (g.ny - 1);
        const T wab = s.w[0][a] * s.w[1][b];
        const int64_t row = (int64_t(ix) * g.ny + iy) * g.nz;
#pragma unroll
        for (int e = 0; e < Sh::N; ++e) {
          const int iz = (c.i[2] + Sh::FIRST + e) & (g.nz - 1);
          const T w = wab * s.w[2][e];
#pragma unroll
          for (int q = 0; q < 6; ++q) F[q] += w * src[q][row + iz];
        }
      }
    }
  }
}

// region slot -> global node index (a pad slot at the end of an x plane
// maps to a node of the plane's last row; nothing is deposited there, and
// what is staged there is never read)
__device__ __forceinline__ int64_t region_node(int r, const Region &rg, const TileGeom &tg,
                                               const RunGeom &g) {
  const int ax = r / tg.sx;
  const int rem = r - ax * tg.sx;
  const int ay = min(rem / tg.e[2], tg.e[1] - 1);
  const int az = rem % tg.e[2];
  const int ix = (rg.org[0] + ax) & (g.nx - 1);
  const int iy = (rg.org[1] + ay) & (g.ny - 1);
  const int iz = (rg.org[2] + az) & (g.nz - 1);
  return (int64_t(ix) * g.ny + iy) * g.nz + iz;
}

enum { kModeRho = 0, kModeDeposit = 1, kModeFused = 2, kModePush = 3 };

// ---- quads and pairs ------------------------------------------------------------
// Lanes 4k .. 4k+3 of a wave form a quad.  A group of G lanes (G = 4: the
// quad; G = 2: lanes 4k, 4k+1 or 4k+2, 4k+3) takes up to G particles of one
// cell at a time, one per lane.  While they share a cell they share its N^3
// node block, and lane m of the group works on a G-th of the block (its
// N*N/G (x, y) node rows) for all of the group's particles: the gather reads
// every node of the block once per group instead of once per particle, and
// the deposit adds the group's contributions to a node in registers before
// one LDS atomic.  In slot s (0 .. G-1) lane m handles the particle of lane
// (m - s) mod G; weights, values and partial sums move between lanes by DPP
// permutations inside the quad (no LDS traffic).  A group whose particles
// do not share a block inside the tile's region falls back to one particle
// per lane.  Quads take a cell's particles four at a time; a remainder of
// one or two particles goes to a pair, so that two such remainders fill one
// quad's lanes.

template <int CTRL>
__device__ __forceinline__ int dpp_int(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_val(float v) {
  return __int_as_float(dpp_int<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_val(double v) {
  const int lo = __double2loint(v);
  const int hi = __double2hiint(v);
  return __hiloint2double(dpp_int<CTRL>(hi), dpp_int<CTRL>(lo));
}
// quad_perm controls: lane m reads lane (m - s) mod G ...
template <int G, typename V>
__device__ __forceinline__ V from_minus(V v, int s) {
  if constexpr (G == 2) {
    return s == 0 ? v : dpp_val<0xB1>(v);  // [1,0,3,2]
  } else {
    switch (s) {
      case 0: return v;
      case 1: return dpp_val<0x93>(v);  // [3,0,1,2]
      case 2: return dpp_val<0x4E>(v);  // [2,3,0,1]
      default: return dpp_val<0x39>(v);  // [1,2,3,0]
    }
  }
}
// ... or lane (m + s) mod G
template <int G, typename V>
__device__ __forceinline__ V from_plus(V v, int s) {
  if constexpr (G == 2) {
    return s == 0 ? v : dpp_val<0xB1>(v);
  } else {
    switch (s) {
      case 0: return v;
      case 1: return dpp_val<0x39>(v);
      case 2: return dpp_val<0x4E>(v);
      default: return dpp_val<0x93>(v);
    }
  }
}
// the group's first lane's value, and whether b holds on every lane of it
template <int G>
__device__ __forceinline__ int lead_int(int v) {
  return G == 2 ? dpp_int<0xA0>(v) : dpp_int<0x00>(v);  // [0,0,2,2] or [0,0,0,0]
}
template <int G>
__device__ __forceinline__ bool group_all(bool b) {
  int v = b ? 1 : 0;
  v &= dpp_int<0xB1>(v);  // [1,0,3,2]
  if constexpr (G == 4) v &= dpp_int<0x4E>(v);
  return v != 0;
}

// The group shares one node block when every lane's block starts at the
// same region-local node and lies inside the region.
template <int ORDER, typename T, int G>
__device__ __forceinline__ bool group_block(const CellPos<T> &c, const Region &rg,
                                            const TileGeom &tg, const RunGeom &g, int hb[3]) {
  const bool in = region_base<ORDER, T>(c, rg, tg, g, hb);
  const int key = hb[0] * tg.sx + hb[1] * tg.e[2] + hb[2];
  return group_all<G>(in && key == lead_int<G>(key));
}

// Weights of the group's particles for lane m's rows: slot s holds the
// particle of lane (m - s) mod G with wxy[s][r] = wx(a) wy(b) for row r
// (row m*ROWS + r of the block, a = row / N, b = row % N) and wz[s][e].
template <int ORDER, typename T, int G>
struct GroupWeights {
  using Sh = Shape<ORDER, T>;
  static constexpr int N = Sh::N;
  static constexpr int ROWS = N * N / G;
  T wxy[G][ROWS];
  T wz[G][N];
  // w[i] by selects on the bits of i (a chain of equality tests can be
  // folded into a private-memory table lookup)
  __device__ __forceinline__ static T pick(const T (&w)[N], int i) {
    const T lo = (i & 1) ? w[1] : w[0];
    if constexpr (N == 2) {
      return lo;
    } else {
      const T hi = (i & 1) ? w[3] : w[2];
      return (i & 2) ? hi : lo;
    }
  }
  __device__ __forceinline__ void build(const T o[3], int m) {
    T wx[N], wy[N], wzo[N];
    Sh::weights(o[0], wx);
    Sh::weights(o[1], wy);
    Sh::weights(o[2], wzo);
#pragma unroll
    for (int s = 0; s < G; ++s) {
      // this lane's particle goes to slot s of lane (m + s) mod G: send
      // that lane's row weights
      const int dst = (m + s) & (G - 1);
      T send[ROWS];
      if constexpr (ROWS % N == 0) {
        // rows dst*ROWS .. +ROWS-1 cover ROWS/N values of a, all of b
#pragma unroll
        for (int ia = 0; ia < ROWS / N; ++ia) {
          const T wxa = pick(wx, dst * (ROWS / N) + ia);
#pragma unroll
          for (int b = 0; b < N; ++b) send[ia * N + b] = wxa * wy[b];
        }
      } else {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          const int row = dst * ROWS + r;
          send[r] = pick(wx, row / N) * pick(wy, row % N);
        }
      }
#pragma unroll
      for (int r = 0; r < ROWS; ++r) wxy[s][r] = from_minus<G>(send[r], s);
#pragma unroll
      for (int e = 0; e < N; ++e) wz[s][e] = from_minus<G>(wzo[e], s);
    }
  }
};

// region-local index of the first node of lane m's row r in the block hb
template <int ORDER, int G>
__device__ __forceinline__ int group_row(const int hb[3], int m, int r, const TileGeom &tg) {
  constexpr int N = ORDER == 1 ? 2 : 4;
  constexpr int ROWS = N * N / G;
  const int row = m * ROWS + r;
  return (hb[0] + row / N) * tg.sx + (hb[1] + row % N) * tg.e[2] + hb[2];
}

// E and B of the group's particles from the shared block; every lane gets
// its own particle's six values.
template <int ORDER, typename T, int G>
__device__ __forceinline__ void gather_group(const int hb[3], const T o[3], int m,
                                             const TileGeom &tg, const T *fld, T F[6]) {
  using GW = GroupWeights<ORDER, T, G>;
  constexpr int N = GW::N;
  GW w;
  w.build(o, m);
  const int R = __builtin_amdgcn_readfirstlane(tg.region);
  T P[G][6];
#pragma unroll
  for (int s = 0; s < G; ++s)
#pragma unroll
    for (int q = 0; q < 6; ++q) P[s][q] = T(0);
#pragma unroll
  for (int r = 0; r < GW::ROWS; ++r) {
    const T *row = fld + group_row<ORDER, G>(hb, m, r, tg);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      T f[N];
#pragma unroll
      for (int e = 0; e < N; ++e) f[e] = row[q * R + e];
#pragma unroll
      for (int s = 0; s < G; ++s) {
        T acc = P[s][q];
#pragma unroll
        for (int e = 0; e < N; ++e) acc += (w.wxy[s][r] * w.wz[s][e]) * f[e];
        P[s][q] = acc;
      }
    }
  }
  // the particle of lane m sits in slot s of lane (m + s) mod G
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    T v = P[0][q];
#pragma unroll
    for (int s = 1; s < G; ++s) v += from_plus<G>(P[s][q], s);
    F[q] = v;
  }
}

// Deposit NQ values per particle (val, zero for an idle lane) of the
// group's particles into the shared block hb of LDS accumulators q0 ..
template <int ORDER, typename T, typename A, int NQ, int G>
__device__ __forceinline__ void deposit_group(const int hb[3], const T o[3], const T val[NQ],
                                              int m, const TileGeom &tg, A *acc, int q0) {
  using GW = GroupWeights<ORDER, T, G>;
  constexpr int N = GW::N;
  GW w;
  w.build(o, m);
  T vs[G][NQ];
#pragma unroll
  for (int s = 0; s < G; ++s)
#pragma unroll
    for (int q = 0; q < NQ; ++q) vs[s][q] = from_minus<G>(val[q], s);
  const int R = __builtin_amdgcn_readfirstlane(tg.region);
  // the z weight goes into the values once per node plane e, the row
  // weight per node: G * NQ multiplies per plane instead of one weight
  // product per node and slot
#pragma unroll
  for (int e = 0; e < N; ++e) {
    T vz[G][NQ];
#pragma unroll
    for (int s = 0; s < G; ++s)
#pragma unroll
      for (int q = 0; q < NQ; ++q) vz[s][q] = w.wz[s][e] * vs[s][q];
#pragma unroll
    for (int r = 0; r < GW::ROWS; ++r) {
      const int row = group_row<ORDER, G>(hb, m, r, tg);
      T sum[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) sum[q] = w.wxy[0][r] * vz[0][q];
#pragma unroll
      for (int s = 1; s < G; ++s)
#pragma unroll
        for (int q = 0; q < NQ; ++q) sum[q] += w.wxy[s][r] * vz[s][q];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        __hip_atomic_fetch_add(acc + size_t(q0 + q) * R + row + e, A(sum[q]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// Deposit of NQ values at position c: the group's shared block if it has
// one, else one particle per lane (an idle lane deposits nothing).
template <int ORDER, typename T, typename A, int NQ, int G>
__device__ __forceinline__ void deposit_at(const CellPos<T> &c, const T val[NQ], bool act,
                                           int m, const Region &rg, const TileGeom &tg,
                                           const RunGeom &g, A *acc, int q0, T *const *dst,
                                           int *fallback) {
  int hb[3];
  if (group_block<ORDER, T, G>(c, rg, tg, g, hb)) {
    T v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = act ? val[q] : T(0);
    deposit_group<ORDER, T, A, NQ, G>(hb, c.o, v, m, tg, acc, q0);
  } else if (act) {
    Support<ORDER, T> s;
    support_of<ORDER, T>(c, rg, tg, g, s);
    deposit<ORDER, T, A>(c, s, tg, g, acc, q0, NQ, val, dst, fallback);
  }
}

// ---- per-tile bucket order ---------------------------------------------------
// At the start of every particle pass the workgroup orders its tile's
// particles by their current cell in LDS (a counting sort of tile-local
// indices), so the quads find four particles of one cell however far the
// particles have moved inside the region since the last global sort.
// Buckets are the cells of the tile plus the drift margin, and one bucket
// for particles beyond it.  A bucket of c particles gives c / 4 quad jobs
// of four, one more quad job of three when c mod 4 = 3, and a pair job of
// one or two when c mod 4 is 1 or 2.  The quad jobs come first in the job
// table, then the pair jobs; a quad takes either one quad job or two pair
// jobs.  A tile with more particles than the list holds is processed in
// memory order instead, by quads only.
struct TileLists {
  int *off;    // nb + 2: first list entry of each bucket
  int *job;    // nb + 2: first quad job | first pair job << 16 of each bucket
  int *fill;   // nb + 1: counts, then fill pointers
  unsigned short *list;  // cap tile-local particle indices
  int *jobs;   // cap / 4 + nb + 2: first list entry | size << 24 of each job
};

// LDS bytes of the bucket tables and lists of a tile geometry
__host__ __device__ constexpr size_t list_bytes(int nb, int cap) {
  return size_t(3) * (nb + 2) * sizeof(int) + ((size_t(cap) * 2 + 3) & ~size_t(3)) +
         (size_t(cap) / 4 + nb + 2) * sizeof(int);
}

template <class L>
__device__ __forceinline__ int bucket_of_key(const typename L::Key &key, const RunGeom &g,
                                             const TileGeom &tg, const int org[3]) {
  int i[3];
  L::key_cell(key, g, i);
  const int n[3] = {g.nx, g.ny, g.nz};
  int b = 0;
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int rel = (i[a] - org[a]) & (n[a] - 1);
    in = in && rel < tg.ce[a];
    b = b * tg.ce[a] + rel;
  }
  return in ? b : tg.nb;
}

template <class L>
__device__ __forceinline__ int bucket_of(const PartPtrs &p, int64_t k, const RunGeom &g,
                                         const TileGeom &tg, const int org[3]) {
  return bucket_of_key<L>(L::load_key(p, k), g, tg, org);
}

// Two exclusive scans at once (n < 2 NT): pack(i) gives the two values of
// entry i (i < n; zero past it), and store(i, a, b) receives the two prefix
// sums of every i in [0, n].  Each thread takes a pair of entries, waves
// scan their pair sums with lane shuffles, one wave scans the wave totals
// of both (lanes 0.. and 32..; tmp[0 .. 2 NT/64)), three barriers in all;
// pack runs before the first and store after the second.
template <int NT, class Pack, class Store>
__device__ __forceinline__ void scan_pair(int n, Pack pack, Store store, int *tmp) {
  constexpr int W = NT / 64;
  static_assert(NT % 64 == 0 && W <= 32, "whole waves, at most 32");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int a0 = 0, b0 = 0, a1 = 0, b1 = 0;
  if (2 * tid < n) pack(2 * tid, a0, b0);
  if (2 * tid + 1 < n) pack(2 * tid + 1, a1, b1);
  int xa = a0 + a1, xb = b0 + b1;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int ya = __shfl_up(xa, off, 64);
    const int yb = __shfl_up(xb, off, 64);
    if (lane >= off) {
      xa += ya;
      xb += yb;
    }
  }
  if (lane == 63) {
    tmp[wave] = xa;
    tmp[W + wave] = xb;
  }
  __syncthreads();
  if (wave == 0) {
    const int half = lane >> 5, k = lane & 31;
    int t = k < W ? tmp[half * W + k] : 0;
#pragma unroll
    for (int off = 1; off < W; off <<= 1) {
      const int y = __shfl_up(t, off, 32);
      if (k >= off) t += y;
    }
    if (k < W) tmp[half * W + k] = t;
  }
  __syncthreads();
  const int ea = xa + (wave ? tmp[wave - 1] : 0) - a0 - a1;
  const int eb = xb + (wave ? tmp[W + wave - 1] : 0) - b0 - b1;
  if (2 * tid <= n) store(2 * tid, ea, eb);
  if (2 * tid + 1 <= n) store(2 * tid + 1, ea + a0, eb + b0);
  __syncthreads();
}

// The default cubic tile geometry (8x8x8 cells; float: one cell of drift
// margin, 13^3 nodes; double: no margin, 11^3 nodes; x planes padded to
// 172 or 124 slots), written over the grid-independent fields of tg.  A
// kernel built for it folds every region index to constants, which keeps
// the fused float kernel within 168 registers.
template <typename T>
struct DefaultCubicTiles {
  static constexpr int kMargin = sizeof(T) == 4 ? 1 : 0;
  static constexpr int kE = 8 + 3 + 2 * kMargin;
  static constexpr int kCe = 8 + 2 * kMargin;
  static constexpr int kSx = kE * kE + (12 - (kE * kE) % 8) % 8;
  __host__ __device__ static void write(TileGeom &tg) {
    for (int a = 0; a < 3; ++a) {
      tg.t[a] = 8;
      tg.lt[a] = 3;
      tg.e[a] = kE;
      tg.ce[a] = kCe;
    }
    tg.margin = kMargin;
    tg.lcpt = 9;
    tg.sx = kSx;
    tg.region = kE * kSx;
    tg.nb = kCe * kCe * kCe;
  }
  static bool matches(const TileGeom &tg) {
    TileGeom d = tg;
    write(d);
    for (int a = 0; a < 3; ++a)
      if (d.t[a] != tg.t[a] || d.lt[a] != tg.lt[a] || d.e[a] != tg.e[a] || d.ce[a] != tg.ce[a])
        return false;
    return d.margin == tg.margin && d.lcpt == tg.lcpt && d.sx == tg.sx &&
           d.region == tg.region && d.nb == tg.nb;
  }
};

// One workgroup of NT threads per tile.  Modes:
//  rho:     rho at the current positions (no move)
//  deposit: move dt/2, J; move dt/2, rho; positions written
//  fused:   gather at the current positions and push u through dt, then as
//           deposit with the new u (one pass over the particles per step)
//  push:    gather and push u through the time step h was built for
template <class L, int ORDER, int MODE, typename A, int NT, bool FIX>
__global__ __launch_bounds__(NT) void k_quad(const PartJob<typename L::T> *__restrict__ jobs,
                                             int njobs, double dt_factor) {
  using T = typename L::T;
  using Sh = Shape<ORDER, T>;
  // the run's entry of the table, through the constant address space
  using CJob = __attribute__((address_space(4))) const PartJob<T>;
  CJob *cjobs = (CJob *)jobs;
  const PartJob<T> *jp = jobs + job_of_block(cjobs, njobs, blockIdx.x);
  const RunGeom g = load_const(&jp->g);
  TileGeom tg = load_const(&jp->tg);
  if constexpr (FIX) DefaultCubicTiles<typename L::T>::write(tg);  // the same values, as constants
  PartPtrs p = load_const(&jp->p);
  globalize(p);
  GridPtrs<T> gr = load_const(&jp->gr);
  globalize(gr);
  const int *__restrict__ start = global_ptr(load_const(&jp->sb.start));
  int *state = global_ptr(load_const(&jp->sb.state));
  const int block0 = load_const(&jp->block0);
  const T h = T(p.q * (dt_factor * g.dt) / (2.0 * p.m));
  constexpr bool kGather = MODE == kModeFused || MODE == kModePush;
  constexpr bool kDeposit = MODE != kModePush;
  constexpr bool kMove = MODE == kModeFused || MODE == kModeDeposit;
  // pair jobs and the job table by rounds (float particles only)
  constexpr bool kSpread = sizeof(T) == 4;
  // float particles: the staged E and B go to LDS after the bucket scans
  // and the placement pass instead of after the count pass (FP64, whose
  // tiles more often take several rounds of the count pass, measured
  // slower so)
  constexpr bool kLateStore = sizeof(T) == 4;
  static_assert(2 * NT >= 1024, "bucket scan covers up to 2 NT buckets");
  extern __shared__ __align__(16) unsigned char smem[];
  // accumulators first (8-byte aligned when A is double), then the fields,
  // then the bucket lists
  const int R = __builtin_amdgcn_readfirstlane(tg.region);
  A *acc = reinterpret_cast<A *>(smem);  // 4 * region
  unsigned char *after_acc = smem + (kDeposit ? 4 * sizeof(A) * R : 0);
  T *fld = reinterpret_cast<T *>(after_acc);
  unsigned char *after_fld = after_acc + (kGather ? 6 * sizeof(T) * R : 0);
  TileLists tl;
  tl.off = reinterpret_cast<int *>(after_fld);
  tl.job = tl.off + (tg.nb + 2);
  tl.fill = tl.job + (tg.nb + 2);
  tl.list = reinterpret_cast<unsigned short *>(tl.fill + (tg.nb + 2));
  tl.jobs = reinterpret_cast<int *>(tl.list + ((tg.cap + 1) & ~1));
  __shared__ int scan_tmp[NT];

  const int tile = tile_of_block(tg, int(blockIdx.x) - block0);
  const Region rg = region_of(tile, tg, g, Sh::FIRST);
  const T qw = T(p.q * p.w / (g.dx * g.dy * g.dz));
  const int tid = threadIdx.x;
  const int64_t tbase = start[tile];
  const int count = start[tile + 1] - start[tile];
  const bool listed = count <= tg.cap;
  int org[3];  // first cell of the bucket block (tile start - margin)
  {
    const int tz = tile % tg.nt[2];
    const int ty = (tile / tg.nt[2]) % tg.nt[1];
    const int tx = tile / (tg.nt[2] * tg.nt[1]);
    org[0] = (tx * tg.t[0] - tg.margin) & (g.nx - 1);
    org[1] = (ty * tg.t[1] - tg.margin) & (g.ny - 1);
    org[2] = (tz * tg.t[2] - tg.margin) & (g.nz - 1);
  }
  int nquad;  // quad jobs (up to four particles) in this tile
  int npair;  // pair jobs (one or two particles), after the quad jobs
  // E and B of the region: kStageNodes nodes per thread and round, all
  // their loads issued before the first LDS store (one memory latency per
  // round; a node past the region loads the last node again and stores
  // nothing).  The first round's loads go out between the loads of the
  // bucket count pass's first round and their use (loads complete in
  // issue order, so the counts wait for the particles' cells only), and
  // are stored after the pass (FP64) or after the scans and the placement
  // pass (float), so that the staging latency overlaps that work.
  const T *src[6] = {gr.E[0], gr.E[1], gr.E[2], gr.B[0], gr.B[1], gr.B[2]};
  T v[kStageNodes][6];
  auto stage_load = [&](int r0) {
#pragma unroll
    for (int u = 0; u < kStageNodes; ++u) {
      const int64_t node = region_node(min(r0 + u * NT, R - 1), rg, tg, g);
#pragma unroll
      for (int q = 0; q < 6; ++q) v[u][q] = src[q][node];
    }
  };
  auto stage_store = [&](int r0) {
#pragma unroll
    for (int u = 0; u < kStageNodes; ++u) {
      const int r = r0 + u * NT;
      if (r < R) {
#pragma unroll
        for (int q = 0; q < 6; ++q) fld[q * R + r] = v[u][q];
      }
    }
  };
  // First pass over the tile's particles: bucket counts, kParts particles
  // per thread and round, their loads together.  A tile that fits one
  // round keeps its buckets in registers for the placement pass, which then
  // loads nothing.
  constexpr int kParts = sizeof(T) == 4 ? kListPartsFloat : kListParts;
  const bool one_round = count <= kParts * NT;
  const bool counted = listed && count > 0;
  int kept[kParts];
  if (listed) {
    for (int b = tid; b <= tg.nb; b += NT) tl.fill[b] = 0;
  }
  __syncthreads();
  typename L::Key key0[kParts];  // the first round's keys (a lane past the end reloads the last)
  if (counted) {
#pragma unroll
    for (int u = 0; u < kParts; ++u) key0[u] = L::load_key(p, tbase + min(tid + u * NT, count - 1));
  }
  auto later_rounds = [&] {
    for (int i0 = tid + kParts * NT; i0 < count; i0 += kParts * NT) {
      int bk[kParts];
#pragma unroll
      for (int u = 0; u < kParts; ++u)
        bk[u] = bucket_of<L>(p, tbase + min(i0 + u * NT, count - 1), g, tg, org);
#pragma unroll
      for (int u = 0; u < kParts; ++u)
        if (i0 + u * NT < count) atomicAdd(&tl.fill[bk[u]], 1);
    }
  };
  auto first_round_counts = [&] {
#pragma unroll
    for (int u = 0; u < kParts; ++u) {
      kept[u] = bucket_of_key<L>(key0[u], g, tg, org);
      if (tid + u * NT < count) atomicAdd(&tl.fill[kept[u]], 1);
    }
  };
  auto stage_rest = [&] {
    stage_store(tid);
    for (int r0 = tid + kStageNodes * NT; r0 < R; r0 += kStageNodes * NT) {
      stage_load(r0);
      stage_store(r0);
    }
  };
  if constexpr (kLateStore) {
    // The later rounds go before the staging loads: the compiler waits for
    // every outstanding load where a loop that loads ends, and the staging
    // loads then stay in flight through the scans and the placement pass.
    if (counted && !one_round) {
      later_rounds();
      if constexpr (kGather) stage_load(tid);
    } else {
      if constexpr (kGather) stage_load(tid);
    }
    if (counted) first_round_counts();
  } else {
    if constexpr (kGather) stage_load(tid);
    if (counted) {
      first_round_counts();
      later_rounds();
    }
    if constexpr (kGather) stage_rest();
  }
  if constexpr (kDeposit) {
    for (int r = tid; r < 4 * R; r += NT) acc[r] = A(0);
  }
  if (listed) {
    __syncthreads();
    // Float particles: the job table holds the first quad job of every
    // bucket, then the second ones, then the rest, then the pair jobs.
    // Neighbouring jobs then come from different cells, so that the quads
    // of a wave do not send the same LDS addresses to one atomic
    // instruction.  Per bucket of c particles (nq quad jobs), two packed
    // scans (run together) give the offsets:
    //   off: c (bits 0-14, c <= cap <= 2^14) | max(nq - 2, 0) << 15
    //   job: [nq >= 1] | [nq >= 2] << 10 | [c mod 4 in {1, 2}] << 20
    // (nb + 1 <= 1001 buckets fit 10 bits; the third and later quad jobs,
    // fewer than cap / 4, fit 12; both sums stay below 2^31).  FP64
    // particles (two waves per SIMD) measured slower with both, and keep
    // quad jobs only, each bucket's in a row: off holds c, job holds nq.
    scan_pair<NT>(
        tg.nb + 1,
        [&](int b, int &va, int &vb) {
          const int c = tl.fill[b];
          const int rem = c & 3;
          if constexpr (kSpread) {
            const int nq = (c >> 2) + (rem == 3);
            va = c | max(nq - 2, 0) << 15;
            vb = int(nq >= 1) | int(nq >= 2) << 10 | int(rem == 1 || rem == 2) << 20;
          } else {
            va = c;
            vb = (c + 3) >> 2;
          }
        },
        [&](int b, int va, int vb) {
          tl.off[b] = va;
          tl.job[b] = vb;
          tl.fill[b] = va & 0x7FFF;  // the placement pass's fill pointers
        },
        scan_tmp);
    const unsigned tot_a = unsigned(tl.off[tg.nb + 1]), tot_b = unsigned(tl.job[tg.nb + 1]);
    const int start1 = int(tot_b & 0x3FF);                       // second quad jobs
    const int start_rest = start1 + int((tot_b >> 10) & 0x3FF);  // third and later
    nquad = kSpread ? start_rest + int(tot_a >> 15) : int(tot_b);
    npair = kSpread ? int(tot_b >> 20) : 0;
    for (int i0 = tid; i0 < count; i0 += kParts * NT) {
      int bk[kParts];
#pragma unroll
      for (int u = 0; u < kParts; ++u)
        bk[u] = one_round ? kept[u]
                          : bucket_of<L>(p, tbase + min(i0 + u * NT, count - 1), g, tg, org);
#pragma unroll
      for (int u = 0; u < kParts; ++u) {
        const int i = i0 + u * NT;
        if (i < count) {
          const int b = bk[u];
          const int pos = atomicAdd(&tl.fill[b], 1);
          tl.list[pos] = static_cast<unsigned short>(i);
          const unsigned oa = unsigned(tl.off[b]);
          const int first = int(oa & 0x7FFF);
          const int c = (tl.off[b + 1] & 0x7FFF) - first;
          const int r = pos - first;
          const int full = c & ~3;
          // the first particle of a job writes its entry
          if (!kSpread) {
            if ((r & 3) == 0) tl.jobs[tl.job[b] + (r >> 2)] = pos | min(4, c - r) << 24;
          } else if ((r & 3) == 0 && r < c && (r < full || c - full == 3)) {
            const unsigned ob = unsigned(tl.job[b]);
            const int k = r >> 2;
            const int at = k == 0   ? int(ob & 0x3FF)
                           : k == 1 ? start1 + int((ob >> 10) & 0x3FF)
                                    : start_rest + int(oa >> 15) + (k - 2);
            tl.jobs[at] = pos | min(4, c - r) << 24;
          } else if (r == full) {
            tl.jobs[nquad + int(unsigned(tl.job[b]) >> 20)] = pos | (c - full) << 24;
          }
        }
      }
    }
  } else {
    nquad = (count + 3) >> 2;
    npair = 0;
  }
  if constexpr (kGather && kLateStore) stage_rest();
  __syncthreads();

  T *jdst[3] = {gr.J[0], gr.J[1], gr.J[2]};
  T *rdst[1] = {gr.rho};
  // One job of group size G: list position (or tile index) of its first
  // particle and its size n (0 .. G).  An idle lane (past the job's last
  // particle) mirrors the group's first lane: it takes the same path
  // through the group code and stores nothing.
  auto run_job = [&](auto gsize, int first, int n) {
    constexpr int G = decltype(gsize)::value;
    const int m = tid & (G - 1);
    const bool act = m < n;
    const int pos = first + (act ? m : 0);
    const int64_t k = tbase + (listed ? int(tl.list[pos]) : pos);
    typename L::State st = load_state<L>(p, k, g);
    T u[3];
    if constexpr (MODE != kModeRho) {
      u[0] = static_cast<const T *>(p.ux)[k];
      u[1] = static_cast<const T *>(p.uy)[k];
      u[2] = static_cast<const T *>(p.uz)[k];
    }
    if constexpr (kGather) {
      const CellPos<T> c0 = L::cell(st, g);
      T F[6];
      int hb[3];
      if (group_block<ORDER, T, G>(c0, rg, tg, g, hb)) {
        gather_group<ORDER, T, G>(hb, c0.o, m, tg, fld, F);
      } else {
        Support<ORDER, T> s;
        support_of<ORDER, T>(c0, rg, tg, g, s);
        gather<ORDER, T>(c0, s, tg, g, fld, gr, F);
      }
      boris(u, F, h);
    }
    if constexpr (MODE == kModeRho) {
      const T val[1] = {qw};
      deposit_at<ORDER, T, A, 1, G>(L::cell(st, g), val, act, m, rg, tg, g, acc, 3, rdst, state);
    }
    if constexpr (kMove) {
      // v - v_gal is a difference of nearly equal numbers for the drifting
      // plasma: keep v = u / gamma correctly rounded per component
      const T gamma = sqrt(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      const T v[3] = {u[0] / gamma, u[1] / gamma, u[2] / gamma};
      L::half_move(st, v, g);
      const T jv[3] = {qw * v[0], qw * v[1], qw * v[2]};
      deposit_at<ORDER, T, A, 3, G>(L::cell(st, g), jv, act, m, rg, tg, g, acc, 0, jdst, state);
      L::half_move(st, v, g);
      const T val[1] = {qw};
      deposit_at<ORDER, T, A, 1, G>(L::cell(st, g), val, act, m, rg, tg, g, acc, 3, rdst, state);
    }
    if (act) {
      if constexpr (kMove) store_state<L>(p, k, st, g);
      if constexpr (kGather) {
        static_cast<T *>(p.ux)[k] = u[0];
        static_cast<T *>(p.uy)[k] = u[1];
        static_cast<T *>(p.uz)[k] = u[2];
      }
    }
  };
  // work unit w < nquad: quad job w; w >= nquad: pair jobs 2 (w - nquad)
  // and the next (lanes 0, 1 and 2, 3 of the quad).  Quad q takes units q,
  // q + NT/4, ...; the units of a wave are consecutive, so at most one wave
  // meets both kinds.  Two loops keep the two kinds' loop-invariant values
  // from being live together.
  const int nwork = nquad + ((npair + 1) >> 1);
  int w = tid >> 2;
  for (; w < nquad; w += NT / 4) {
    int first, n;
    if (listed) {
      const int e = tl.jobs[w];
      first = e & 0xFFFFFF;
      n = e >> 24;
    } else {
      first = 4 * w;
      n = min(4, count - first);
    }
    run_job(std::integral_constant<int, 4>{}, first, n);
  }
  if constexpr (kSpread) {
    for (; w < nwork; w += NT / 4) {
      // the second pair of an odd count's last unit is idle: it mirrors
      // the first pair's job with no particle
      const int pj = 2 * (w - nquad) + ((tid >> 1) & 1);
      const int e = tl.jobs[nquad + min(pj, npair - 1)];
      run_job(std::integral_constant<int, 2>{}, e & 0xFFFFFF, pj < npair ? e >> 24 : 0);
    }
  }
  if constexpr (kDeposit) {
    __syncthreads();
    T *buf = MODE == kModeRho ? nullptr : load_const(&jp->regbuf);
    if (buf) {
      // plain stores of the whole region (zeros included) into the tile's
      // slot of the region buffer; k_region_reduce adds the slots per node
      T *__restrict__ slot = global_ptr(buf) + size_t(tile) * 4 * size_t(R);
      for (int i = tid; i < 4 * R; i += NT) slot[i] = T(acc[i]);
    } else {
      T *dst[4] = {gr.J[0], gr.J[1], gr.J[2], gr.rho};
      const int q_first = MODE == kModeRho ? 3 : 0;
      for (int r = tid; r < R; r += NT) {
        const int64_t node = region_node(r, rg, tg, g);
        for (int q = q_first; q < 4; ++q) {
          const T vq = T(acc[q * R + r]);
          if (vq != T(0)) unsafeAtomicAdd(dst[q] + node, vq);
        }
      }
    }
  }
}

// ---- region buffer reduction --------------------------------------------------
// Tile t's region starts at node t * t_a + FIRST - margin along axis a and
// spans e_a nodes (periodic; a node appears twice when e_a exceeds the grid).
// The (tile, region index) pairs that hold node i along one axis: at most
// kPairs (e_a <= 8 + 3 + 2 and t_a >= 1 give at most 13 on a grid of 8).
constexpr int kPairs = 16;

__device__ __forceinline__ int axis_pairs(int i, int n, int ta, int nt, int e, int off,
                                          int *tiles, int *locs) {
  int cnt = 0;
  auto add = [&](int t) {
    int l = (i - (t * ta + off)) % n;
    if (l < 0) l += n;
    for (; l < e && cnt < kPairs; l += n) {
      tiles[cnt] = t;
      locs[cnt] = l;
      ++cnt;
    }
  };
  const int span = (e + ta - 1) / ta;  // candidate tiles below the one holding i - off
  if (nt <= span + 1) {
    for (int t = 0; t < nt; ++t) add(t);
  } else {
    int t0 = (i - off) >= 0 ? (i - off) / ta : -((ta - 1 - (i - off)) / ta);
    for (int k = 0; k <= span; ++k) add(((t0 - k) % nt + nt) % nt);
  }
  return cnt;
}

// Workgroup row blockIdx.y = run; grid-stride over its nodes.  Adds to J and
// rho (zeroed before the pass, holding the global-path contributions).
template <typename T, int ORDER>
__global__ __launch_bounds__(256) void k_region_reduce(const PartJob<T> *__restrict__ jobs) {
  using CJob = __attribute__((address_space(4))) const PartJob<T>;
  const PartJob<T> *jp = jobs + blockIdx.y;
  T *raw = load_const(&jp->regbuf);
  if (!raw) return;
  const T *__restrict__ buf = global_ptr(raw);
  const RunGeom g = load_const(&jp->g);
  const TileGeom tg = load_const(&jp->tg);
  GridPtrs<T> gr = load_const(&jp->gr);
  globalize(gr);
  (void)sizeof(CJob);
  const int off = Shape<ORDER, T>::FIRST - tg.margin;
  const size_t R = size_t(tg.region);
  const int n[3] = {g.nx, g.ny, g.nz};
  // usual geometry (regions at most two tiles long, three or more tiles per
  // axis): each axis gives the tile holding i - off and, if the region
  // reaches that far, the one before it
  bool two = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) two = two && tg.e[a] <= 2 * tg.t[a] && tg.nt[a] >= 3;
  if (two) {
    // one workgroup per tile (numbered XCD-contiguously, so that tiles that
    // are neighbours along z share an L2): the nodes of the tile's own
    // block, each the sum of the slots of the tile and of the tiles before
    // it whose regions reach the node
    const unsigned tile = xcd_contiguous(blockIdx.x, gridDim.x);
    if (tile >= unsigned(tg.n_tiles)) return;
    const int tt[3] = {int(tile) / (tg.nt[2] * tg.nt[1]), (int(tile) / tg.nt[2]) % tg.nt[1],
                       int(tile) % tg.nt[2]};
    for (int w = threadIdx.x; w < (1 << tg.lcpt); w += blockDim.x) {
      const int l0[3] = {w >> (tg.lt[2] + tg.lt[1]), (w >> tg.lt[2]) & (tg.t[1] - 1),
                         w & (tg.t[2] - 1)};
      int i[3], t1[3];
      bool has1[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        i[a] = (tt[a] * tg.t[a] + off + l0[a] + n[a]) & (n[a] - 1);
        t1[a] = tt[a] == 0 ? tg.nt[a] - 1 : tt[a] - 1;
        has1[a] = l0[a] + tg.t[a] < tg.e[a];
      }
      const int64_t c = (int64_t(i[0]) * g.ny + i[1]) * g.nz + i[2];
      // all eight (tile, index) combinations load unconditionally, so that
      // their 32 loads are in flight together: one whose second tile along
      // some axis does not reach the node reads the first tile's slot again
      // and adds nothing
      T v[8][4];
      bool use[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool sx = (k >> 2) && has1[0], sy = ((k >> 1) & 1) && has1[1],
                   sz = (k & 1) && has1[2];
        use[k] = ((k >> 2) == int(sx)) && (((k >> 1) & 1) == int(sy)) && ((k & 1) == int(sz));
        const int txy = (sx ? t1[0] : tt[0]) * tg.nt[1] + (sy ? t1[1] : tt[1]);
        const int lxy = (l0[0] + (sx ? tg.t[0] : 0)) * tg.sx + (l0[1] + (sy ? tg.t[1] : 0)) * tg.e[2];
        const size_t tl = size_t(txy) * tg.nt[2] + (sz ? t1[2] : tt[2]);
        const size_t base = tl * 4 * R + size_t(lxy) + l0[2] + (sz ? tg.t[2] : 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[k][q] = buf[base + q * R];
      }
      // the grids' own values (global-path deposits), all read before the
      // first store so that the reads need not wait for it
      const T old[4] = {gr.J[0][c], gr.J[1][c], gr.J[2][c], gr.rho[c]};
      T sum[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) sum[q] += use[k] ? v[k][q] : T(0);
      gr.J[0][c] = old[0] + sum[0];
      gr.J[1][c] = old[1] + sum[1];
      gr.J[2][c] = old[2] + sum[2];
      gr.rho[c] = old[3] + sum[3];
    }
    return;
  }
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < g.ncell;
       c += int64_t(gridDim.x) * blockDim.x) {
    const int i[3] = {int(c >> (g.lz + g.ly)), int((c >> g.lz) & (g.ny - 1)),
                      int(c & (g.nz - 1))};
    int tl[3][kPairs], ll[3][kPairs], cnt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      cnt[a] = axis_pairs(i[a], n[a], tg.t[a], tg.nt[a], tg.e[a], off, tl[a], ll[a]);
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    for (int x = 0; x < cnt[0]; ++x)
      for (int y = 0; y < cnt[1]; ++y) {
        const int txy = tl[0][x] * tg.nt[1] + tl[1][y];
        const int lxy = ll[0][x] * tg.sx + ll[1][y] * tg.e[2];
        for (int z = 0; z < cnt[2]; ++z) {
          const size_t tile = size_t(txy) * tg.nt[2] + tl[2][z];
          const size_t base = tile * 4 * R + size_t(lxy) + ll[2][z];
          s0 += buf[base];
          s1 += buf[base + R];
          s2 += buf[base + 2 * R];
          s3 += buf[base + 3 * R];
        }
      }
    gr.J[0][c] += s0;
    gr.J[1][c] += s1;
    gr.J[2][c] += s2;
    gr.rho[c] += s3;
  }
}

// ---- tile sort (run only when flagged) --------------------------------------
// A counting sort by tile-major cell index: the particles of a tile end up
// grouped by cell, in tile order.  Per run, state[0]: particles that used
// the global path since the last decision; state[1]: sort flag of this
// step; state[2]: sorts done; state[3]: force flag (set by the host at
// binding).  Every kernel covers all runs of the table: workgroup row
// blockIdx.y (or the workgroup, for the per-tile and per-run kernels) picks
// the run, and a run whose flag is off returns at once.
template <typename T>
__global__ void k_sort_decide(const PartJob<T> *__restrict__ jobs, int njobs) {
  for (int j = threadIdx.x; j < njobs; j += blockDim.x) {
    int *state = global_ptr(jobs[j].sb.state);
    const int threshold = jobs[j].resort_threshold;
    const int need = (state[3] != 0 || state[0] > threshold) ? 1 : 0;
    state[1] = need;
    state[0] = 0;
    state[3] = 0;
    if (need) state[2] += 1;
  }
}

template <typename T>
__global__ void k_sort_clear(const PartJob<T> *__restrict__ jobs) {
  PartJob<T> job = jobs[blockIdx.y];
  globalize(job.p);
  globalize(job.sb);
  if (!job.sb.state[1]) return;
  const int64_t n = int64_t(job.tg.n_tiles) << job.tg.lcpt;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    job.sb.cell_count[i] = 0;
}

// tile-major cell index: tile * cells_per_tile + (x, y, z) inside the tile
__device__ __forceinline__ int tile_major_cell(const int i[3], const TileGeom &tg) {
  const int tile = ((i[0] >> tg.lt[0]) * tg.nt[1] + (i[1] >> tg.lt[1])) * tg.nt[2] +
                   (i[2] >> tg.lt[2]);
  const int local = (((i[0] & (tg.t[0] - 1)) << tg.lt[1] | (i[1] & (tg.t[1] - 1))) << tg.lt[2]) |
                    (i[2] & (tg.t[2] - 1));
  return (tile << tg.lcpt) | local;
}

template <class L>
__global__ void k_sort_count(const PartJob<typename L::T> *__restrict__ jobs) {
  PartJob<typename L::T> job = jobs[blockIdx.y];
  globalize(job.p);
  globalize(job.sb);
  if (!job.sb.state[1]) return;
  // A wave takes 64 consecutive particles per round (the round's start is
  // the same for all its lanes, so the loop and the shuffles stay
  // wave-uniform).  The particles are mostly in cell order already, so a
  // run of lanes with one cell takes its ranks with one atomic on the
  // cell's counter, made by the run's first lane, instead of one atomic per
  // particle on a contended counter.
  const int lane = int(threadIdx.x) & 63;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k0 = int64_t(blockIdx.x) * blockDim.x + (int(threadIdx.x) & ~63); k0 < job.p.n;
       k0 += stride) {
    const int64_t k = k0 + lane;
    const bool in = k < job.p.n;  // the lanes past the end are a suffix of the wave
    int cell = -1;
    if (in) {
      const typename L::State st = load_state<L>(job.p, k, job.g);
      const auto c = L::cell(st, job.g);
      cell = tile_major_cell(c.i, job.tg);
    }
    const int prev = __shfl_up(cell, 1, 64);
    const bool head = in && (lane == 0 || prev != cell);
    const uint64_t heads = __ballot(head);
    const uint64_t ends = heads | ~__ballot(in);  // a run ends where another starts or at the end
    const uint64_t upto = (2ull << lane) - 1;     // lanes 0 .. lane (all ones for lane 63)
    int base = 0;
    if (head) {
      const uint64_t later = ends & ~upto;
      const int next = later ? __builtin_ctzll(later) : 64;
      base = atomicAdd(job.sb.cell_count + cell, next - lane);
    }
    const int first = in ? 63 - __builtin_clzll(heads & upto) : lane;
    base = __shfl(base, first, 64);
    if (in) {
      job.sb.key[k] = cell;
      job.sb.rank[k] = base + (lane - first);
    }
  }
}

// Inclusive scan of v over the workgroup (blockDim.x <= 1024) in LDS.
__device__ __forceinline__ int block_scan_incl(int v, int *buf) {
  const int tid = threadIdx.x;
  buf[tid] = v;
  __syncthreads();
  for (int off = 1; off < int(blockDim.x); off <<= 1) {
    const int add = tid >= off ? buf[tid - off] : 0;
    __syncthreads();
    buf[tid] += add;
    __syncthreads();
  }
  const int r = buf[tid];
  __syncthreads();
  return r;
}

// Per tile (workgroups of kNT >= cells per tile threads; row blockIdx.y
// is the run, each workgroup takes tiles blockIdx.x, + gridDim.x, ...):
// offsets of its cells inside the tile and the tile total.
template <typename T>
__global__ __launch_bounds__(kNT) void k_sort_tile_scan(const PartJob<T> *__restrict__ jobs) {
  __shared__ int buf[kNT];
  PartJob<T> job = jobs[blockIdx.y];
  globalize(job.sb);
  if (!job.sb.state[1]) return;
  const int tid = threadIdx.x;
  const int cpt = 1 << job.tg.lcpt;
  for (int tile = blockIdx.x; tile < job.tg.n_tiles; tile += gridDim.x) {
    const int v = tid < cpt ? job.sb.cell_count[(tile << job.tg.lcpt) + tid] : 0;
    const int incl = block_scan_incl(v, buf);
    if (tid < cpt) job.sb.cell_off[(tile << job.tg.lcpt) + tid] = incl - v;
    if (tid == kNT - 1) job.sb.tile_total[tile] = incl;
  }
}

// Per run (one workgroup each): exclusive scan of the tile totals into
// start[0 .. n_tiles].
template <typename T>
__global__ __launch_bounds__(1024) void k_sort_scan(const PartJob<T> *__restrict__ jobs) {
  __shared__ int part[1024];
  PartJob<T> job = jobs[blockIdx.x];
  globalize(job.sb);
  if (!job.sb.state[1]) return;
  const int n = job.tg.n_tiles;
  const int *total = job.sb.tile_total;
  int *start = job.sb.start;
  const int tid = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = tid * chunk;
  const int hi = min(n, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += total[i];
  const int incl = block_scan_incl(s, part);
  int run = incl - s;
  for (int i = lo; i < hi; ++i) {
    start[i] = run;
    run += total[i];
  }
  if (tid == 1023) start[n] = incl;
}

struct Columns {
  void *a[8];   // particle arrays
  void *b[8];   // scratch arrays of the same element size
  int size[8];  // 4 or 8 bytes
  int n;
};

// The particle arrays of a run and their scratch columns (same order as
// the host allocates the scratch: positions, momenta, then ids).
template <typename T>
__device__ __forceinline__ Columns columns_of(const PartJob<T> &job) {
  Columns c{};
  int n = 0;
  auto add = [&](void *a, int size) {
    c.a[n] = a;
    c.b[n] = job.sb.tmp[n];
    c.size[n] = size;
    ++n;
  };
  if constexpr (sizeof(T) == 8) {
    add(job.p.x, 8);
    add(job.p.y, 8);
    add(job.p.z, 8);
  } else {
    add(job.p.x, 4);
    add(job.p.ox, 4);
    add(job.p.oy, 4);
    add(job.p.oz, 4);
  }
  add(job.p.ux, int(sizeof(T)));
  add(job.p.uy, int(sizeof(T)));
  add(job.p.uz, int(sizeof(T)));
  if (job.p.id) add(job.p.id, 8);
  c.n = n;
  return c;
}

// All loads before the stores, over the fixed maximum of 8 columns: with
// constant indices the column pointers stay in registers (a loop over the
// run-time count indexed the table in scratch memory, and waited for each
// load in turn).
__device__ __forceinline__ void copy_columns(const Columns &cols, bool to_scratch, int64_t src,
                                             int64_t dst) {
  int64_t v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (c < cols.n) {
      const void *from = global_ptr(to_scratch ? cols.a[c] : cols.b[c]);
      v[c] = cols.size[c] == 8 ? static_cast<const int64_t *>(from)[src]
                               : int64_t(static_cast<const int *>(from)[src]);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (c < cols.n) {
      void *to = global_ptr(to_scratch ? cols.b[c] : cols.a[c]);
      if (cols.size[c] == 8)
        static_cast<int64_t *>(to)[dst] = v[c];
      else
        static_cast<int *>(to)[dst] = int(v[c]);
    }
  }
}

// particle k -> scratch position start[tile] + cell_off[cell] + rank
template <typename T>
__global__ void k_sort_scatter(const PartJob<T> *__restrict__ jobs) {
  PartJob<T> job = jobs[blockIdx.y];
  globalize(job.p);
  globalize(job.sb);
  if (!job.sb.state[1]) return;
  const Columns cols = columns_of(job);
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < job.p.n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const int cell = job.sb.key[k];
    const int64_t pos =
        int64_t(job.sb.start[cell >> job.tg.lcpt]) + job.sb.cell_off[cell] + job.sb.rank[k];
    copy_columns(cols, true, k, pos);
  }
}

// scratch -> particle arrays (same, cell-grouped order)
template <typename T>
__global__ void k_sort_copyback(const PartJob<T> *__restrict__ jobs) {
  PartJob<T> job = jobs[blockIdx.y];
  globalize(job.p);
  globalize(job.sb);
  if (!job.sb.state[1]) return;
  const Columns cols = columns_of(job);
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < job.p.n;
       k += int64_t(gridDim.x) * blockDim.x)
    copy_columns(cols, false, k, k);
}

unsigned stride_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return unsigned(b);
}

template <class L, int ORDER, int MODE, typename A, bool FIX>
void launch_tile_kernel(const PartJob<typename L::T> *jobs, const PartBatch &b, double dt_factor,
                        hipStream_t s) {
  using T = typename L::T;
  constexpr int NT = quad_threads(sizeof(T));
  static bool attr_set = false;  // allow dynamic LDS above 64 KiB (gfx950: 160 KiB)
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_quad<L, ORDER, MODE, A, NT, FIX>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(kLdsBytes - scan_bytes(sizeof(T))));
    attr_set = true;
  }
  hipLaunchKernelGGL((k_quad<L, ORDER, MODE, A, NT, FIX>), dim3(unsigned(b.nblocks)), dim3(NT),
                     b.lds[MODE], s, jobs, b.njobs, dt_factor);
}

template <class L, int MODE, typename A>
void launch_tile_order(int order, const PartJob<typename L::T> *jobs, const PartBatch &b,
                       double dt_factor, hipStream_t s) {
  if (order == 1)
    launch_tile_kernel<L, 1, MODE, A, false>(jobs, b, dt_factor, s);
  else if (b.fixed_geom)
    launch_tile_kernel<L, 3, MODE, A, true>(jobs, b, dt_factor, s);
  else
    launch_tile_kernel<L, 3, MODE, A, false>(jobs, b, dt_factor, s);
}

template <typename T>
struct LayoutOf;
template <>
struct LayoutOf<double> {
  using type = LayoutAbs;
  using acc = double;
};
template <>
struct LayoutOf<float> {
  using type = LayoutCell;
  using acc = double;  // float contributions, double tile sums
};

}  // namespace

TileGeom make_tile_geom(const RunGeom &g, size_t real_size, const int tile[3]) {
  TileGeom tg{};
  const int n[3] = {g.nx, g.ny, g.nz};
  const int halo = g.order == 3 ? 3 : 1;  // shape width - 1
  int lcpt = 0;
  for (int a = 0; a < 3; ++a) {
    int t = tile && tile[a] > 0 ? tile[a] : 8;
    while (t > n[a]) t >>= 1;
    tg.t[a] = t;
    int l = 0;
    while ((1 << l) < t) ++l;
    tg.lt[a] = l;
    lcpt += l;
    tg.nt[a] = n[a] / t;
  }
  tg.lcpt = lcpt;
  tg.n_tiles = tg.nt[0] * tg.nt[1] * tg.nt[2];
  // LDS of the fused pass for a margin: 6 fields and 4 double accumulators
  // per region node, the static scan buffer, the bucket tables and lists
  // (3 bytes per particle)
  auto fixed = [&](int margin, TileGeom &t) {
    t.margin = margin;
    t.nb = 1;
    for (int a = 0; a < 3; ++a) {
      t.e[a] = t.t[a] + halo + 2 * margin;
      t.ce[a] = t.t[a] + 2 * margin;
      t.nb *= t.ce[a];
    }
    // x planes padded to 4 mod 8 slots: the quads' four lanes sit one x
    // plane apart, and with 169 slots per plane (13 x 13) their 64-bit LDS
    // atomics met in the same banks (measured: 16.5 against 10.8 cycles
    // per wave instruction with eight waves, 172 slots)
    const int plane = t.e[1] * t.e[2];
    t.sx = plane + ((12 - plane % 8) % 8);
    t.region = t.e[0] * t.sx;
    return size_t(t.region) * (6 * real_size + 4 * sizeof(double)) + scan_bytes(real_size);
  };
  // one cell of drift margin when the lists still hold 4096 particles
  size_t used = fixed(1, tg);
  if (used + list_bytes(tg.nb, 4096) > kLdsBytes) used = fixed(0, tg);
  int cap = 16384;
  while (used + list_bytes(tg.nb, cap) > kLdsBytes) cap -= 64;
  tg.cap = cap;
  return tg;
}

bool default_cubic_tiles(const TileGeom &tg, size_t real_size) {
  return real_size == sizeof(float) ? DefaultCubicTiles<float>::matches(tg)
                                    : DefaultCubicTiles<double>::matches(tg);
}

template <typename T>
void launch_sort(const PartJob<T> *jobs, const PartBatch &b, hipStream_t s) {
  using L = typename LayoutOf<T>::type;
  if (b.njobs <= 0) return;
  const unsigned nj = unsigned(b.njobs);
  // most steps sort nothing and every workgroup returns at once: keep the
  // grids near 4096 workgroups in all, however many runs
  const unsigned per_run = std::max(16u, 4096u / nj);
  const unsigned pblocks = std::min(stride_blocks(b.max_n), per_run);
  const unsigned cblocks = std::min(stride_blocks(b.max_cells), per_run);
  const unsigned tblocks = unsigned(std::min<int64_t>(b.max_tiles, per_run));
  hipLaunchKernelGGL((k_sort_decide<T>), dim3(1), dim3(256), 0, s, jobs, b.njobs);
  hipLaunchKernelGGL((k_sort_clear<T>), dim3(cblocks, nj), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL((k_sort_count<L>), dim3(pblocks, nj), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL((k_sort_tile_scan<T>), dim3(tblocks, nj), dim3(kNT), 0, s, jobs);
  hipLaunchKernelGGL((k_sort_scan<T>), dim3(nj), dim3(1024), 0, s, jobs);
  hipLaunchKernelGGL((k_sort_scatter<T>), dim3(pblocks, nj), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL((k_sort_copyback<T>), dim3(pblocks, nj), dim3(256), 0, s, jobs);
}

template <typename T>
void launch_particles(int mode, const PartJob<T> *jobs, const PartBatch &b, double dt_factor,
                      hipStream_t s) {
  using L = typename LayoutOf<T>::type;
  using A = typename LayoutOf<T>::acc;
  if (b.njobs <= 0) return;
  const int order = b.order;
  switch (mode) {
    case kPartRho: launch_tile_order<L, kModeRho, A>(order, jobs, b, dt_factor, s); break;
    case kPartDeposit: launch_tile_order<L, kModeDeposit, A>(order, jobs, b, dt_factor, s); break;
    case kPartFused: launch_tile_order<L, kModeFused, A>(order, jobs, b, dt_factor, s); break;
    case kPartPush: launch_tile_order<L, kModePush, A>(order, jobs, b, dt_factor, s); break;
    default: break;
  }
}

template <typename T>
void launch_region_reduce(const PartJob<T> *jobs, const PartBatch &b, hipStream_t s) {
  if (b.njobs <= 0 || !b.any_regbuf) return;
  // one workgroup per tile on the usual geometry; the general path strides
  // over the nodes with the same grid
  const unsigned blocks = unsigned(std::max(1, b.max_tiles));
  if (b.order == 1)
    hipLaunchKernelGGL((k_region_reduce<T, 1>), dim3(blocks, unsigned(b.njobs)), dim3(256), 0, s,
                       jobs);
  else
    hipLaunchKernelGGL((k_region_reduce<T, 3>), dim3(blocks, unsigned(b.njobs)), dim3(256), 0, s,
                       jobs);
}

template <typename T>
size_t particle_lds_bytes(int mode, const TileGeom &tg) {
  using A = typename LayoutOf<T>::acc;
  const bool gather = mode == kPartFused || mode == kPartPush;
  const bool deposit = mode != kPartPush;
  return size_t(tg.region) * ((gather ? 6 * sizeof(T) : 0) + (deposit ? 4 * sizeof(A) : 0)) +
         list_bytes(tg.nb, tg.cap);
}

static_assert(int(kPartRho) == int(kModeRho) && int(kPartDeposit) == int(kModeDeposit) &&
                  int(kPartFused) == int(kModeFused) && int(kPartPush) == int(kModePush),
              "launcher modes name the kernel modes");

template void launch_sort<float>(const PartJob<float> *, const PartBatch &, hipStream_t);
template void launch_sort<double>(const PartJob<double> *, const PartBatch &, hipStream_t);
template void launch_particles<float>(int, const PartJob<float> *, const PartBatch &, double,
                                      hipStream_t);
template void launch_particles<double>(int, const PartJob<double> *, const PartBatch &, double,
                                       hipStream_t);
template void launch_region_reduce<float>(const PartJob<float> *, const PartBatch &, hipStream_t);
template void launch_region_reduce<double>(const PartJob<double> *, const PartBatch &,
                                           hipStream_t);
template size_t particle_lds_bytes<float>(int, const TileGeom &);
template size_t particle_lds_bytes<double>(int, const TileGeom &);

}  // namespace galpic
