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
// GPU design.  Particles are kept sorted by tile (8x8x8 cells) and, inside a
// tile, in slot-major order: first the first particle of every occupied
// cell (cells in tile order), then the second particle of every cell with
// two or more, and so on.  One 512-thread workgroup owns one tile; thread t
// takes the tile's particles t, t + 512, ...  The loads are coalesced and
// the lanes of a wave sit in different, neighbouring cells, so their LDS
// atomics neither collide nor pile onto one bank.  The workgroup stages the
// tile's node region (the tile plus the shape's halo) of E and B in LDS for
// the gather, accumulates J and rho of its particles in LDS, and adds the
// region into the global grid once at the end.  In mixed precision the
// per-tile sums are carried in double (no-return LDS atomics), so the only
// float roundings of a deposited value are the per-particle contribution and
// the final conversion: the tile sum itself is compensated.  A particle
// whose shape support leaves its tile's region (it drifted since the last
// sort) uses global memory directly and is counted; the next step re-sorts
// when that count passes n/64.
//
// Position layouts: FP64 stores absolute doubles in [0, L); the mixed form
// stores an int32 linear cell index and float offsets in [0, 1), so that a
// particle static on the Galilean grid keeps its position exactly.
#include "kernels.hpp"

namespace galpic {
namespace {

constexpr int kNT = 512;  // threads per tile workgroup

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

__device__ __forceinline__ int tile_of_block(const TileGeom &tg) {
  // XCD-aware: consecutive workgroups go to different XCDs round-robin;
  // give each XCD a contiguous run of tiles so neighbours share its L2.
  const int b = blockIdx.x;
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
// region (type A: float, or double for compensated float sums) or, outside
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
        const int row = ((s.base[0] + a) * tg.e[1] + (s.base[1] + b)) * tg.e[2] + s.base[2];
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
        const int row = ((s.base[0] + a) * tg.e[1] + (s.base[1] + b)) * tg.e[2] + s.base[2];
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

// region slot -> global node index
__device__ __forceinline__ int64_t region_node(int r, const Region &rg, const TileGeom &tg,
                                               const RunGeom &g) {
  const int az = r % tg.e[2];
  const int ay = (r / tg.e[2]) % tg.e[1];
  const int ax = r / (tg.e[2] * tg.e[1]);
  const int ix = (rg.org[0] + ax) & (g.nx - 1);
  const int iy = (rg.org[1] + ay) & (g.ny - 1);
  const int iz = (rg.org[2] + az) & (g.nz - 1);
  return (int64_t(ix) * g.ny + iy) * g.nz + iz;
}

enum { kModeRho = 0, kModeDeposit = 1, kModeFused = 2, kModePush = 3 };

// Deposit batches.  Thread t of a tile's workgroup takes the tile's
// particles t, t + kNT, ... in batches of K.  In slot-major order those
// started out in one cell (tile cell t) and, in a cold or slowly drifting
// plasma, move together, so they usually still share one cell: the batch
// members in the cell of the batch's first particle share that cell's
// 4x4x4 (or 2x2x2) node block, and their J and rho contributions to a node
// are summed in registers before a single LDS atomic per node and quantity.
// The others are deposited on their own.
// Weight of node a (0 .. N-1, i.e. cell + FIRST + a) for offset d, for a
// runtime a: the B-spline of the distance r = |d - FIRST - a|.
template <int ORDER, typename T>
__device__ __forceinline__ T weight_at(int a, T d) {
  if constexpr (ORDER == 1) {
    return a == 0 ? T(1) - d : d;
  } else {
    const T r = fabs(d + T(1) - T(a));
    const T r2 = r * r;
    const T s = T(2) - r;
    return r < T(1) ? T(2.0 / 3.0) - r2 + T(0.5) * r2 * r : s * s * s * T(1.0 / 6.0);
  }
}

// deposit of NQ values per batch member flagged `in` into the block of
// nodes whose first node is hb (region-local)
template <int ORDER, typename T, typename A, int K, int NQ>
__device__ __forceinline__ void deposit_home(const int hb[3], const TileGeom &tg, A *acc,
                                             int q0, const bool in[K], const T ox[K],
                                             const T wy[K][Shape<ORDER, T>::N],
                                             const T wz[K][Shape<ORDER, T>::N],
                                             const T val[K][NQ]) {
  constexpr int N = Shape<ORDER, T>::N;
  const int R = tg.region;
#pragma unroll 1
  for (int a = 0; a < N; ++a) {
    T wxa[K];
#pragma unroll
    for (int j = 0; j < K; ++j) wxa[j] = in[j] ? weight_at<ORDER, T>(a, ox[j]) : T(0);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int row = ((hb[0] + a) * tg.e[1] + (hb[1] + b)) * tg.e[2] + hb[2];
#pragma unroll
      for (int e = 0; e < N; ++e) {
        T sum[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) sum[q] = T(0);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const T wj = wxa[j] * wy[j][b] * wz[j][e];
#pragma unroll
          for (int q = 0; q < NQ; ++q) sum[q] += wj * val[j][q];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          __hip_atomic_fetch_add(acc + size_t(q0 + q) * R + row + e, A(sum[q]), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int ORDER, typename T>
__device__ __forceinline__ bool same_cell(const CellPos<T> &c, const int cell[3]) {
  return c.i[0] == cell[0] && c.i[1] == cell[1] && c.i[2] == cell[2];
}

// Everything the tile kernel needs besides the particle index.
template <class L>
struct TileCtx {
  using T = typename L::T;
  RunGeom g;
  TileGeom tg;
  PartPtrs p;
  GridPtrs<T> gr;
  Region rg;
  T qw, h;
  int *fallback;
};

// Gather E, B at particle k's current position (LDS region or global) and
// push its momentum through the step h was built for.
template <class L, int ORDER>
__device__ __forceinline__ void push_one(const TileCtx<L> &tc, int64_t k,
                                         const typename L::T *fld) {
  using T = typename L::T;
  const typename L::State st = load_state<L>(tc.p, k, tc.g);
  T u[3] = {static_cast<const T *>(tc.p.ux)[k], static_cast<const T *>(tc.p.uy)[k],
            static_cast<const T *>(tc.p.uz)[k]};
  const CellPos<T> c = L::cell(st, tc.g);
  Support<ORDER, T> s;
  support_of<ORDER, T>(c, tc.rg, tc.tg, tc.g, s);
  T F[6];
  gather<ORDER, T>(c, s, tc.tg, tc.g, fld, tc.gr, F);
  boris(u, F, tc.h);
  static_cast<T *>(tc.p.ux)[k] = u[0];
  static_cast<T *>(tc.p.uy)[k] = u[1];
  static_cast<T *>(tc.p.uz)[k] = u[2];
}

// Per-particle deposit of particle k from memory (position x^n, current u):
// rho at x^n (rho mode), or J at x^n + (v - v_gal) dt/2 and rho at
// x^n + (v - v_gal) dt.  The position is not written.
template <class L, int ORDER, int MODE, typename A>
__device__ void deposit_one(const TileCtx<L> &tc, int64_t k, A *acc, bool do_j, bool do_rho) {
  using T = typename L::T;
  typename L::State st = load_state<L>(tc.p, k, tc.g);
  if constexpr (MODE == kModeRho) {
    const CellPos<T> c = L::cell(st, tc.g);
    Support<ORDER, T> s;
    support_of<ORDER, T>(c, tc.rg, tc.tg, tc.g, s);
    T *dst[1] = {tc.gr.rho};
    const T val[1] = {tc.qw};
    deposit<ORDER, T, A>(c, s, tc.tg, tc.g, acc, 3, 1, val, dst, tc.fallback);
  } else {
    const T u[3] = {static_cast<const T *>(tc.p.ux)[k], static_cast<const T *>(tc.p.uy)[k],
                    static_cast<const T *>(tc.p.uz)[k]};
    const T gamma = sqrt(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const T v[3] = {u[0] / gamma, u[1] / gamma, u[2] / gamma};
    L::half_move(st, v, tc.g);
    if (do_j) {
      const CellPos<T> c = L::cell(st, tc.g);
      Support<ORDER, T> s;
      support_of<ORDER, T>(c, tc.rg, tc.tg, tc.g, s);
      T *dst[3] = {tc.gr.J[0], tc.gr.J[1], tc.gr.J[2]};
      const T val[3] = {tc.qw * v[0], tc.qw * v[1], tc.qw * v[2]};
      deposit<ORDER, T, A>(c, s, tc.tg, tc.g, acc, 0, 3, val, dst, tc.fallback);
    }
    L::half_move(st, v, tc.g);
    if (do_rho) {
      const CellPos<T> c = L::cell(st, tc.g);
      Support<ORDER, T> s;
      support_of<ORDER, T>(c, tc.rg, tc.tg, tc.g, s);
      T *dst[1] = {tc.gr.rho};
      const T val[1] = {tc.qw};
      deposit<ORDER, T, A>(c, s, tc.tg, tc.g, acc, 3, 1, val, dst, tc.fallback);
    }
  }
}

// One workgroup per tile.  Modes:
//  rho:     rho at the current positions (no move)
//  deposit: move dt/2, J; move dt/2, rho; positions written
//  fused:   gather at the current positions and push u through dt, then as
//           deposit with the new u (one particle pass per step)
//  push:    gather and push u through the time step h was built for
//
// Gather + push run with four lanes per cell: in slot-major order lanes
// 4c .. 4c+3 of a quad take the particles of one cell from four rounds, so
// the quad reads the same LDS node values and the LDS broadcasts them.  The
// deposit runs with one thread per cell and batches of K of its particles
// (see deposit_home); a particle whose half-way or end position is outside
// the thread's home cell is deposited on its own.
template <class L, int ORDER, int MODE, typename A, int K>
__global__ __launch_bounds__(kNT) void k_tile(RunGeom g, TileGeom tg, PartPtrs p,
                                              GridPtrs<typename L::T> gr,
                                              const int *__restrict__ start, int *state,
                                              typename L::T h) {
  using T = typename L::T;
  using Sh = Shape<ORDER, T>;
  constexpr int N = Sh::N;
  constexpr bool kGather = MODE == kModeFused || MODE == kModePush;
  constexpr bool kDeposit = MODE != kModePush;
  extern __shared__ __align__(16) unsigned char smem[];
  // accumulators first (8-byte aligned when A is double), then the fields
  A *acc = reinterpret_cast<A *>(smem);                                  // 4 * region
  T *fld = reinterpret_cast<T *>(smem + (kDeposit ? 4 * sizeof(A) * tg.region : 0));
  const int tile = tile_of_block(tg);
  TileCtx<L> tc;
  tc.g = g;
  tc.tg = tg;
  tc.p = p;
  tc.gr = gr;
  tc.rg = region_of(tile, tg, g, Sh::FIRST);
  tc.qw = T(p.q * p.w / (g.dx * g.dy * g.dz));
  tc.h = h;
  tc.fallback = state;
  const int R = tg.region;
  const int tid = threadIdx.x;
  if constexpr (kGather) {
    const T *src[6] = {gr.E[0], gr.E[1], gr.E[2], gr.B[0], gr.B[1], gr.B[2]};
    for (int r = tid; r < R; r += kNT) {
      const int64_t node = region_node(r, tc.rg, tg, g);
#pragma unroll
      for (int q = 0; q < 6; ++q) fld[q * R + r] = src[q][node];
    }
  }
  if constexpr (kDeposit) {
    for (int r = tid; r < 4 * R; r += kNT) acc[r] = A(0);
  }
  __syncthreads();
  const int b0 = start[tile];
  const int count = start[tile + 1] - b0;
  if constexpr (kGather) {
    // quads: lane (cell slot c, member m) of chunk q takes local index
    // q * 4 kNT + m * kNT + c (rounds 4q + m of cell slot c)
    const int cslot = tid >> 2;
    const int m = tid & 3;
    for (int chunk = 0; chunk * 4 * kNT < count; ++chunk) {
#pragma unroll 1
      for (int cb = 0; cb < 4; ++cb) {
        const int local = chunk * 4 * kNT + m * kNT + cb * (kNT / 4) + cslot;
        if (local < count) push_one<L, ORDER>(tc, int64_t(b0) + local, fld);
      }
    }
    if constexpr (kDeposit) {
      __threadfence_block();
      __syncthreads();
    }
  }
  if constexpr (kDeposit) {
    // Thread t takes the particles t, t + kNT, ... in batches of K: in
    // slot-major order these started in one cell and, moving together,
    // usually still share one.  The batch cell is the cell of the batch's
    // first particle (at the half-way position for J, at the end position
    // for rho); members in it share the node block, others are deposited
    // on their own.
    for (int r0 = 0; tid + kNT * r0 < count; r0 += K) {
      typename L::State st[K], sh[K];
      int64_t idx[K];
      T v[K][3];
      unsigned valid = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int local = tid + kNT * (r0 + j);
        if (local < count) valid |= 1u << j;
        idx[j] = int64_t(b0) + (local < count ? local : 0);
        st[j] = load_state<L>(p, idx[j], g);
        if constexpr (MODE == kModeRho) {
          sh[j] = st[j];
        } else {
          const T u[3] = {static_cast<const T *>(p.ux)[idx[j]],
                          static_cast<const T *>(p.uy)[idx[j]],
                          static_cast<const T *>(p.uz)[idx[j]]};
          const T gamma = sqrt(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
          v[j][0] = u[0] / gamma;
          v[j][1] = u[1] / gamma;
          v[j][2] = u[2] / gamma;
          L::half_move(st[j], v[j], g);
          sh[j] = st[j];
          L::half_move(st[j], v[j], g);
        }
      }
      // J at the half-way positions, rho at the end positions: group the
      // batch by cell and deposit each group through its shared node block
      T ox[K], wy[K][N], wz[K][N];
      int cell_j[K][3], cell_r[K][3];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const CellPos<T> ch = L::cell(sh[j], g);
        const CellPos<T> ce = L::cell(st[j], g);
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) {
          cell_j[j][a2] = ch.i[a2];
          cell_r[j][a2] = ce.i[a2];
        }
      }
      if constexpr (MODE != kModeRho) {
        T val[K][3];
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const CellPos<T> c = L::cell(sh[j], g);
          ox[j] = c.o[0];
          Sh::weights(c.o[1], wy[j]);
          Sh::weights(c.o[2], wz[j]);
#pragma unroll
          for (int q = 0; q < 3; ++q) val[j][q] = tc.qw * v[j][q];
        }
        unsigned left = valid;
#pragma unroll 1
        while (left) {
          // the group of the lowest remaining particle
          int lead[3];
#pragma unroll
          for (int j = K - 1; j >= 0; --j)
            if ((left >> j) & 1u) {
              lead[0] = cell_j[j][0];
              lead[1] = cell_j[j][1];
              lead[2] = cell_j[j][2];
            }
          bool dep[K];
          unsigned grp = 0;
#pragma unroll
          for (int j = 0; j < K; ++j) {
            dep[j] = ((left >> j) & 1u) && cell_j[j][0] == lead[0] && cell_j[j][1] == lead[1] &&
                     cell_j[j][2] == lead[2];
            if (dep[j]) grp |= 1u << j;
          }
          left &= ~grp;
          CellPos<T> lc;
          lc.i[0] = lead[0];
          lc.i[1] = lead[1];
          lc.i[2] = lead[2];
          int hb[3];
          if (region_base<ORDER, T>(lc, tc.rg, tg, g, hb)) {
            deposit_home<ORDER, T, A, K, 3>(hb, tg, acc, 0, dep, ox, wy, wz, val);
          } else {
            // outside the tile's region: global memory, one particle at a time
#pragma unroll 1
            for (int j = 0; j < K; ++j)
              if ((grp >> j) & 1u)
                deposit_one<L, ORDER, MODE, A>(tc, int64_t(b0) + tid + kNT * (r0 + j), acc, true,
                                               false);
          }
        }
      }
      {
        T val[K][1];
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const CellPos<T> c = L::cell(st[j], g);
          ox[j] = c.o[0];
          Sh::weights(c.o[1], wy[j]);
          Sh::weights(c.o[2], wz[j]);
          val[j][0] = tc.qw;
        }
        unsigned left = valid;
#pragma unroll 1
        while (left) {
          int lead[3];
#pragma unroll
          for (int j = K - 1; j >= 0; --j)
            if ((left >> j) & 1u) {
              lead[0] = cell_r[j][0];
              lead[1] = cell_r[j][1];
              lead[2] = cell_r[j][2];
            }
          bool dep[K];
          unsigned grp = 0;
#pragma unroll
          for (int j = 0; j < K; ++j) {
            dep[j] = ((left >> j) & 1u) && cell_r[j][0] == lead[0] && cell_r[j][1] == lead[1] &&
                     cell_r[j][2] == lead[2];
            if (dep[j]) grp |= 1u << j;
          }
          left &= ~grp;
          CellPos<T> lc;
          lc.i[0] = lead[0];
          lc.i[1] = lead[1];
          lc.i[2] = lead[2];
          int hb[3];
          if (region_base<ORDER, T>(lc, tc.rg, tg, g, hb)) {
            deposit_home<ORDER, T, A, K, 1>(hb, tg, acc, 3, dep, ox, wy, wz, val);
          } else {
#pragma unroll 1
            for (int j = 0; j < K; ++j)
              if ((grp >> j) & 1u)
                deposit_one<L, ORDER, MODE, A>(tc, int64_t(b0) + tid + kNT * (r0 + j), acc, false,
                                               true);
          }
        }
      }
      if constexpr (MODE != kModeRho) {
#pragma unroll
        for (int j = 0; j < K; ++j)
          if ((valid >> j) & 1u) store_state<L>(p, idx[j], st[j], g);
      }
    }
    __syncthreads();
    T *dst[4] = {gr.J[0], gr.J[1], gr.J[2], gr.rho};
    const int q_first = MODE == kModeRho ? 3 : 0;
    for (int r = tid; r < R; r += kNT) {
      const int64_t node = region_node(r, tc.rg, tg, g);
      for (int q = q_first; q < 4; ++q) {
        const T vq = T(acc[q * R + r]);
        if (vq != T(0)) unsafeAtomicAdd(dst[q] + node, vq);
      }
    }
  }
}

// ---- tile sort (run only when flagged) --------------------------------------
// A counting sort by tile-major cell index, then a per-tile reorder into
// slot-major order.  state[0]: particles that used the global path since the
// last decision; state[1]: sort flag of this step; state[2]: sorts done;
// state[3]: force flag (set by the host at binding).
__global__ void k_sort_decide(int *state, int threshold) {
  const int need = (state[3] != 0 || state[0] > threshold) ? 1 : 0;
  state[1] = need;
  state[0] = 0;
  state[3] = 0;
  if (need) state[2] += 1;
}

__global__ void k_sort_clear(const int *state, int *cell_count, int64_t n) {
  if (!state[1]) return;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    cell_count[i] = 0;
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
__global__ void k_sort_count(RunGeom g, TileGeom tg, PartPtrs p, const int *state,
                             int *cell_count, int *key, int *rank) {
  if (!state[1]) return;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < p.n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const typename L::State st = load_state<L>(p, k, g);
    const auto c = L::cell(st, g);
    const int cell = tile_major_cell(c.i, tg);
    key[k] = cell;
    rank[k] = atomicAdd(cell_count + cell, 1);
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

// Per tile: offsets of its cells inside the tile (cell-grouped order) and
// the tile total.  One workgroup of kNT >= cells per tile threads per tile.
__global__ __launch_bounds__(kNT) void k_sort_tile_scan(TileGeom tg, const int *state,
                                                        const int *cell_count, int *cell_off,
                                                        int *tile_total) {
  if (!state[1]) return;
  __shared__ int buf[kNT];
  const int tile = blockIdx.x;
  const int tid = threadIdx.x;
  const int cpt = 1 << tg.lcpt;
  const int v = tid < cpt ? cell_count[(tile << tg.lcpt) + tid] : 0;
  const int incl = block_scan_incl(v, buf);
  if (tid < cpt) cell_off[(tile << tg.lcpt) + tid] = incl - v;
  if (tid == kNT - 1) tile_total[tile] = incl;
}

// exclusive scan of tile_total[0..n) into start[0..n] (one workgroup)
__global__ __launch_bounds__(1024) void k_sort_scan(const int *state, const int *total,
                                                    int *start, int n) {
  if (!state[1]) return;
  __shared__ int part[1024];
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

__device__ __forceinline__ void copy_columns(const Columns &cols, bool to_scratch, int64_t src,
                                             int64_t dst) {
  for (int c = 0; c < cols.n; ++c) {
    const void *from = to_scratch ? cols.a[c] : cols.b[c];
    void *to = to_scratch ? cols.b[c] : cols.a[c];
    if (cols.size[c] == 8)
      static_cast<int64_t *>(to)[dst] = static_cast<const int64_t *>(from)[src];
    else
      static_cast<int *>(to)[dst] = static_cast<const int *>(from)[src];
  }
}

// particle k -> scratch position start[tile] + cell_off[cell] + rank
__global__ void k_sort_scatter(TileGeom tg, const int *state, Columns cols, int64_t np,
                               const int *key, const int *rank, const int *cell_off,
                               const int *start) {
  if (!state[1]) return;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < np;
       k += int64_t(gridDim.x) * blockDim.x) {
    const int cell = key[k];
    const int64_t pos = int64_t(start[cell >> tg.lcpt]) + cell_off[cell] + rank[k];
    copy_columns(cols, true, k, pos);
  }
}

// Per tile: scratch (cell-grouped) -> particle arrays in slot-major order.
__global__ __launch_bounds__(kNT) void k_sort_reorder(TileGeom tg, const int *state,
                                                      Columns cols, const int *cell_count,
                                                      const int *cell_off, const int *start) {
  if (!state[1]) return;
  __shared__ int buf[kNT];
  __shared__ int maxc;
  const int tile = blockIdx.x;
  const int tid = threadIdx.x;
  const int cpt = 1 << tg.lcpt;
  const int cnt = tid < cpt ? cell_count[(tile << tg.lcpt) + tid] : 0;
  const int off = tid < cpt ? cell_off[(tile << tg.lcpt) + tid] : 0;
  if (tid == 0) maxc = 0;
  __syncthreads();
  atomicMax(&maxc, cnt);
  __syncthreads();
  const int rounds = maxc;
  const int64_t base = start[tile];
  int64_t slot_base = base;
  for (int r = 0; r < rounds; ++r) {
    const int f = cnt > r ? 1 : 0;
    const int incl = block_scan_incl(f, buf);
    if (f) copy_columns(cols, false, base + off + r, slot_base + incl - 1);
    // total of this round: the last thread's inclusive value
    if (tid == kNT - 1) buf[0] = incl;
    __syncthreads();
    slot_base += buf[0];
    __syncthreads();
  }
}

unsigned stride_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return unsigned(b);
}

template <class L, int ORDER, int MODE, typename A>
void launch_tile_kernel(const RunGeom &g, const TileGeom &tg, const PartPtrs &p,
                        const GridPtrs<typename L::T> &gr, const SortBufs &sb, double hval,
                        hipStream_t s) {
  using T = typename L::T;
  constexpr bool kGather = MODE == kModeFused || MODE == kModePush;
  constexpr bool kDeposit = MODE != kModePush;
  constexpr int kK = sizeof(T) == 8 ? 2 : 4;  // batch size (register budget)
  const size_t lds = size_t(tg.region) * ((kGather ? 6 * sizeof(T) : 0) +
                                          (kDeposit ? 4 * sizeof(A) : 0));
  static bool attr_set = false;  // allow dynamic LDS above 64 KiB (gfx950: 160 KiB)
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile<L, ORDER, MODE, A, kK>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL((k_tile<L, ORDER, MODE, A, kK>), dim3(unsigned(tg.n_tiles)), dim3(kNT), lds,
                     s, g, tg, p, gr, sb.start, sb.state, T(hval));
}

template <class L, int MODE, typename A>
void launch_tile_order(const RunGeom &g, const TileGeom &tg, const PartPtrs &p,
                       const GridPtrs<typename L::T> &gr, const SortBufs &sb, double hval,
                       hipStream_t s) {
  if (g.order == 1)
    launch_tile_kernel<L, 1, MODE, A>(g, tg, p, gr, sb, hval, s);
  else
    launch_tile_kernel<L, 3, MODE, A>(g, tg, p, gr, sb, hval, s);
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
  using acc = double;  // compensated: float contributions, double tile sums
};

}  // namespace

TileGeom make_tile_geom(const RunGeom &g, size_t real_size) {
  TileGeom tg{};
  const int n[3] = {g.nx, g.ny, g.nz};
  const int halo = g.order == 3 ? 3 : 1;  // shape width - 1
  // one cell of drift margin when the fused kernel's LDS (6 fields and 4
  // double accumulators per region node) still fits in 160 KiB
  {
    int e = 8 + halo + 2;
    const size_t bytes = size_t(e) * e * e * (6 * real_size + 4 * sizeof(double));
    tg.margin = bytes <= 160 * 1024 ? 1 : 0;
  }
  int lcpt = 0;
  for (int a = 0; a < 3; ++a) {
    int t = 8;
    while (t > n[a]) t >>= 1;
    tg.t[a] = t;
    int l = 0;
    while ((1 << l) < t) ++l;
    tg.lt[a] = l;
    lcpt += l;
    tg.nt[a] = n[a] / t;
    tg.e[a] = t + halo + 2 * tg.margin;
  }
  tg.lcpt = lcpt;
  tg.n_tiles = tg.nt[0] * tg.nt[1] * tg.nt[2];
  tg.region = tg.e[0] * tg.e[1] * tg.e[2];
  return tg;
}

template <typename T>
void launch_sort(const RunGeom &g, const TileGeom &tg, const PartPtrs &p, const SortBufs &sb,
                 hipStream_t s) {
  using L = typename LayoutOf<T>::type;
  if (p.n == 0) return;
  const int threshold = int(p.n / 64);
  const int64_t ncell = int64_t(tg.n_tiles) << tg.lcpt;
  hipLaunchKernelGGL(k_sort_decide, dim3(1), dim3(1), 0, s, sb.state, threshold);
  hipLaunchKernelGGL(k_sort_clear, dim3(stride_blocks(ncell)), dim3(256), 0, s, sb.state,
                     sb.cell_count, ncell);
  hipLaunchKernelGGL((k_sort_count<L>), dim3(stride_blocks(p.n)), dim3(256), 0, s, g, tg, p,
                     sb.state, sb.cell_count, sb.key, sb.rank);
  hipLaunchKernelGGL(k_sort_tile_scan, dim3(unsigned(tg.n_tiles)), dim3(kNT), 0, s, tg,
                     sb.state, sb.cell_count, sb.cell_off, sb.tile_total);
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, sb.state, sb.tile_total, sb.start,
                     tg.n_tiles);
  Columns cols{};
  void *arrays[8];
  int sizes[8];
  int nc = 0;
  if (sizeof(T) == 8) {
    arrays[nc] = p.x; sizes[nc++] = 8;
    arrays[nc] = p.y; sizes[nc++] = 8;
    arrays[nc] = p.z; sizes[nc++] = 8;
  } else {
    arrays[nc] = p.x; sizes[nc++] = 4;
    arrays[nc] = p.ox; sizes[nc++] = 4;
    arrays[nc] = p.oy; sizes[nc++] = 4;
    arrays[nc] = p.oz; sizes[nc++] = 4;
  }
  arrays[nc] = p.ux; sizes[nc++] = int(sizeof(T));
  arrays[nc] = p.uy; sizes[nc++] = int(sizeof(T));
  arrays[nc] = p.uz; sizes[nc++] = int(sizeof(T));
  if (p.id) {
    arrays[nc] = p.id;
    sizes[nc++] = 8;
  }
  cols.n = nc;
  for (int c = 0; c < nc; ++c) {
    cols.a[c] = arrays[c];
    cols.b[c] = sb.tmp[c];
    cols.size[c] = sizes[c];
  }
  hipLaunchKernelGGL(k_sort_scatter, dim3(stride_blocks(p.n)), dim3(256), 0, s, tg, sb.state,
                     cols, p.n, sb.key, sb.rank, sb.cell_off, sb.start);
  hipLaunchKernelGGL(k_sort_reorder, dim3(unsigned(tg.n_tiles)), dim3(kNT), 0, s, tg, sb.state,
                     cols, sb.cell_count, sb.cell_off, sb.start);
}

template <typename T>
void launch_particles(int mode, const RunGeom &g, const TileGeom &tg, const PartPtrs &p,
                      const GridPtrs<T> &gr, const SortBufs &sb, double dt_push,
                      hipStream_t s) {
  using L = typename LayoutOf<T>::type;
  using A = typename LayoutOf<T>::acc;
  if (p.n == 0) return;
  const double h = p.q * dt_push / (2.0 * p.m);
  switch (mode) {
    case kPartRho: launch_tile_order<L, kModeRho, A>(g, tg, p, gr, sb, h, s); break;
    case kPartDeposit: launch_tile_order<L, kModeDeposit, A>(g, tg, p, gr, sb, h, s); break;
    case kPartFused: launch_tile_order<L, kModeFused, A>(g, tg, p, gr, sb, h, s); break;
    case kPartPush: launch_tile_order<L, kModePush, A>(g, tg, p, gr, sb, h, s); break;
    default: break;
  }
}

template void launch_sort<float>(const RunGeom &, const TileGeom &, const PartPtrs &,
                                 const SortBufs &, hipStream_t);
template void launch_sort<double>(const RunGeom &, const TileGeom &, const PartPtrs &,
                                  const SortBufs &, hipStream_t);
template void launch_particles<float>(int, const RunGeom &, const TileGeom &, const PartPtrs &,
                                      const GridPtrs<float> &, const SortBufs &, double,
                                      hipStream_t);
template void launch_particles<double>(int, const RunGeom &, const TileGeom &,
                                       const PartPtrs &, const GridPtrs<double> &,
                                       const SortBufs &, double, hipStream_t);

}  // namespace galpic
