// Particle kernels: deposition, gather and relativistic Boris push.
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
// Position layouts: FP64 stores absolute doubles in [0, L); the mixed form
// stores an int32 linear cell index and float offsets in [0, 1), so that a
// particle static on the Galilean grid keeps its position exactly.
#include "kernels.hpp"

namespace galpic {
namespace {

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

// ---- FP64 layout: absolute positions ---------------------------------------
struct LayoutAbs {
  using T = double;
  __device__ __forceinline__ static void load(const PartPtrs &p, int64_t k, const RunGeom &g,
                                              double x[3]) {
    x[0] = static_cast<const double *>(p.x)[k];
    x[1] = static_cast<const double *>(p.y)[k];
    x[2] = static_cast<const double *>(p.z)[k];
  }
  __device__ __forceinline__ static void store(const PartPtrs &p, int64_t k, const double x[3]) {
    static_cast<double *>(p.x)[k] = x[0];
    static_cast<double *>(p.y)[k] = x[1];
    static_cast<double *>(p.z)[k] = x[2];
  }
  __device__ __forceinline__ static double wrap(double x, double L) {
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
  }
  // x += dxyz (absolute displacement), periodic
  __device__ __forceinline__ static void move(double x[3], const double d[3], const RunGeom &g) {
    x[0] = wrap(x[0] + d[0], g.nx * g.dx);
    x[1] = wrap(x[1] + d[1], g.ny * g.dy);
    x[2] = wrap(x[2] + d[2], g.nz * g.dz);
  }
  __device__ __forceinline__ static CellPos<double> cell(const double x[3], const RunGeom &g) {
    CellPos<double> c;
    const double s[3] = {x[0] / g.dx, x[1] / g.dy, x[2] / g.dz};
    const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double f = floor(s[a]);
      c.o[a] = s[a] - f;
      int i = int(f);
      if (i >= n[a]) i -= n[a];
      if (i < 0) i += n[a];
      c.i[a] = i;
    }
    return c;
  }
};

// ---- mixed layout: int32 cell + float offsets ------------------------------
struct LayoutCell {
  using T = float;
  struct Pos {
    int i[3];
    float o[3];
  };
};

__device__ __forceinline__ void decode_cell(int cell, const RunGeom &g, int i[3]) {
  i[2] = cell & (g.nz - 1);
  i[1] = (cell >> g.lz) & (g.ny - 1);
  i[0] = cell >> (g.lz + g.ly);
}
__device__ __forceinline__ int encode_cell(const int i[3], const RunGeom &g) {
  return (((i[0] << g.ly) | i[1]) << g.lz) | i[2];
}

// offset += d (in cells); carry into the cell index, periodic
__device__ __forceinline__ void move_cell(int i[3], float o[3], const float d[3],
                                          const RunGeom &g) {
  const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float x = o[a] + d[a];
    const float f = floorf(x);
    x -= f;
    int carry = int(f);
    if (x >= 1.0f) {  // rounding of a tiny negative offset up to 1
      x = 0.0f;
      carry += 1;
    }
    o[a] = x;
    i[a] = (i[a] + carry) & (n[a] - 1);
  }
}

template <typename T>
__device__ __forceinline__ void atomic_add(T *p, T v) {
  unsafeAtomicAdd(p, v);
}

template <int ORDER, typename T>
__device__ __forceinline__ void scatter(const RunGeom &g, const CellPos<T> &c, T *const *dst,
                                        const T *val, int nq) {
  using Sh = Shape<ORDER, T>;
  T wx[Sh::N], wy[Sh::N], wz[Sh::N];
  Sh::weights(c.o[0], wx);
  Sh::weights(c.o[1], wy);
  Sh::weights(c.o[2], wz);
#pragma unroll
  for (int a = 0; a < Sh::N; ++a) {
    const int ix = (c.i[0] + Sh::FIRST + a) & (g.nx - 1);
#pragma unroll
    for (int b = 0; b < Sh::N; ++b) {
      const int iy = (c.i[1] + Sh::FIRST + b) & (g.ny - 1);
      const T wab = wx[a] * wy[b];
      const int64_t row = (int64_t(ix) * g.ny + iy) * g.nz;
#pragma unroll
      for (int e = 0; e < Sh::N; ++e) {
        const int iz = (c.i[2] + Sh::FIRST + e) & (g.nz - 1);
        const T w = wab * wz[e];
        for (int q = 0; q < nq; ++q) atomic_add(dst[q] + row + iz, w * val[q]);
      }
    }
  }
}

template <int ORDER, typename T>
__device__ __forceinline__ void interpolate(const RunGeom &g, const CellPos<T> &c,
                                            const GridPtrs<T> &gr, T F[6]) {
  using Sh = Shape<ORDER, T>;
  T wx[Sh::N], wy[Sh::N], wz[Sh::N];
  Sh::weights(c.o[0], wx);
  Sh::weights(c.o[1], wy);
  Sh::weights(c.o[2], wz);
#pragma unroll
  for (int q = 0; q < 6; ++q) F[q] = T(0);
#pragma unroll
  for (int a = 0; a < Sh::N; ++a) {
    const int ix = (c.i[0] + Sh::FIRST + a) & (g.nx - 1);
#pragma unroll
    for (int b = 0; b < Sh::N; ++b) {
      const int iy = (c.i[1] + Sh::FIRST + b) & (g.ny - 1);
      const T wab = wx[a] * wy[b];
      const int64_t row = (int64_t(ix) * g.ny + iy) * g.nz;
#pragma unroll
      for (int e = 0; e < Sh::N; ++e) {
        const int iz = (c.i[2] + Sh::FIRST + e) & (g.nz - 1);
        const T w = wab * wz[e];
        const int64_t o = row + iz;
        F[0] += w * gr.E[0][o];
        F[1] += w * gr.E[1][o];
        F[2] += w * gr.E[2][o];
        F[3] += w * gr.B[0][o];
        F[4] += w * gr.B[1][o];
        F[5] += w * gr.B[2][o];
      }
    }
  }
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

template <typename T>
__device__ __forceinline__ void load_u(const PartPtrs &p, int64_t k, T u[3]) {
  u[0] = static_cast<const T *>(p.ux)[k];
  u[1] = static_cast<const T *>(p.uy)[k];
  u[2] = static_cast<const T *>(p.uz)[k];
}

// ---- FP64 kernels ----------------------------------------------------------
template <int ORDER>
__global__ __launch_bounds__(256) void k_deposit_abs(RunGeom g, PartPtrs p, GridPtrs<double> gr,
                                                     int move) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= p.n) return;
  const double qw = p.q * p.w / (g.dx * g.dy * g.dz);
  double x[3];
  LayoutAbs::load(p, k, g, x);
  if (!move) {
    double *dst[1] = {gr.rho};
    const double one[1] = {qw};
    scatter<ORDER, double>(g, LayoutAbs::cell(x, g), dst, one, 1);
    return;
  }
  double u[3];
  load_u(p, k, u);
  const double gamma = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double v[3] = {u[0] / gamma, u[1] / gamma, u[2] / gamma};
  const double hdt = 0.5 * g.dt;
  const double d[3] = {(v[0] - g.vgal[0]) * hdt, (v[1] - g.vgal[1]) * hdt,
                       (v[2] - g.vgal[2]) * hdt};
  LayoutAbs::move(x, d, g);
  {
    double *dst[3] = {gr.J[0], gr.J[1], gr.J[2]};
    const double val[3] = {qw * v[0], qw * v[1], qw * v[2]};
    scatter<ORDER, double>(g, LayoutAbs::cell(x, g), dst, val, 3);
  }
  LayoutAbs::move(x, d, g);
  {
    double *dst[1] = {gr.rho};
    const double one[1] = {qw};
    scatter<ORDER, double>(g, LayoutAbs::cell(x, g), dst, one, 1);
  }
  LayoutAbs::store(p, k, x);
}

template <int ORDER>
__global__ __launch_bounds__(256) void k_gather_push_abs(RunGeom g, PartPtrs p,
                                                         GridPtrs<double> gr, double h) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= p.n) return;
  double x[3], u[3], F[6];
  LayoutAbs::load(p, k, g, x);
  load_u(p, k, u);
  interpolate<ORDER, double>(g, LayoutAbs::cell(x, g), gr, F);
  boris(u, F, h);
  static_cast<double *>(p.ux)[k] = u[0];
  static_cast<double *>(p.uy)[k] = u[1];
  static_cast<double *>(p.uz)[k] = u[2];
}

// ---- mixed kernels ---------------------------------------------------------
__device__ __forceinline__ CellPos<float> load_cellpos(const PartPtrs &p, int64_t k,
                                                       const RunGeom &g) {
  CellPos<float> c;
  decode_cell(static_cast<const int *>(p.x)[k], g, c.i);
  c.o[0] = static_cast<const float *>(p.ox)[k];
  c.o[1] = static_cast<const float *>(p.oy)[k];
  c.o[2] = static_cast<const float *>(p.oz)[k];
  return c;
}

template <int ORDER>
__global__ __launch_bounds__(256) void k_deposit_cell(RunGeom g, PartPtrs p, GridPtrs<float> gr,
                                                      int move) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= p.n) return;
  const float qw = float(p.q * p.w / (g.dx * g.dy * g.dz));
  CellPos<float> c = load_cellpos(p, k, g);
  if (!move) {
    float *dst[1] = {gr.rho};
    const float one[1] = {qw};
    scatter<ORDER, float>(g, c, dst, one, 1);
    return;
  }
  float u[3];
  load_u(p, k, u);
  const float gamma = sqrtf(1.0f + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const float v[3] = {u[0] / gamma, u[1] / gamma, u[2] / gamma};
  const float d[3] = {(v[0] - float(g.vgal[0])) * float(0.5 * g.dt / g.dx),
                      (v[1] - float(g.vgal[1])) * float(0.5 * g.dt / g.dy),
                      (v[2] - float(g.vgal[2])) * float(0.5 * g.dt / g.dz)};
  move_cell(c.i, c.o, d, g);
  {
    float *dst[3] = {gr.J[0], gr.J[1], gr.J[2]};
    const float val[3] = {qw * v[0], qw * v[1], qw * v[2]};
    scatter<ORDER, float>(g, c, dst, val, 3);
  }
  move_cell(c.i, c.o, d, g);
  {
    float *dst[1] = {gr.rho};
    const float one[1] = {qw};
    scatter<ORDER, float>(g, c, dst, one, 1);
  }
  static_cast<int *>(p.x)[k] = encode_cell(c.i, g);
  static_cast<float *>(p.ox)[k] = c.o[0];
  static_cast<float *>(p.oy)[k] = c.o[1];
  static_cast<float *>(p.oz)[k] = c.o[2];
}

template <int ORDER>
__global__ __launch_bounds__(256) void k_gather_push_cell(RunGeom g, PartPtrs p,
                                                          GridPtrs<float> gr, float h) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= p.n) return;
  float u[3], F[6];
  const CellPos<float> c = load_cellpos(p, k, g);
  load_u(p, k, u);
  interpolate<ORDER, float>(g, c, gr, F);
  boris(u, F, h);
  static_cast<float *>(p.ux)[k] = u[0];
  static_cast<float *>(p.uy)[k] = u[1];
  static_cast<float *>(p.uz)[k] = u[2];
}

unsigned blocks_for(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace

template <>
void launch_deposit<double>(const RunGeom &g, const PartPtrs &p, const GridPtrs<double> &gr,
                            hipStream_t s) {
  if (p.n == 0) return;
  if (g.order == 1)
    hipLaunchKernelGGL((k_deposit_abs<1>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 1);
  else
    hipLaunchKernelGGL((k_deposit_abs<3>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 1);
}
template <>
void launch_deposit<float>(const RunGeom &g, const PartPtrs &p, const GridPtrs<float> &gr,
                           hipStream_t s) {
  if (p.n == 0) return;
  if (g.order == 1)
    hipLaunchKernelGGL((k_deposit_cell<1>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 1);
  else
    hipLaunchKernelGGL((k_deposit_cell<3>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 1);
}
template <>
void launch_deposit_rho<double>(const RunGeom &g, const PartPtrs &p, const GridPtrs<double> &gr,
                                hipStream_t s) {
  if (p.n == 0) return;
  if (g.order == 1)
    hipLaunchKernelGGL((k_deposit_abs<1>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 0);
  else
    hipLaunchKernelGGL((k_deposit_abs<3>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 0);
}
template <>
void launch_deposit_rho<float>(const RunGeom &g, const PartPtrs &p, const GridPtrs<float> &gr,
                               hipStream_t s) {
  if (p.n == 0) return;
  if (g.order == 1)
    hipLaunchKernelGGL((k_deposit_cell<1>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 0);
  else
    hipLaunchKernelGGL((k_deposit_cell<3>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr, 0);
}
template <>
void launch_gather_push<double>(const RunGeom &g, const PartPtrs &p,
                                const GridPtrs<double> &gr, double dt_push, hipStream_t s) {
  if (p.n == 0) return;
  const double h = p.q * dt_push / (2.0 * p.m);
  if (g.order == 1)
    hipLaunchKernelGGL((k_gather_push_abs<1>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr,
                       h);
  else
    hipLaunchKernelGGL((k_gather_push_abs<3>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr,
                       h);
}
template <>
void launch_gather_push<float>(const RunGeom &g, const PartPtrs &p, const GridPtrs<float> &gr,
                               double dt_push, hipStream_t s) {
  if (p.n == 0) return;
  const float h = float(p.q * dt_push / (2.0 * p.m));
  if (g.order == 1)
    hipLaunchKernelGGL((k_gather_push_cell<1>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr,
                       h);
  else
    hipLaunchKernelGGL((k_gather_push_cell<3>), dim3(blocks_for(p.n)), dim3(256), 0, s, g, p, gr,
                       h);
}

}  // namespace galpic
