// Galilean-PSATD k-space update and small spectral/real helpers.
//
// The update is one streaming pass over the half-spectrum modes: per mode it
// reads E, B (3+3), J (3), rho^n, rho^{n+1} and the six coefficients
// c0..c5 (see coef.hip), and writes E, B (paper's update equations):
//
//   B' = c0 B - c1 (ik x E) + c2 (ik x J)
//   E' = c0 E + c1 (ik x B) + c3 J + (c4 rho^{n+1} + c5 rho^n) ik
//
// k comes from the run's per-axis wavenumber tables (the exact k, or the
// symbol [k] of a finite-order stencil).  Modes on a Nyquist plane and
// k = 0 are written as zero, except in the slab solve's local grids, which
// advance every mode (at [k] = 0 the coefficients' limits give E' = E - dt J,
// B' = B).  HBM-bound: 17 complex values per mode move
// (136 B in float, 272 B in double) plus the 6 coefficients.
#include "kernels.hpp"

namespace galpic {
namespace {

// (ik x F)_a for real k and complex F
template <typename T>
__device__ __forceinline__ void ik_cross(T kx, T ky, T kz, const Cx<T> F[3], Cx<T> out[3]) {
  const Cx<T> c0 = cx(ky * F[2].re - kz * F[1].re, ky * F[2].im - kz * F[1].im);
  const Cx<T> c1 = cx(kz * F[0].re - kx * F[2].re, kz * F[0].im - kx * F[2].im);
  const Cx<T> c2 = cx(kx * F[1].re - ky * F[0].re, kx * F[1].im - ky * F[0].im);
  out[0] = mul_i(c0);
  out[1] = mul_i(c1);
  out[2] = mul_i(c2);
}

// Workgroup row blockIdx.y picks the run of the table (all of one grid shape).
template <typename T>
__global__ __launch_bounds__(256) void k_update(RunGeom g, const UpdatePtrs<T> *__restrict__ sets) {
  UpdatePtrs<T> p = sets[blockIdx.y];
  for (int a = 0; a < 3; ++a) {
    p.E[a] = global_ptr(p.E[a]);
    p.B[a] = global_ptr(p.B[a]);
    p.J[a] = global_ptr(p.J[a]);
  }
  p.rho_old = global_ptr(p.rho_old);
  p.rho_new = global_ptr(p.rho_new);
  for (int k = 0; k < 6; ++k) p.coef[k] = global_ptr(p.coef[k]);
  for (int a = 0; a < 3; ++a) p.k[a] = global_ptr(p.k[a]);
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= g.nmode) return;
  const int iz = int(idx % g.nzh);
  const int iy = int((idx / g.nzh) % g.ny);
  const int ix = int(idx / (int64_t(g.nzh) * g.ny));
  const bool held = !p.no_hold && (ix == g.nx / 2 || iy == g.ny / 2 || iz == g.nz / 2 ||
                                    (ix == 0 && iy == 0 && iz == 0));
  if (held) {
    const Cx<T> z = cx(T(0), T(0));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      p.E[a][idx] = z;
      p.B[a][idx] = z;
    }
    return;
  }
  const T kx = p.k[0][ix];
  const T ky = p.k[1][iy];
  const T kz = p.k[2][iz];
  Cx<T> E[3], B[3], J[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    E[a] = p.E[a][idx];
    B[a] = p.B[a][idx];
    J[a] = p.J[a][idx];
  }
  const Cx<T> r0 = p.rho_old[idx];
  const Cx<T> r1 = p.rho_new[idx];
  if (p.correct) {
    // Optional Galilean current correction: keep the transverse part of J
    // and set k.J so that the k-space continuity equation, integrated over
    // the step with J constant, holds exactly:
    //   rho^{n+1} = theta^2 rho^n + F k.J,  F = -i dt theta sinc(k.v_gal dt/2)
    const T kdv = kx * T(p.vgal[0]) + ky * T(p.vgal[1]) + kz * T(p.vgal[2]);
    const T half = T(0.5) * kdv * T(p.dt);
    const T sn = sin(half);
    const T cs = cos(half);
    const T sinc = half != T(0) ? sn / half : T(1);
    const Cx<T> th = cx(cs, sn);
    const Cx<T> num = r1 - (th * th) * r0;
    // target k.J = num / F = i num conj(theta) / (dt sinc)
    const Cx<T> target = (T(1) / (T(p.dt) * sinc)) * mul_i(num * conj(th));
    const Cx<T> kJ = kx * J[0] + ky * J[1] + kz * J[2];
    const Cx<T> alpha = (T(1) / (kx * kx + ky * ky + kz * kz)) * (target - kJ);
    J[0] = J[0] + kx * alpha;
    J[1] = J[1] + ky * alpha;
    J[2] = J[2] + kz * alpha;
  }
  const Cx<T> c0 = p.coef[0][idx];
  const Cx<T> c1 = p.coef[1][idx];
  const Cx<T> c2 = p.coef[2][idx];
  const Cx<T> c3 = p.coef[3][idx];
  const Cx<T> c4 = p.coef[4][idx];
  const Cx<T> c5 = p.coef[5][idx];
  Cx<T> kE[3], kB[3], kJ[3];
  ik_cross(kx, ky, kz, E, kE);
  ik_cross(kx, ky, kz, B, kB);
  ik_cross(kx, ky, kz, J, kJ);
  // (c4 rho^{n+1} + c5 rho^n) i
  const Cx<T> rho_i = mul_i(c4 * r1 + c5 * r0);
  const T kk[3] = {kx, ky, kz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const Cx<T> bn = c0 * B[a] - c1 * kE[a] + c2 * kJ[a];
    const Cx<T> en = c0 * E[a] + c1 * kB[a] + c3 * J[a] + kk[a] * rho_i;
    p.B[a][idx] = bn;
    p.E[a][idx] = en;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_project(RunGeom g, const T *__restrict__ kt, Cx<T> *F0,
                                                 Cx<T> *F1, Cx<T> *F2, int transverse) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= g.nmode) return;
  const int iz = int(idx % g.nzh);
  const int iy = int((idx / g.nzh) % g.ny);
  const int ix = int(idx / (int64_t(g.nzh) * g.ny));
  const bool held = ix == g.nx / 2 || iy == g.ny / 2 || iz == g.nz / 2 ||
                    (ix == 0 && iy == 0 && iz == 0);
  if (held) {
    const Cx<T> z = cx(T(0), T(0));
    F0[idx] = z;
    F1[idx] = z;
    F2[idx] = z;
    return;
  }
  if (!transverse) return;
  const T kx = kt[ix];
  const T ky = kt[g.nx + iy];
  const T kz = kt[g.nx + g.ny + iz];
  const T inv_k2 = T(1) / (kx * kx + ky * ky + kz * kz);
  const Cx<T> a = F0[idx], b = F1[idx], c = F2[idx];
  const Cx<T> kf = inv_k2 * (kx * a + ky * b + kz * c);
  F0[idx] = a - kx * kf;
  F1[idx] = b - ky * kf;
  F2[idx] = c - kz * kf;
}

template <typename T>
__global__ __launch_bounds__(256) void k_sum_squares(const T *__restrict__ a,
                                                     const T *__restrict__ b,
                                                     const T *__restrict__ c, int64_t n,
                                                     double *out) {
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double x = a[i], y = b[i], z = c[i];
    acc += x * x + y * y + z * z;
  }
  // wave reduction then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

// Workgroup row blockIdx.y clears segment blockIdx.y (a multiple of 16 bytes).
__global__ __launch_bounds__(256) void k_zero_segments(const ZeroSeg *__restrict__ segs) {
  const ZeroSeg &sg = segs[blockIdx.y];
  uint4 *p16 = static_cast<uint4 *>(global_ptr(sg.p));
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < sg.n16; i += stride)
    p16[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ __launch_bounds__(256) void k_zero(uint4 *p16, size_t n16, uint32_t *p4, size_t n4) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    p16[i] = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride) p4[i] = 0u;
}

}  // namespace

template <typename T>
void launch_update(const RunGeom &g, const UpdatePtrs<T> *sets, int nsets, hipStream_t s) {
  const unsigned blocks = unsigned((g.nmode + 255) / 256);
  hipLaunchKernelGGL((k_update<T>), dim3(blocks, unsigned(nsets)), dim3(256), 0, s, g, sets);
}

template <typename T>
void launch_project(const RunGeom &g, const T *kt, Cx<T> *F0, Cx<T> *F1, Cx<T> *F2,
                    bool transverse, hipStream_t s) {
  const unsigned blocks = unsigned((g.nmode + 255) / 256);
  hipLaunchKernelGGL((k_project<T>), dim3(blocks), dim3(256), 0, s, g, kt, F0, F1, F2,
                     transverse ? 1 : 0);
}

template <typename T>
void launch_sum_squares(const T *a, const T *b, const T *c, int64_t n, double *out,
                        hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_sum_squares<T>), dim3(unsigned(blocks)), dim3(256), 0, s, a, b, c, n,
                     out);
}

void launch_zero_segments(const ZeroSeg *segs, int nseg, size_t max_n16, hipStream_t s) {
  if (nseg <= 0 || max_n16 == 0) return;
  size_t blocks = (max_n16 + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_zero_segments, dim3(unsigned(blocks), unsigned(nseg)), dim3(256), 0, s,
                     segs);
}

void launch_zero(void *p, size_t nbytes, hipStream_t s) {
  if (nbytes == 0) return;
  // allocations are 256-byte aligned; the tail (if any) is cleared by words
  const size_t n16 = nbytes / 16;
  const size_t n4 = (nbytes - n16 * 16) / 4;
  uint32_t *tail = reinterpret_cast<uint32_t *>(static_cast<char *>(p) + n16 * 16);
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3(unsigned(blocks)), dim3(256), 0, s,
                     static_cast<uint4 *>(p), n16, tail, n4);
}

template void launch_update<float>(const RunGeom &, const UpdatePtrs<float> *, int, hipStream_t);
template void launch_update<double>(const RunGeom &, const UpdatePtrs<double> *, int,
                                    hipStream_t);
template void launch_project<float>(const RunGeom &, const float *, Cx<float> *, Cx<float> *,
                                    Cx<float> *, bool, hipStream_t);
template void launch_project<double>(const RunGeom &, const double *, Cx<double> *,
                                     Cx<double> *, Cx<double> *, bool, hipStream_t);
template void launch_sum_squares<float>(const float *, const float *, const float *, int64_t,
                                        double *, hipStream_t);
template void launch_sum_squares<double>(const double *, const double *, const double *,
                                         int64_t, double *, hipStream_t);

}  // namespace galpic
