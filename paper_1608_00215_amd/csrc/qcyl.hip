// Quasi-cylindrical (azimuthal-mode) Galilean-PSATD field solve.
//
// The paper's own runs use a quasi-3D spectral code (azimuthal modes, with
// discrete Hankel transforms along r in place of the transverse Fourier
// transforms) and state that the Galilean scheme does not depend on the
// geometry.  Readings (the paper does not print the cylindrical scheme):
//  - a mode m field is F_m(r, z) exp(i m theta); its components combine as
//    G_+ = (F_r + i F_theta) / 2 (Hankel order m+1), G_- = (F_r - i F_theta)
//    / 2 (order m-1), F_z and rho (order m);
//  - radial nodes r_j = (j + 1/2) dr; one spectral grid per mode for all
//    three orders, k_i = alpha_{m,i} / R (zeros of J_m, R = nr dr); the
//    backward transform of order p is F(r_j) = sum_i F^_i J_p(k_i r_j) and
//    the forward one its matrix inverse; z is periodic with the Cartesian
//    Fourier convention, and the k_z Nyquist plane is held at zero;
//  - the update is the Cartesian Galilean-PSATD update at k = (k_r, 0, k_z)
//    applied to F^_x = i (G^_- - G^_+), F^_y = -(G^_+ + G^_-), F^_z = G^_z
//    (the azimuth-0 Cartesian spectral field of the mode, up to a factor
//    common to every component), which is exact for v_gal along z since the
//    update commutes with rotations about z.
//
// Layout: every field is complex [mode][z][r] (r contiguous).  A step:
//  z transforms of J, rho (strided complex lines, the Cartesian c2c tile
//  kernel) -> forward Hankel transforms (a real matrix times complex rows: a
//  batched GEMM on the matrix cores) -> the mode update (one streaming pass
//  per mode) -> backward Hankel transforms of E, B -> inverse z transforms.
#include "galpic.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace galpic {
namespace {

constexpr int kQWaves = 4;  // waves per Hankel-transform workgroup, one z-row tile each
constexpr int kTC = 4;      // 16-column MFMA tiles per wave (64 output radial nodes)

enum { kVecFwd = 0, kVecBwd = 1, kScalarFwd = 2 };

// In/out arrays of one field of a Hankel-transform launch.
struct QcSet {
  const void *in[3];
  void *out[3];
};

typedef float qf32x4 __attribute__((ext_vector_type(4)));
typedef double qf64x4 __attribute__((ext_vector_type(4)));
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
  using type = qf32x4;
};
template <>
struct MfmaAcc<double> {
  using type = qf64x4;
};

// D += A B for a 16 x 4 A and a 4 x 16 B over one wave: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; element r of its accumulator is
// D[4 (l / 16) + r][l % 16] for the f32 instruction but D[l / 16 + 4 r][l % 16]
// for the f64 one (both checked on gfx950).
__device__ __forceinline__ qf32x4 mfma16(float a, float b, qf32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ qf64x4 mfma16(double a, double b, qf64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The Hankel transforms along r as batched real GEMMs on the matrix cores.
// Per (mode m, transform) the complex rows of a field ([z][r], r contiguous)
// are multiplied by a real nr x nr matrix stored as [k][i] (input radial or
// spectral index k, output index i).  A workgroup takes a tile of 8 z rows --
// 16 GEMM rows holding their real and imaginary parts -- against kTC
// 16-column tiles of outputs; its kQWaves waves split K (4 k per MFMA) and
// sum their partial tiles through LDS at the end, which keeps each wave's
// chain of dependent loads short on small grids.  Operands come straight
// from global memory (a row piece is 32 contiguous bytes per z, a matrix
// row piece 16 contiguous values, reused from L1/L2 by every workgroup of
// the mode).
//
// Matrix slots per mode: 0 = order m-1, 1 = order m, 2 = order m+1.
//  kVecFwd:    part 0: G^_+ (slot 2) and G^_- (slot 0) of (F_r +- i F_theta) / 2,
//              part 1: G^_z (slot 1) of F_z (all z-transformed)
//  kVecBwd:    part 0: F_r = G_+ + G_-, F_theta = -i (G_+ - G_-) from G^_+
//              (slot 2) and G^_- (slot 0); part 1: F_z (slot 1).  The inverse z
//              transform follows; the backward matrices carry its 1/nz.
//  kScalarFwd: in[0] -> out[0], slot 1.
// Grid: x = z-row tiles (or groups of 8), y = column blocks, z = (set, mode,
// part).
// One wave's share of a Hankel-transform launch: RT z-row tiles (8 rows
// each, 16 GEMM rows) against kTC column tiles, over the groups of K that
// fall to it.  KS = kQWaves: the workgroup's waves split K and sum their
// partial tiles through red (small grids: short load chains per wave);
// KS = 1: each wave takes all of K for its own row tiles (large grids: the
// RT row tiles share every matrix operand).
template <typename T, int KIND, bool PAIR, int RT, int KS>
__device__ __forceinline__ void hankel_tile(const QcSet &st, const T *__restrict__ mats, int nz,
                                            int nr, int m, int rt0, int col0, int lane,
                                            int wave, T *__restrict__ red) {
  using V = typename MfmaAcc<T>::type;
  const int l16 = lane & 15, g = lane >> 4;
  const int64_t plane = int64_t(m) * nz * nr;
  // GEMM row rho of a 16-row tile <-> z row 8 rt + zr(rho), real (c = 0)
  // or imaginary (c = 1) part, chosen per instruction so that the four
  // accumulator elements of a lane are two whole complex values: f32 rows
  // 4 g + r give zr = 2 g + r / 2, c = r & 1; f64 rows g + 4 r give
  // zr = g + 4 (r / 2), c = r & 1.
  constexpr bool kF32 = sizeof(T) == 4;
  const int zr = kF32 ? (l16 >> 1) : ((l16 & 3) + ((l16 >> 3) << 2));
  const int ca = kF32 ? (l16 & 1) : ((l16 >> 2) & 1);
  int64_t arow[RT];  // in T units
#pragma unroll
  for (int q = 0; q < RT; ++q) arow[q] = 2 * (plane + int64_t((rt0 + q) * 8 + zr) * nr) + ca;
  const int64_t msz = int64_t(nr) * nr;
  const T *__restrict__ M = global_ptr(mats) + int64_t(m) * 3 * msz;
  const T *__restrict__ B0 = M + (PAIR ? 2 : 1) * msz;
  const T *__restrict__ B1 = M;  // slot 0 (pair only)
  const T *__restrict__ in0 =
      global_ptr(static_cast<const T *>(st.in[KIND == kScalarFwd ? 0 : (PAIR ? 0 : 2)]));
  const T *__restrict__ in1 = global_ptr(static_cast<const T *>(st.in[PAIR ? 1 : 0]));

  V acc0[RT][kTC], acc1[RT][kTC];
#pragma unroll
  for (int q = 0; q < RT; ++q)
#pragma unroll
    for (int t = 0; t < kTC; ++t) {
      acc0[q][t] = V{0, 0, 0, 0};
      acc1[q][t] = V{0, 0, 0, 0};
    }
  // Operands of kKU consecutive k-steps.  Every index is clamped into range,
  // so the loads need no branches; the K padding (k >= nr) is zeroed by
  // multiplying the matrix operand by 0 (matrix entries are finite, so this
  // is exact, and the padded products then vanish), and columns i >= nr are
  // computed from clamped values but never stored.
  constexpr int kKU = 2;
  struct Ops {
    T a0[kKU][RT], a1[kKU][RT], b0[kKU][kTC], b1[kKU][kTC];
  };
  int icl[kTC];
#pragma unroll
  for (int t = 0; t < kTC; ++t) icl[t] = min(col0 + 16 * t + l16, nr - 1);
  auto load = [&](int s0, Ops &o) {
#pragma unroll
    for (int u = 0; u < kKU; ++u) {
      const int k = 4 * (s0 + u) + g;
      const int kc = min(k, nr - 1);
      const T kmask = k < nr ? T(1) : T(0);
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        const int64_t at = arow[q] + 2 * int64_t(kc);
        if (KIND == kVecFwd && PAIR) {
          // (F_r +- i F_theta) / 2: the real part takes F_r.re -+ F_theta.im,
          // the imaginary part F_r.im +- F_theta.re
          const T fr = in0[at];
          const T ft = in1[at + (ca ? -1 : 1)];
          const T sft = ca ? ft : -ft;
          o.a0[u][q] = T(0.5) * (fr + sft);
          o.a1[u][q] = T(0.5) * (fr - sft);
        } else {
          o.a0[u][q] = in0[at];
          if (PAIR) o.a1[u][q] = in1[at];
        }
      }
      const int64_t row = int64_t(kc) * nr;
#pragma unroll
      for (int t = 0; t < kTC; ++t) {
        o.b0[u][t] = B0[row + icl[t]] * kmask;
        if (PAIR) o.b1[u][t] = B1[row + icl[t]] * kmask;
      }
    }
  };
  auto mma = [&](const Ops &o) {
#pragma unroll
    for (int u = 0; u < kKU; ++u)
#pragma unroll
      for (int q = 0; q < RT; ++q) {
#pragma unroll
        for (int t = 0; t < kTC; ++t)
          acc0[q][t] = mfma16(o.a0[u][q], o.b0[u][t], acc0[q][t]);
        if (PAIR) {
#pragma unroll
          for (int t = 0; t < kTC; ++t)
            acc1[q][t] = mfma16(o.a1[u][q], o.b1[u][t], acc1[q][t]);
        }
      }
  };
  // Groups of kKU k-steps; this wave takes groups kw, kw + KS, kw + 2 KS, ...
  // (kw = its place among the KS waves sharing K), two at a time through two
  // operand sets, so the loads of one group are in flight during the other's
  // MFMAs.  A group past nr has a zero matrix operand and adds nothing, so
  // the count is rounded up to even; the last prefetch rereads a group in
  // range.
  const int kw = KS > 1 ? wave : 0;
  const int ngroups = (nr + 4 * kKU - 1) / (4 * kKU);
  const int mine = (ngroups - kw + KS - 1) / KS;  // may be 0
  const int npairs = (mine + 1) / 2;
  auto group = [&](int j) { return kKU * min(kw + KS * j, ngroups); };
  Ops X, Y;
  if (npairs > 0) load(group(0), X);
  for (int s = 0; s < npairs; ++s) {
    load(group(2 * s + 1), Y);
    mma(X);
    load(group(min(2 * s + 2, 2 * npairs - 1)), X);
    mma(Y);
  }
  constexpr int kNA = PAIR ? 2 : 1;
  if (KS > 1) {
    // partial tiles of the waves: red holds [wave][acc][t][4][64] (RT = 1);
    // wave w then finishes the column tiles t with t % KS == w
#pragma unroll
    for (int t = 0; t < kTC; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        red[(((wave * kNA + 0) * kTC + t) * 4 + r) * 64 + lane] = acc0[0][t][r];
        if (PAIR) red[(((wave * kNA + 1) * kTC + t) * 4 + r) * 64 + lane] = acc1[0][t][r];
      }
    __syncthreads();
  }
  // accumulator elements 2 h, 2 h + 1 of a lane: the real and imaginary
  // parts at z row 8 rt + (2 g + h) (f32) or 8 rt + (g + 4 h) (f64)
#pragma unroll
  for (int q = 0; q < RT; ++q)
#pragma unroll
    for (int t = 0; t < kTC; ++t) {
      if (KS > 1 && t % KS != wave) continue;
      const int i = col0 + 16 * t + l16;
      if (i >= nr) continue;
      T s0[4], s1[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (KS > 1) {
          s0[r] = T(0);
          s1[r] = T(0);
#pragma unroll
          for (int w = 0; w < KS; ++w) {
            s0[r] += red[(((w * kNA + 0) * kTC + t) * 4 + r) * 64 + lane];
            if (PAIR) s1[r] += red[(((w * kNA + 1) * kTC + t) * 4 + r) * 64 + lane];
          }
        } else {
          s0[r] = acc0[q][t][r];
          s1[r] = acc1[q][t][r];
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int zo = (rt0 + q) * 8 + (kF32 ? 2 * g + h : g + 4 * h);
        const int64_t at = plane + int64_t(zo) * nr + i;
        const Cx<T> p = cx(s0[2 * h], s0[2 * h + 1]);
        if (!PAIR) {
          Cx<T> *o = global_ptr(static_cast<Cx<T> *>(st.out[KIND == kScalarFwd ? 0 : 2]));
          o[at] = p;
          continue;
        }
        const Cx<T> qv = cx(s1[2 * h], s1[2 * h + 1]);
        Cx<T> *o0 = global_ptr(static_cast<Cx<T> *>(st.out[0]));
        Cx<T> *o1 = global_ptr(static_cast<Cx<T> *>(st.out[1]));
        if (KIND == kVecBwd) {
          o0[at] = p + qv;                  // F_r
          o1[at] = T(-1) * mul_i(p - qv);   // F_theta = -i (G_+ - G_-)
        } else {
          o0[at] = p;                       // G^_+
          o1[at] = qv;                      // G^_-
        }
      }
    }
}

// WIDE = false: a workgroup is one z-row tile, its waves splitting K.
// WIDE = true: a workgroup is 8 z-row tiles, 2 per wave (needs nz % 64 == 0).
template <typename T, int KIND, bool WIDE>
__global__ __launch_bounds__(64 * kQWaves) void k_qc_hankel(const QcSet *__restrict__ sets,
                                                            const T *__restrict__ mats, int nz,
                                                            int nr, int nmodes, int nparts) {
  // partial tiles of the waves when they split K: [wave][pair][kTC][4][64]
  __shared__ T red[WIDE ? 1 : kQWaves * 2 * kTC * 4 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int part = blockIdx.z % nparts;
  const int m = (blockIdx.z / nparts) % nmodes;
  const QcSet st = sets[blockIdx.z / (nparts * nmodes)];
  const int col0 = blockIdx.y * 16 * kTC;
  if (WIDE) {
    const int rt0 = (blockIdx.x * kQWaves + wave) * 2;  // z rows 8 rt0 .. 8 rt0 + 15
    if (KIND != kScalarFwd && part == 0)
      hankel_tile<T, KIND, true, 2, 1>(st, mats, nz, nr, m, rt0, col0, lane, wave, red);
    else
      hankel_tile<T, KIND, false, 2, 1>(st, mats, nz, nr, m, rt0, col0, lane, wave, red);
  } else {
    const int rt = blockIdx.x;  // z rows 8 rt .. 8 rt + 7 (nz is a multiple of 8)
    if (KIND != kScalarFwd && part == 0)
      hankel_tile<T, KIND, true, 1, kQWaves>(st, mats, nz, nr, m, rt, col0, lane, wave, red);
    else
      hankel_tile<T, KIND, false, 1, kQWaves>(st, mats, nz, nr, m, rt, col0, lane, wave, red);
  }
}

// The mode update's arrays.
template <typename T>
struct QcUpd {
  Cx<T> *E[3], *B[3];           // G^_+, G^_-, G^_z
  const Cx<T> *J[3];
  const Cx<T> *rho_old, *rho_new;
  const Cx<T> *coef[6];         // [mode][k_z][k_r]
  const T *kr;                  // [mode][k_r]
};

// (ik x F) for k = (kr, 0, kz)
template <typename T>
__device__ __forceinline__ void ik_cross_r0z(T kr, T kz, const Cx<T> F[3], Cx<T> o[3]) {
  o[0] = mul_i(T(-1) * (kz * F[1]));
  o[1] = mul_i(kz * F[0] - kr * F[2]);
  o[2] = mul_i(kr * F[1]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_qc_update(QcUpd<T> p, int nmodes, int nz, int nr,
                                                   T kzfac) {
  const int64_t n = int64_t(nmodes) * nz * nr;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int i = int(idx % nr);
  const int iz = int((idx / nr) % nz);
  const int m = int(idx / (int64_t(nz) * nr));
  if (iz == nz / 2) {
    const Cx<T> z = cx(T(0), T(0));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      p.E[a][idx] = z;
      p.B[a][idx] = z;
    }
    return;
  }
  const T kr = p.kr[int64_t(m) * nr + i];  // 0 in a held column
  const T kz = T(iz < nz / 2 ? iz : iz - nz) * kzfac;
  // modes m >= 1 hold the last k_r column of G_+, G_z and the scalars at
  // zero; G_- carries its k_r = 0 function there
  const bool held = m >= 1 && i == nr - 1;
  // azimuth-0 Cartesian components: x = i (G_- - G_+), y = -(G_+ + G_-), z
  auto to_cart = [](const Cx<T> g[3], Cx<T> f[3]) {
    f[0] = mul_i(g[1] - g[0]);
    f[1] = T(-1) * (g[0] + g[1]);
    f[2] = g[2];
  };
  Cx<T> Eg[3], Bg[3], Jg[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool zero = held && a != 1;
    Eg[a] = zero ? cx(T(0), T(0)) : p.E[a][idx];
    Bg[a] = zero ? cx(T(0), T(0)) : p.B[a][idx];
    Jg[a] = zero ? cx(T(0), T(0)) : p.J[a][idx];
  }
  Cx<T> E[3], B[3], J[3];
  to_cart(Eg, E);
  to_cart(Bg, B);
  to_cart(Jg, J);
  const Cx<T> r0 = held ? cx(T(0), T(0)) : p.rho_old[idx];
  const Cx<T> r1 = held ? cx(T(0), T(0)) : p.rho_new[idx];
  const Cx<T> c0 = p.coef[0][idx], c1 = p.coef[1][idx], c2 = p.coef[2][idx];
  const Cx<T> c3 = p.coef[3][idx], c4 = p.coef[4][idx], c5 = p.coef[5][idx];
  Cx<T> kE[3], kB[3], kJ[3];
  ik_cross_r0z(kr, kz, E, kE);
  ik_cross_r0z(kr, kz, B, kB);
  ik_cross_r0z(kr, kz, J, kJ);
  const Cx<T> rho_i = mul_i(c4 * r1 + c5 * r0);
  const T kk[3] = {kr, T(0), kz};
  Cx<T> En[3], Bn[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Bn[a] = c0 * B[a] - c1 * kE[a] + c2 * kJ[a];
    En[a] = c0 * E[a] + c1 * kB[a] + c3 * J[a] + kk[a] * rho_i;
  }
  // back: G_+ = (i / 2)(x + i y), G_- = -(i / 2)(x - i y)
  auto from_cart = [held](const Cx<T> f[3], Cx<T> *const g[3], int64_t at) {
    const Cx<T> z = cx(T(0), T(0));
    g[0][at] = held ? z : T(0.5) * mul_i(f[0] + mul_i(f[1]));
    g[1][at] = T(-0.5) * mul_i(f[0] - mul_i(f[1]));
    g[2][at] = held ? z : f[2];
  };
  from_cart(En, p.E, idx);
  from_cart(Bn, p.B, idx);
}

// ---- particles: deposition and gather by azimuthal mode --------------------
// B-spline shapes of order O (1 linear, 3 cubic) in r (nodes (j + 1/2) dr)
// and z (nodes k dz, periodic).  A stored mode-m field is c_m f_m (c_0 = 1,
// c_m = 2), so the physical field is Re sum_m g_m exp(i m theta).  A radial
// node j < 0 (at r = (j + 1/2) dr < 0) is node -j-1 seen across the axis: its
// weight goes there with (-1)^m for scalars and z components and (-1)^(m+1)
// for r and theta components.  Node j's volume is the integral of its
// (folded) weight against 2 pi r dr dz.  Weights past the last node are
// dropped.  At r = 0 the angle is taken as 0.

template <typename T>
struct QcPart {
  T *x, *y, *z, *ux, *uy, *uz;
  int64_t n;
};

template <typename T>
struct QcGeo {
  int nmodes, nz, nr;
  T inv_dz, inv_dr, lz;
  const T *inv_vol;  // [nr]
};

// B-spline weights of the O + 1 nodes around an offset f in [0, 1): linear
// {1 - f, f} on nodes 0, 1; cubic on nodes -1 .. 2.
template <typename T, int O>
__device__ __forceinline__ void qc_weights(T f, T *w) {
  if (O == 1) {
    w[0] = T(1) - f;
    w[1] = f;
  } else {
    const T g = T(1) - f, f2 = f * f, f3 = f2 * f;
    w[0] = g * g * g / T(6);
    w[1] = (T(4) - T(6) * f2 + T(3) * f3) / T(6);
    w[2] = (T(1) + T(3) * f + T(3) * f2 - T(3) * f3) / T(6);
    w[3] = f3 / T(6);
  }
}

template <typename T, int O>
struct QcNodes {
  int j0;          // first radial node (may be negative: folded)
  T wr[O + 1];
  int k[O + 1];    // z nodes, wrapped
  T wz[O + 1];
};

template <typename T, int O>
__device__ __forceinline__ QcNodes<T, O> qc_nodes(const QcGeo<T> &g, T r, T z) {
  QcNodes<T, O> o;
  constexpr int lo = O == 1 ? 0 : -1;  // offset of the first node
  const T sr = r * g.inv_dr - T(0.5);
  const T fj = floor(sr);
  o.j0 = int(fj) + lo;
  qc_weights<T, O>(sr - fj, o.wr);
  const T sz = z * g.inv_dz;
  const T fk = floor(sz);
  qc_weights<T, O>(sz - fk, o.wz);
  int k = (int(fk) + lo) % g.nz;
  if (k < 0) k += g.nz;
#pragma unroll
  for (int b = 0; b <= O; ++b) {
    o.k[b] = k;
    k = k + 1 == g.nz ? 0 : k + 1;
  }
  return o;
}

// cos, sin of the particle's angle (1, 0 at r = 0) and r
template <typename T>
__device__ __forceinline__ void qc_angle(T x, T y, T &r, T &c, T &s) {
  r = sqrt(x * x + y * y);
  if (r > T(0)) {
    c = x / r;
    s = y / r;
  } else {
    c = T(1);
    s = T(0);
  }
}

// Add c_m val exp(-i m theta) W s / V to the four nodes of every mode,
// through add(m, k, j, re, im).
template <typename T, int O, typename Add>
__device__ __forceinline__ void qc_deposit(const QcGeo<T> &g, const QcNodes<T, O> &nd, T c, T s,
                                           T val, bool transverse, Add &&add) {
  T er = T(1), ei = T(0);  // exp(-i m theta), advanced per mode
  for (int m = 0; m < g.nmodes; ++m) {
    const T cm = m == 0 ? T(1) : T(2);
    const T fold = ((m + (transverse ? 1 : 0)) & 1) ? T(-1) : T(1);
    const T vr = cm * val * er, vi = cm * val * ei;
#pragma unroll
    for (int a = 0; a <= O; ++a) {
      const int j = nd.j0 + a;
      const int jj = j < 0 ? -j - 1 : j;
      if (jj >= g.nr) continue;
      const T wr = nd.wr[a] * (j < 0 ? fold : T(1)) * g.inv_vol[jj];
#pragma unroll
      for (int b = 0; b <= O; ++b) {
        const T w = wr * nd.wz[b];
        add(m, nd.k[b], jj, w * vr, w * vi);
      }
    }
    // exp(-i (m+1) theta) = exp(-i m theta) (c - i s)
    const T nr_ = er * c + ei * s, ni = ei * c - er * s;
    er = nr_;
    ei = ni;
  }
}

// global atomics into a [mode][z][r] complex array (mode 0 adds no
// imaginary parts: they are exact zeros)
template <typename T>
struct GlobalSink {
  T *arr;
  int nz, nr;
  __device__ __forceinline__ void operator()(int m, int k, int j, T re, T im) const {
    const int64_t at = 2 * ((int64_t(m) * nz + k) * nr + j);
    atomicAdd(arr + at, re);
    if (m > 0) atomicAdd(arr + at + 1, im);
  }
};

// Re sum_m (sum over nodes of W s g_m) exp(i m theta) for one component.
template <typename T, int O>
__device__ __forceinline__ T qc_gather(const QcGeo<T> &g, const T *__restrict__ arr,
                                       const QcNodes<T, O> &nd, T c, T s, bool transverse) {
  const int64_t plane = int64_t(g.nz) * g.nr;
  T er = T(1), ei = T(0);  // exp(i m theta)
  T out = T(0);
  for (int m = 0; m < g.nmodes; ++m) {
    const T fold = ((m + (transverse ? 1 : 0)) & 1) ? T(-1) : T(1);
    T ar = T(0), ai = T(0);
#pragma unroll
    for (int a = 0; a <= O; ++a) {
      const int j = nd.j0 + a;
      const int jj = j < 0 ? -j - 1 : j;
      if (jj >= g.nr) continue;
      const T wr = nd.wr[a] * (j < 0 ? fold : T(1));
#pragma unroll
      for (int b = 0; b <= O; ++b) {
        const int k = nd.k[b];
        const T w = wr * nd.wz[b];
        const int64_t at = 2 * (int64_t(m) * plane + int64_t(k) * g.nr + jj);
        ar += w * arr[at];
        ai += w * arr[at + 1];
      }
    }
    out += ar * er - ai * ei;
    const T nr_ = er * c - ei * s, ni = ei * c + er * s;
    er = nr_;
    ei = ni;
  }
  return out;
}

template <typename T>
struct QcSrc {
  T *jr, *jt, *jz, *rho;
};

// One particle's part of a move-and-deposit: with move, x^n -> x_h (J
// deposited with v = u / gamma) -> x^{n+1} (stored; rho deposited there);
// without, rho at x.  Moves use v - v_gal (v_gal along z); z wraps, x and y
// are open.  sink(s) gives the sink of source s (0 J_r, 1 J_theta, 2 J_z,
// 3 rho).
template <typename T, int O, typename SinkOf>
__device__ __forceinline__ void qc_particle_deposit(const QcPart<T> &p, const QcGeo<T> &g,
                                                    int64_t i, T dt, T vgal, T qw, int move,
                                                    SinkOf &&sink) {
  T x = p.x[i], y = p.y[i], z = p.z[i];
  if (move) {
    const T ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
    const T ig = T(1) / sqrt(T(1) + ux * ux + uy * uy + uz * uz);
    const T vx = ux * ig, vy = uy * ig, vz = uz * ig;
    const T h = T(0.5) * dt;
    auto wrap = [&](T zz) {
      zz -= g.lz * floor(zz / g.lz);
      return zz >= g.lz ? zz - g.lz : zz;
    };
    x += h * vx;
    y += h * vy;
    z = wrap(z + h * (vz - vgal));
    T r, c, s;
    qc_angle(x, y, r, c, s);
    const QcNodes<T, O> nd = qc_nodes<T, O>(g, r, z);
    const T vr = vx * c + vy * s, vt = -vx * s + vy * c;
    qc_deposit(g, nd, c, s, qw * vr, true, sink(0));
    qc_deposit(g, nd, c, s, qw * vt, true, sink(1));
    qc_deposit(g, nd, c, s, qw * vz, false, sink(2));
    x += h * vx;
    y += h * vy;
    z = wrap(z + h * (vz - vgal));
    p.x[i] = x;
    p.y[i] = y;
    p.z[i] = z;
  }
  T r, c, s;
  qc_angle(x, y, r, c, s);
  qc_deposit(g, qc_nodes<T, O>(g, r, z), c, s, qw, false, sink(3));
}

template <typename T, int O>
__global__ __launch_bounds__(256) void k_qc_move_deposit(QcPart<T> p, QcGeo<T> g, QcSrc<T> src,
                                                         T dt, T vgal, T qw, int move) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  T *arrs[4] = {global_ptr(src.jr), global_ptr(src.jt), global_ptr(src.jz),
                global_ptr(src.rho)};
  qc_particle_deposit<T, O>(p, g, i, dt, vgal, qw, move, [=](int si) {
    return GlobalSink<T>{arrs[si], g.nz, g.nr};
  });
}

// The same with an LDS window: a workgroup takes per x kQcDepThreads consecutive
// particles (sorted along z at binding, so a chunk covers few z nodes),
// accumulates the nodes of a window of z planes (4 for linear shapes from
// one plane below its first particle, 6 for cubic ones from two below) in
// LDS, sends every other node straight to global atomics, and flushes the
// window's nonzero entries with global atomics at the end.  The window is
// [source][mode][plane][part][r] in double for either precision: real and
// imaginary parts in separate rows, so that lanes adding to random radial
// nodes spread over all LDS banks (interleaved, the real parts of a row
// would fall on a quarter of them).  512 threads share one window (the
// cubic window allows one workgroup per CU): eight waves per CU hide the
// LDS atomics' conflicts better than four; measured against 256 x 8 and
// 512 x 1 particles per workgroup, 512 x 2 or 3 were fastest.  The launch
// picks per (2 to 4 particles per thread) to leave the smallest tail of
// workgroup rounds on the device.
constexpr int kQcDepThreads = 512;
template <int O>
constexpr int qc_win() {
  return O == 1 ? 4 : 6;
}

template <typename T, int O>
__global__ __launch_bounds__(kQcDepThreads) void k_qc_move_deposit_tiled(QcPart<T> p, QcGeo<T> g,
                                                                         QcSrc<T> src, T dt,
                                                                         T vgal, T qw, int move,
                                                                         int per, int *outside) {
  // the window accumulates in double whatever T is (as the Cartesian tiles do)
  extern __shared__ __align__(16) unsigned char qdsm[];
  double *win = reinterpret_cast<double *>(qdsm);
  __shared__ int zs_sh;
  const int64_t first = int64_t(blockIdx.x) * kQcDepThreads * per;
  constexpr int kQcWin = qc_win<O>();
  const int plane = g.nr * 2;                            // values per z plane
  const int per_src = g.nmodes * kQcWin * plane;
  const int total = 4 * per_src;
  if (threadIdx.x == 0) {
    // one plane (linear) or two (cubic) below the first particle's z cell
    // after its first half move
    T z = p.z[first];
    if (move) {
      const T ux = p.ux[first], uy = p.uy[first], uz = p.uz[first];
      const T vz = uz / sqrt(T(1) + ux * ux + uy * uy + uz * uz);
      z += T(0.5) * dt * (vz - vgal);
    }
    int k = int(floor(z * g.inv_dz)) % g.nz;
    if (k < 0) k += g.nz;
    zs_sh = (k - (O == 1 ? 1 : 2) + 2 * g.nz) % g.nz;
  }
  for (int t = threadIdx.x; t < total; t += kQcDepThreads) win[t] = 0.0;
  __syncthreads();
  const int zs = zs_sh;
  T *arrs[4] = {global_ptr(src.jr), global_ptr(src.jt), global_ptr(src.jz),
                global_ptr(src.rho)};
  const int nz = g.nz, nr = g.nr;
  int n_out = 0;  // this thread's particles with a node outside the window
  for (int q = 0; q < per; ++q) {
    const int64_t i = first + int64_t(q) * kQcDepThreads + threadIdx.x;
    if (i >= p.n) break;
    bool out = false;
    qc_particle_deposit<T, O>(p, g, i, dt, vgal, qw, move, [=, &out](int si) {
      T *garr = arrs[si];
      double *warr = win + si * per_src;
      return [=, &out](int m, int k, int j, T re, T im) {
        int slot = k - zs;
        if (slot < 0) slot += nz;
        // workgroup-scope adds for the window, device-scope ones for the
        // grid (distinct scopes also keep the two from being merged into
        // one flat atomic on a selected address)
        if (slot < kQcWin) {
          double *w = warr + (m * kQcWin + slot) * plane + j;
          __hip_atomic_fetch_add(w, double(re), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (m > 0)
            __hip_atomic_fetch_add(w + nr, double(im), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
          const int64_t at = 2 * ((int64_t(m) * nz + k) * nr + j);
          __hip_atomic_fetch_add(garr + at, re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (m > 0)
            __hip_atomic_fetch_add(garr + at + 1, im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          out = true;
        }
      };
    });
    n_out += out ? 1 : 0;
  }
  // the count for the re-sort decision: one atomic per wave
  for (int off = 32; off > 0; off >>= 1) n_out += __shfl_down(n_out, off, 64);
  if ((threadIdx.x & 63) == 0 && n_out > 0) atomicAdd(outside, n_out);
  __syncthreads();
  for (int t = threadIdx.x; t < total; t += kQcDepThreads) {
    const T v = T(win[t]);
    if (v == T(0)) continue;
    const int si = t / per_src;
    const int r1 = t % per_src;
    const int m = r1 / (kQcWin * plane);
    const int r2 = r1 % (kQcWin * plane);
    const int slot = r2 / plane;
    const int e0 = r2 % plane;  // part * nr + j
    const int e = 2 * (e0 % g.nr) + e0 / g.nr;
    const int k = (zs + slot) % g.nz;
    atomicAdd(global_ptr(arrs[si] + 2 * ((int64_t(m) * g.nz + k) * g.nr) + e), v);
  }
}

// ---- re-sort of the particles along z ---------------------------------------
// The order along z made at binding decays as the particles move, and the
// deposit's chunks then reach outside their LDS windows (on the 1.18 M-
// particle cubic column: 0.8 % of the particles at step 100, 4.5 % at step
// 1000, with the deposit 240 -> 374 us).  The deposit counts them; before
// each deposit a one-thread kernel decides from that count whether to sort
// again (more than n / resort_div since the last decision), and the sort
// kernels return at once when it did not.  The sort is a counting sort by z
// cell: global counts, their scan, then each workgroup's particles placed by
// a per-workgroup histogram (one global atomic per bin and workgroup) into
// staging arrays, and copied back.  Control words: ctl[0] the count,
// ctl[1] the decision, ctl[2 .. 2 + nz) counts, ctl[2 + nz .. 2 + 2 nz)
// offsets.
constexpr int kQcSortThreads = 256;
constexpr int kQcSortPer = 8;  // particles per thread of the count and scatter
constexpr int kQcMaxNz = 1024;
constexpr int kQcResortEvery = 16;

__global__ void k_qcz_decide(int *ctl, int64_t n, int div) {
  const int64_t out = ctl[0];
  ctl[1] = (div > 0 && out * div > n) ? 1 : 0;
  ctl[0] = 0;
}

template <typename T>
__device__ __forceinline__ int qc_zcell(T z, const QcGeo<T> &g) {
  int k = int(floor(z * g.inv_dz)) % g.nz;
  return k < 0 ? k + g.nz : k;
}

template <typename T>
__global__ __launch_bounds__(kQcSortThreads) void k_qcz_count(QcPart<T> p, QcGeo<T> g,
                                                              int *ctl) {
  if (!ctl[1]) return;
  __shared__ int h[kQcMaxNz];
  for (int b = threadIdx.x; b < g.nz; b += kQcSortThreads) h[b] = 0;
  __syncthreads();
  const int64_t first = int64_t(blockIdx.x) * kQcSortThreads * kQcSortPer;
  for (int q = 0; q < kQcSortPer; ++q) {
    const int64_t i = first + int64_t(q) * kQcSortThreads + threadIdx.x;
    if (i < p.n) atomicAdd(&h[qc_zcell(p.z[i], g)], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < g.nz; b += kQcSortThreads)
    if (h[b]) atomicAdd(&ctl[2 + b], h[b]);
}

// exclusive scan of the counts into the offsets; the counts cleared
__global__ __launch_bounds__(kQcMaxNz) void k_qcz_scan(int *ctl, int nz) {
  if (!ctl[1]) return;
  __shared__ int v[kQcMaxNz];
  const int t = threadIdx.x;
  v[t] = t < nz ? ctl[2 + t] : 0;
  __syncthreads();
  for (int off = 1; off < kQcMaxNz; off <<= 1) {
    const int a = t >= off ? v[t - off] : 0;
    __syncthreads();
    v[t] += a;
    __syncthreads();
  }
  if (t < nz) {
    ctl[2 + nz + t] = v[t] - ctl[2 + t];
    ctl[2 + t] = 0;
  }
}

template <typename T>
__global__ __launch_bounds__(kQcSortThreads) void k_qcz_scatter(QcPart<T> p, QcGeo<T> g,
                                                                int *ctl, T *tmp) {
  if (!ctl[1]) return;
  __shared__ int h[kQcMaxNz];
  __shared__ int base[kQcMaxNz];
  for (int b = threadIdx.x; b < g.nz; b += kQcSortThreads) h[b] = 0;
  __syncthreads();
  const int64_t first = int64_t(blockIdx.x) * kQcSortThreads * kQcSortPer;
  int key[kQcSortPer];
#pragma unroll
  for (int q = 0; q < kQcSortPer; ++q) {
    const int64_t i = first + int64_t(q) * kQcSortThreads + threadIdx.x;
    key[q] = i < p.n ? qc_zcell(p.z[i], g) : -1;
    if (key[q] >= 0) atomicAdd(&h[key[q]], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < g.nz; b += kQcSortThreads) {
    base[b] = h[b] ? atomicAdd(&ctl[2 + g.nz + b], h[b]) : 0;
    h[b] = 0;
  }
  __syncthreads();
  T *src[6] = {p.x, p.y, p.z, p.ux, p.uy, p.uz};
#pragma unroll
  for (int q = 0; q < kQcSortPer; ++q) {
    if (key[q] < 0) continue;
    const int64_t i = first + int64_t(q) * kQcSortThreads + threadIdx.x;
    const int64_t to = base[key[q]] + atomicAdd(&h[key[q]], 1);
#pragma unroll
    for (int a = 0; a < 6; ++a) tmp[a * p.n + to] = src[a][i];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_qcz_copyback(QcPart<T> p, const int *ctl,
                                                      const T *tmp) {
  if (!ctl[1]) return;
  T *dst[6] = {p.x, p.y, p.z, p.ux, p.uy, p.uz};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < p.n;
       i += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 6; ++a) dst[a][i] = tmp[a * p.n + i];
  }
}

// Reset the four real-space sources before a deposit: each takes the
// background's values, or zero (n values of the real type per array).
template <typename T>
__global__ __launch_bounds__(256) void k_qc_reset_sources(QcSrc<T> dst, QcSrc<T> bg, int has_bg,
                                                          int64_t n) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= 4 * n) return;
  const int a = int(idx / n);
  const int64_t i = idx % n;
  T *d = a == 0 ? dst.rho : (a == 1 ? dst.jr : (a == 2 ? dst.jt : dst.jz));
  const T *b = a == 0 ? bg.rho : (a == 1 ? bg.jr : (a == 2 ? bg.jt : bg.jz));
  d[i] = has_bg ? b[i] : T(0);
}

// Gather E, B at x (the mode fields [m][z][r]: r, theta, z components), then
// the relativistic Boris push of u over dt (c = 1).
// Gather and push over blocks of 256 particles.  The particles are sorted
// along z only, so consecutive ones sit at random radii; a counting sort of
// each block by radial cell in LDS hands lane l the block's particle of rank
// l, so that neighbouring lanes read neighbouring nodes (the particles stay
// where they are; each is still pushed exactly once).  Measured on the
// 1.18 M-particle column: cubic gathers 5-9 % faster, linear double 11 %;
// linear float, whose gather is cheapest, 7 % slower, so it keeps the plain
// order.
constexpr int kQcGatherBins = 512;  // radial cells (nr <= 512; larger radii clamp)

template <typename T, int O>
__global__ __launch_bounds__(256) void k_qc_gather_push(QcPart<T> p, QcGeo<T> g,
                                                        const T *__restrict__ E0,
                                                        const T *__restrict__ E1,
                                                        const T *__restrict__ E2,
                                                        const T *__restrict__ B0,
                                                        const T *__restrict__ B1,
                                                        const T *__restrict__ B2, T h) {
  const int tid = threadIdx.x;
  const int64_t base = int64_t(blockIdx.x) * 256;
  const int here = int(p.n - base < 256 ? p.n - base : 256);
  constexpr bool kSort = !(O == 1 && sizeof(T) == 4);
  int64_t i = base + tid;
  if constexpr (kSort) {
    __shared__ int hist[kQcGatherBins];
    __shared__ int part[256];  // per-thread bin pair sums, then their exclusive scan
    __shared__ int perm[256];
    int key = 0;
    if (tid < here) {
      const T x = p.x[base + tid], y = p.y[base + tid];
      const T rc = sqrt(x * x + y * y) * g.inv_dr;
      key = rc < T(kQcGatherBins - 1) ? int(rc) : kQcGatherBins - 1;
    }
    for (int t = tid; t < kQcGatherBins; t += 256) hist[t] = 0;
    __syncthreads();
    const int within = tid < here ? atomicAdd(&hist[key], 1) : 0;
    __syncthreads();
    // exclusive scan of the 512 bins: thread t owns bins 2t and 2t + 1
    const int h0 = hist[2 * tid], h1 = hist[2 * tid + 1];
    part[tid] = h0 + h1;
    __syncthreads();
    for (int off = 1; off < 256; off *= 2) {
      const int v = tid >= off ? part[tid - off] : 0;
      __syncthreads();
      part[tid] += v;
      __syncthreads();
    }
    const int start0 = part[tid] - (h0 + h1);  // exclusive prefix of bin 2t
    __syncthreads();
    hist[2 * tid] = start0;
    hist[2 * tid + 1] = start0 + h0;
    __syncthreads();
    if (tid < here) perm[hist[key] + within] = tid;
    __syncthreads();
    if (tid < here) i = base + perm[tid];
  }
  if (tid >= here) return;
  T r, c, s;
  qc_angle(p.x[i], p.y[i], r, c, s);
  const QcNodes<T, O> nd = qc_nodes<T, O>(g, r, p.z[i]);
  const T er = qc_gather(g, E0, nd, c, s, true), et = qc_gather(g, E1, nd, c, s, true);
  const T ez = qc_gather(g, E2, nd, c, s, false);
  const T br = qc_gather(g, B0, nd, c, s, true), bt = qc_gather(g, B1, nd, c, s, true);
  const T bz = qc_gather(g, B2, nd, c, s, false);
  const T Ex = er * c - et * s, Ey = er * s + et * c, Ez = ez;
  const T Bx = br * c - bt * s, By = br * s + bt * c, Bz = bz;
  // h = q dt / (2 m c)
  const T mx = p.ux[i] + h * Ex, my = p.uy[i] + h * Ey, mz = p.uz[i] + h * Ez;
  const T ig = T(1) / sqrt(T(1) + mx * mx + my * my + mz * mz);
  const T tx = h * Bx * ig, ty = h * By * ig, tz = h * Bz * ig;
  const T sf = T(2) / (T(1) + tx * tx + ty * ty + tz * tz);
  const T sx = sf * tx, sy = sf * ty, sz = sf * tz;
  const T px = mx + (my * tz - mz * ty), py = my + (mz * tx - mx * tz), pz = mz + (mx * ty - my * tx);
  const T ax = mx + (py * sz - pz * sy), ay = my + (pz * sx - px * sz), az = mz + (px * sy - py * sx);
  p.ux[i] = ax + h * Ex;
  p.uy[i] = ay + h * Ey;
  p.uz[i] = az + h * Ez;
}

// E^ of the initial charge: i k.E = rho^n with no curl, at k = (k_r, 0, k_z)
// through the Cartesian map (E^_x = -i k_r rho / k^2, E^_z = -i k_z rho / k^2;
// G_+ = (i/2) E_x, G_- = -(i/2) E_x, G_z = E_z); the held k_z row is zero.
template <typename T>
__global__ __launch_bounds__(256) void k_qc_electrostatic(Cx<T> *Ep, Cx<T> *Em, Cx<T> *Ez,
                                                          const Cx<T> *__restrict__ rho,
                                                          const T *__restrict__ kr, int nmodes,
                                                          int nz, int nr, T kzfac) {
  const int64_t n = int64_t(nmodes) * nz * nr;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int i = int(idx % nr);
  const int iz = int((idx / nr) % nz);
  const int m = int(idx / (int64_t(nz) * nr));
  // the held k_z row, and the held last k_r column of modes m >= 1 (its
  // charge is held at zero)
  if (iz == nz / 2 || (m >= 1 && i == nr - 1)) {
    Ep[idx] = Em[idx] = Ez[idx] = cx(T(0), T(0));
    return;
  }
  const T k_r = kr[int64_t(m) * nr + i];
  const T k_z = T(iz < nz / 2 ? iz : iz - nz) * kzfac;
  const T k2 = k_r * k_r + k_z * k_z;
  const Cx<T> q = rho[idx];
  // -i k rho / k^2
  const Cx<T> ex = cx(q.im * k_r / k2, -q.re * k_r / k2);
  const Cx<T> ez = cx(q.im * k_z / k2, -q.re * k_z / k2);
  Ep[idx] = T(0.5) * mul_i(ex);
  Em[idx] = T(-0.5) * mul_i(ex);
  Ez[idx] = ez;
}

// ---- host -------------------------------------------------------------------

gp_status qfail(gp_status st, const std::string &msg) {
  set_last_error(msg);
  return st;
}

// J_0 .. J_n at x > 0 (n <= 64), to about 1e-15 absolute.  For x >= 25 and
// x > 2 n: Hankel's asymptotic expansion of J_0 and J_1 (its terms fall
// below 1e-17 long before they start to grow at k ~ 2x), then the upward
// recurrence J_{k+1} = (2k / x) J_k - J_{k-1}, stable while k < x.  Else
// Miller's method: the same recurrence run downward from an order far above
// x and n with an arbitrary start, normalised by J_0 + 2 (J_2 + J_4 + ...)
// = 1.  (The C++ library's cyl_bessel_j loses about 1e-11 relative at
// arguments of several hundred, which the transform matrices of wide grids
// reach.)
void bessel_j_orders(int n, double x, double *J) {
  if (x >= 25.0 && x > 2.0 * n) {
    double P[2], Q[2];
    for (int nu = 0; nu < 2; ++nu) {
      const double mu = 4.0 * nu * nu;
      double term = 1.0, prev = 2.0;
      P[nu] = 1.0;
      Q[nu] = 0.0;
      for (int k = 1; k < 80; ++k) {
        term *= (mu - double(2 * k - 1) * (2 * k - 1)) / (8.0 * k * x);
        if (std::fabs(term) > std::fabs(prev)) break;  // the series turns
        prev = term;
        if (k % 2 == 0)
          P[nu] += (k / 2) % 2 ? -term : term;
        else
          Q[nu] += ((k - 1) / 2) % 2 ? -term : term;
        if (std::fabs(term) < 1e-17) break;
      }
    }
    // chi_0 = x - pi/4, chi_1 = chi_0 - pi/2
    const double c = std::cos(x), s = std::sin(x);
    const double r2 = std::sqrt(0.5);
    const double cq = (c + s) * r2, sq = (s - c) * r2;  // cos, sin of x - pi/4
    const double A = std::sqrt(2.0 / (kPi * x));
    J[0] = A * (P[0] * cq - Q[0] * sq);
    if (n >= 1) J[1] = A * (P[1] * sq + Q[1] * cq);
    for (int k = 1; k < n; ++k) J[k + 1] = (2.0 * k / x) * J[k] - J[k - 1];
    return;
  }
  const int top = 2 * ((std::max(n, int(x)) + 60) / 2);  // even start order
  double fk1 = 0.0, fk = 1e-30, sum = 0.0;
  for (int i = 0; i <= n; ++i) J[i] = 0.0;
  for (int k = top; k >= 1; --k) {
    // fk = f_k, fk1 = f_{k+1}  ->  f_{k-1}
    const double fm = (2.0 * k / x) * fk - fk1;
    if (k <= n) J[k] = fk;
    if (k % 2 == 0) sum += 2.0 * fk;
    fk1 = fk;
    fk = fm;
    if (std::fabs(fk) > 1e250) {  // rescale everything held so far
      fk *= 1e-250;
      fk1 *= 1e-250;
      sum *= 1e-250;
      for (int i = 0; i <= n; ++i) J[i] *= 1e-250;
    }
  }
  J[0] = fk;
  sum += fk;
  for (int i = 0; i <= n; ++i) J[i] /= sum;
}

// J_p for any integer |p| <= 64: J_{-p} = (-1)^p J_p
double bessel_j(int p, double x) {
  double J[66];
  const int a = p < 0 ? -p : p;
  bessel_j_orders(a, x, J);
  return (p < 0 && (a % 2)) ? -J[a] : J[a];
}

// The first n positive zeros of J_m: sign changes on a fine scan from x = m
// (J_m has none below), each refined by bisection to the nearest double.
std::vector<double> bessel_zeros(int m, int n) {
  std::vector<double> z;
  const double h = 0.05;
  double a = std::max(1e-6, double(m));
  double fa = bessel_j(m, a);
  while (int(z.size()) < n) {
    const double b = a + h;
    const double fb = bessel_j(m, b);
    if (fa == 0.0) {
      z.push_back(a);
    } else if ((fa < 0) != (fb < 0)) {
      // bisect down to adjacent doubles, then keep the end with the smaller |J_m|
      double lo = a, hi = b, flo = fa, fhi = fb;
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double fm = bessel_j(m, mid);
        if (fm == 0.0) {
          lo = hi = mid;
          flo = fhi = 0.0;
          break;
        }
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
          fhi = fm;
        }
      }
      z.push_back(std::fabs(flo) <= std::fabs(fhi) ? lo : hi);
    }
    a = b;
    fa = fb;
  }
  return z;
}

// In-place inverse of an n x n row-major matrix (Gauss-Jordan, partial
// pivoting); false if singular.
bool invert(std::vector<double> &a, int n) {
  std::vector<double> inv(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[size_t(r) * n + c]) > std::fabs(a[size_t(piv) * n + c])) piv = r;
    if (a[size_t(piv) * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[size_t(c) * n + k], a[size_t(piv) * n + k]);
        std::swap(inv[size_t(c) * n + k], inv[size_t(piv) * n + k]);
      }
    const double d = 1.0 / a[size_t(c) * n + c];
    for (int k = 0; k < n; ++k) {
      a[size_t(c) * n + k] *= d;
      inv[size_t(c) * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[size_t(r) * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[size_t(r) * n + k] -= f * a[size_t(c) * n + k];
        inv[size_t(r) * n + k] -= f * inv[size_t(c) * n + k];
      }
    }
  }
  a.swap(inv);
  return true;
}

// k_i = alpha_{m,i} / R, R = nr dr: mode m's spectral grid
std::vector<double> spectral_kr(int m, int nr, double dr) {
  std::vector<double> k = bessel_zeros(m, nr);
  for (double &v : k) v /= nr * dr;
  return k;
}

// The backward matrix of Hankel order p on mode m's grid k: M[j][i] =
// J_p(k_i r_j) (row-major nr x nr, r_j = (j + 1/2) dr).  For p = m - 1,
// m >= 1, the last column is (r_j / R)^{m-1}: on the zeros of J_m the
// functions J_{m-1}(k_i r) form a Dini series (x J'_{m-1} = (m-1) J_{m-1}
// there) that is complete only with that k_r = 0 eigenfunction; it takes
// the place of the last J_{m-1}, whose column of the other orders is held.
std::vector<double> backward_hankel(int p, int m, const std::vector<double> &k, int nr,
                                    double dr) {
  std::vector<double> M(size_t(nr) * nr);
  for (int j = 0; j < nr; ++j)
    for (int i = 0; i < nr; ++i) M[size_t(j) * nr + i] = bessel_j(p, k[i] * (j + 0.5) * dr);
  if (m >= 1 && p == m - 1)
    for (int j = 0; j < nr; ++j)
      M[size_t(j) * nr + nr - 1] = std::pow((j + 0.5) / nr, double(m - 1));
  return M;
}

}  // namespace
}  // namespace galpic

using namespace galpic;

enum {
  kQReal = 10,  // E_r E_t E_z B_r B_t B_z J_r J_t J_z rho
  kQSpec = 11,  // E_+ E_- E_z B_+ B_- B_z J_+ J_- J_z rho (two buffers)
  kQScr = 6
};

struct gp_qc_ctx {
  gp_qc_desc d{};
  size_t real_size = 8;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void *> allocs;
  void *real[kQReal] = {};
  void *spec[kQSpec] = {};
  void *scr[kQScr] = {};
  void *coef[6] = {};
  double *kr_d = nullptr;  // [mode][k_r], double
  void *kr_t = nullptr;    // the same in the real type
  void *fmat = nullptr, *bmat = nullptr;
  void *tw = nullptr;
  void *tab = nullptr;     // device tables (FieldSet, QcSet)
  int rho_old = 9;         // spec slot of rho^n (the other holds rho^{n+1})
  double vgal = 0.0;
  bool coef_ready = false;
  bool timing = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;  // events of timed launches, until gp_qc_stage_times
  // particles (caller-owned device arrays of the real type) and sources
  gp_qc_particles part{};
  bool bound = false;
  void *bg[4] = {};        // background rho, J_r, J_theta, J_z (allocated once)
  bool has_bg = false;
  void *inv_vol = nullptr; // [nr] 1 / V_j in the real type
  int dep_per = 0;         // deposit particles per thread (0: not chosen yet)
  int order = 1;           // particle shape: 1 linear, 3 cubic
  // re-sort along z (k_qcz_*): control words (count, decision, nz counts,
  // nz offsets), staging for the six particle arrays, its capacity in
  // particles, and the threshold divisor (0: never)
  int *zs_ctl = nullptr;
  void *zs_tmp = nullptr;
  int64_t zs_cap = 0;
  int resort_div = 0;
  int64_t zs_steps = 0;  // particle steps since binding
};

namespace {

// device table layout (byte offsets)
enum { kFsFwdEB = 0, kFsFwdSrc, kFsInvEB, kNFs };
enum { kQsEB = 0, kQsJ = 2, kQsRho0 = 3, kQsRho1 = 4, kQsBwdEB = 5, kNQs = 7 };

size_t field_bytes(const gp_qc_ctx *c) {
  return size_t(c->d.nmodes) * c->d.nz * c->d.nr * 2 * c->real_size;
}

gp_status qalloc(gp_qc_ctx *c, size_t bytes, void **out) {
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    return qfail(GP_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->allocs.push_back(p);
  *out = p;
  return GP_OK;
}

#define QTRY(expr)                \
  do {                            \
    gp_status st_ = (expr);       \
    if (st_ != GP_OK) return st_; \
  } while (0)

gp_status qcheck(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return qfail(GP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return GP_OK;
}

// Device events around one launch when timing is on (stages as in the header:
// 0 z forward, 1 Hankel forward, 2 update, 3 Hankel backward, 4 z inverse).
struct QStamp {
  gp_qc_ctx *c;
  gp_qc_ctx::Rec rec{};
  bool on;
  QStamp(gp_qc_ctx *ctx, int stage) : c(ctx), on(ctx->timing) {
    if (!on) return;
    rec.stage = stage;
    if (hipEventCreate(&rec.a) != hipSuccess) {
      on = false;
      return;
    }
    if (hipEventCreate(&rec.b) != hipSuccess) {
      (void)hipEventDestroy(rec.a);
      on = false;
      return;
    }
    (void)hipEventRecord(rec.a, c->stream);
  }
  ~QStamp() {
    if (!on) return;
    (void)hipEventRecord(rec.b, c->stream);
    c->recs.push_back(rec);
  }
};

template <typename T>
const FieldSet *fs_at(gp_qc_ctx *c, int k) {
  return reinterpret_cast<const FieldSet *>(c->tab) + k;
}
template <typename T>
const QcSet *qs_at(gp_qc_ctx *c, int k) {
  return reinterpret_cast<const QcSet *>(static_cast<char *>(c->tab) + kNFs * sizeof(FieldSet)) +
         k;
}

template <typename T>
void z_transform(gp_qc_ctx *c, int fs, int nf, bool inverse) {
  int lz = 0;
  while ((1 << lz) < c->d.nz) ++lz;
  QStamp stamp(c, inverse ? 4 : 0);
  launch_c2c_lines<T>(fs_at<T>(c, fs), 1, nf, lz, c->d.nr, c->d.nr,
                      int64_t(c->d.nz) * c->d.nr, c->d.nmodes, inverse,
                      static_cast<const Cx<T> *>(c->tw), c->stream);
}

// The wide form (two row tiles per wave, no K split) halves the matrix
// operand traffic per flop but has an eighth of the workgroups; it is taken
// when it still gives 4 waves per SIMD (8192 narrow workgroups).  Measured on
// 1024 x 512 x 2 modes: f64 backward 383 -> 300 us, f32 unchanged; with
// only 2 waves per SIMD (the one-set forward launch) it was slower.
constexpr int64_t kWideMin = 8192;

template <typename T, int KIND>
void hankel(gp_qc_ctx *c, int qs, int nsets, const void *mats) {
  const int nparts = KIND == kScalarFwd ? 1 : 2;
  const unsigned cols = unsigned((c->d.nr + 16 * kTC - 1) / (16 * kTC));
  const unsigned zdim = unsigned(nsets * c->d.nmodes * nparts);
  const int64_t narrow = int64_t(c->d.nz / 8) * cols * zdim;
  QStamp stamp(c, KIND == kVecBwd ? 3 : 1);
  if (c->d.nz % 64 == 0 && narrow >= kWideMin) {
    hipLaunchKernelGGL((k_qc_hankel<T, KIND, true>), dim3(unsigned(c->d.nz / 64), cols, zdim),
                       dim3(64 * kQWaves), 0, c->stream, qs_at<T>(c, qs),
                       static_cast<const T *>(mats), c->d.nz, c->d.nr, c->d.nmodes, nparts);
  } else {
    hipLaunchKernelGGL((k_qc_hankel<T, KIND, false>), dim3(unsigned(c->d.nz / 8), cols, zdim),
                       dim3(64 * kQWaves), 0, c->stream, qs_at<T>(c, qs),
                       static_cast<const T *>(mats), c->d.nz, c->d.nr, c->d.nmodes, nparts);
  }
}

template <typename T>
void enqueue_sources_fwd(gp_qc_ctx *c) {
  z_transform<T>(c, kFsFwdSrc, 4, false);
  hankel<T, kVecFwd>(c, kQsJ, 1, c->fmat);
  hankel<T, kScalarFwd>(c, c->rho_old == 9 ? kQsRho1 : kQsRho0, 1, c->fmat);
}

template <typename T>
void enqueue_update(gp_qc_ctx *c) {
  QcUpd<T> p;
  for (int a = 0; a < 3; ++a) {
    p.E[a] = static_cast<Cx<T> *>(c->spec[a]);
    p.B[a] = static_cast<Cx<T> *>(c->spec[3 + a]);
    p.J[a] = static_cast<const Cx<T> *>(c->spec[6 + a]);
  }
  p.rho_old = static_cast<const Cx<T> *>(c->spec[c->rho_old]);
  p.rho_new = static_cast<const Cx<T> *>(c->spec[c->rho_old == 9 ? 10 : 9]);
  for (int k = 0; k < 6; ++k) p.coef[k] = static_cast<const Cx<T> *>(c->coef[k]);
  p.kr = static_cast<const T *>(c->kr_t);
  const int64_t n = int64_t(c->d.nmodes) * c->d.nz * c->d.nr;
  QStamp stamp(c, 2);
  hipLaunchKernelGGL((k_qc_update<T>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, c->stream,
                     p, c->d.nmodes, c->d.nz, c->d.nr, T(2.0 * kPi / (c->d.nz * c->d.dz)));
  c->rho_old = c->rho_old == 9 ? 10 : 9;
}

template <typename T>
void enqueue_fields_inv(gp_qc_ctx *c) {
  hankel<T, kVecBwd>(c, kQsBwdEB, 2, c->bmat);
  z_transform<T>(c, kFsInvEB, 6, true);
}

template <typename T>
void enqueue_fields_fwd(gp_qc_ctx *c) {
  z_transform<T>(c, kFsFwdEB, 6, false);
  hankel<T, kVecFwd>(c, kQsEB, 2, c->fmat);
}

template <typename F>
gp_status qdispatch(gp_qc_ctx *c, F &&f) {
  if (c->d.precision == GP_FP64)
    f(double{});
  else
    f(float{});
  return qcheck("kernel launch");
}

gp_status qcheck_ctx(gp_qc_ctx *c) {
  if (!c) return qfail(GP_ERR_ARG, "context is NULL");
  return GP_OK;
}

// transform matrices (transposed, real type) and k_r of every mode
template <typename T>
gp_status build_transforms(gp_qc_ctx *c) {
  const int nr = c->d.nr, nm = c->d.nmodes;
  const size_t mat = size_t(nr) * nr;
  std::vector<T> fh(size_t(nm) * 3 * mat), bh(size_t(nm) * 3 * mat), kt(size_t(nm) * nr);
  std::vector<double> kd(size_t(nm) * nr);
  for (int m = 0; m < nm; ++m) {
    const std::vector<double> k = spectral_kr(m, nr, c->d.dr);
    // k_r of the update and the coefficients: the zeros, with 0 in the last
    // column of modes m >= 1 (G_-'s k_r = 0 function; the others held)
    for (int i = 0; i < nr; ++i) {
      const double ku = (m >= 1 && i == nr - 1) ? 0.0 : k[i];
      kd[size_t(m) * nr + i] = ku;
      kt[size_t(m) * nr + i] = T(ku);
    }
    for (int slot = 0; slot < 3; ++slot) {
      const int p = m - 1 + slot;
      const std::vector<double> M = backward_hankel(p, m, k, nr, c->d.dr);
      std::vector<double> Minv = M;
      if (!invert(Minv, nr))
        return qfail(GP_ERR_ARG, "the Hankel matrix of order " + std::to_string(p) +
                                     " is singular for this nr");
      T *F = fh.data() + (size_t(m) * 3 + slot) * mat;
      T *Bk = bh.data() + (size_t(m) * 3 + slot) * mat;
      // forward A = Minv (spectral i <- radial j): AT[j][i] = Minv[i][j]
      // backward A = M / nz (radial j <- spectral i): AT[i][j] = M[j][i] / nz
      for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nr; ++i) {
          F[size_t(j) * nr + i] = T(Minv[size_t(i) * nr + j]);
          Bk[size_t(i) * nr + j] = T(M[size_t(j) * nr + i] / c->d.nz);
        }
    }
  }
  const size_t mbytes = fh.size() * sizeof(T);
  QTRY(qalloc(c, mbytes, &c->fmat));
  QTRY(qalloc(c, mbytes, &c->bmat));
  void *p = nullptr;
  QTRY(qalloc(c, kd.size() * sizeof(double), &p));
  c->kr_d = static_cast<double *>(p);
  QTRY(qalloc(c, kt.size() * sizeof(T), &c->kr_t));
  // 1 / V_j, V_j = 2 pi dz times the integral of node j's folded weight
  // against r dr: dr^2 (j + 1/2) where the shape's support stays off the
  // axis; (13/24) dr^2 for the linear axis node; for cubic shapes the axis
  // nodes 0 and 1 are integrated exactly (the folded weight times r is a
  // polynomial between the breakpoints (n + 1/2) dr: 4-point Gauss-Legendre
  // per piece)
  std::vector<T> iv(nr);
  const double dr2 = c->d.dr * c->d.dr;
  for (int j = 0; j < nr; ++j) {
    double v = (j + 0.5) * dr2;
    if (c->order == 1 && j == 0) v = 13.0 / 24.0 * dr2;
    if (c->order == 3 && j < 2) {
      auto cubic = [](double x) {  // the centred cubic B-spline
        const double a = std::fabs(x);
        return a < 1.0 ? (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0
                       : (a < 2.0 ? (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0 : 0.0);
      };
      // nodes and weights of 4-point Gauss-Legendre on [-1, 1]
      const double gx[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563,
                            0.8611363115940526};
      const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461,
                            0.3478548451374538};
      double acc = 0.0;  // in units of dr: int_0^{j+2.5} w(u) u du
      for (int piece = 0; piece <= j + 2; ++piece) {
        const double a = piece == 0 ? 0.0 : piece - 0.5, b = piece + 0.5;
        for (int q = 0; q < 4; ++q) {
          const double u = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
          const double w = cubic(u - (j + 0.5)) + cubic(u + (j + 0.5));  // node + mirror
          acc += 0.5 * (b - a) * gw[q] * w * u;
        }
      }
      v = acc * dr2;
    }
    iv[j] = T(1.0 / (2.0 * kPi * c->d.dz * v));
  }
  QTRY(qalloc(c, iv.size() * sizeof(T), &c->inv_vol));
  if (hipMemcpyAsync(c->inv_vol, iv.data(), iv.size() * sizeof(T), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "volume upload failed");
  if (hipMemcpyAsync(c->fmat, fh.data(), mbytes, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->bmat, bh.data(), mbytes, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->kr_d, kd.data(), kd.size() * sizeof(double), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(c->kr_t, kt.data(), kt.size() * sizeof(T), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "transform upload failed");
  return GP_OK;
}

gp_status build_tables(gp_qc_ctx *c) {
  std::vector<unsigned char> host(kNFs * sizeof(FieldSet) + kNQs * sizeof(QcSet), 0);
  FieldSet *fs = reinterpret_cast<FieldSet *>(host.data());
  QcSet *qs = reinterpret_cast<QcSet *>(host.data() + kNFs * sizeof(FieldSet));
  for (int f = 0; f < 6; ++f) {
    fs[kFsFwdEB].in[f] = c->real[f];
    fs[kFsFwdEB].out[f] = c->scr[f];
    fs[kFsInvEB].in[f] = c->scr[f];
    fs[kFsInvEB].out[f] = c->real[f];
  }
  for (int f = 0; f < 4; ++f) {
    fs[kFsFwdSrc].in[f] = c->real[6 + f];
    fs[kFsFwdSrc].out[f] = c->scr[f];
  }
  for (int v = 0; v < 2; ++v)
    for (int a = 0; a < 3; ++a) {
      qs[kQsEB + v].in[a] = c->scr[3 * v + a];
      qs[kQsEB + v].out[a] = c->spec[3 * v + a];
      qs[kQsBwdEB + v].in[a] = c->spec[3 * v + a];
      qs[kQsBwdEB + v].out[a] = c->scr[3 * v + a];
    }
  for (int a = 0; a < 3; ++a) {
    qs[kQsJ].in[a] = c->scr[a];
    qs[kQsJ].out[a] = c->spec[6 + a];
  }
  // rho^{n+1} into slot 9 (parity 0) or 10 (parity 1)
  qs[kQsRho0].in[0] = c->scr[3];
  qs[kQsRho0].out[0] = c->spec[9];
  qs[kQsRho1].in[0] = c->scr[3];
  qs[kQsRho1].out[0] = c->spec[10];
  QTRY(qalloc(c, host.size(), &c->tab));
  if (hipMemcpyAsync(c->tab, host.data(), host.size(), hipMemcpyHostToDevice, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "table upload failed");
  return GP_OK;
}

// which -> buffer
void *slot_of(gp_qc_ctx *c, int which) {
  if (which >= GP_QC_ER && which <= GP_QC_RHO) return c->real[which - GP_QC_ER];
  if (which >= GP_QC_E_PLUS && which <= GP_QC_J_Z_HAT) return c->spec[which - GP_QC_E_PLUS];
  if (which == GP_QC_RHO_HAT_OLD) return c->spec[c->rho_old];
  if (which == GP_QC_RHO_HAT_NEW) return c->spec[c->rho_old == 9 ? 10 : 9];
  if (which >= GP_QC_COEF0 && which <= GP_QC_COEF5) return c->coef[which - GP_QC_COEF0];
  return nullptr;
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

template <typename T>
QcGeo<T> qc_geo(gp_qc_ctx *c) {
  QcGeo<T> g;
  g.nmodes = c->d.nmodes;
  g.nz = c->d.nz;
  g.nr = c->d.nr;
  g.inv_dz = T(1.0 / c->d.dz);
  g.inv_dr = T(1.0 / c->d.dr);
  g.lz = T(c->d.nz * c->d.dz);
  g.inv_vol = static_cast<const T *>(c->inv_vol);
  return g;
}

template <typename T>
QcPart<T> qc_part(gp_qc_ctx *c) {
  QcPart<T> q;
  q.x = static_cast<T *>(c->part.x);
  q.y = static_cast<T *>(c->part.y);
  q.z = static_cast<T *>(c->part.z);
  q.ux = static_cast<T *>(c->part.ux);
  q.uy = static_cast<T *>(c->part.uy);
  q.uz = static_cast<T *>(c->part.uz);
  q.n = c->part.n;
  return q;
}

// the real-space sources start each deposit as the background (or zero),
// in one launch
gp_status fill_sources(gp_qc_ctx *c) {
  return qdispatch(c, [&](auto t) {
    using T = decltype(t);
    QcSrc<T> dst, bg;
    dst.rho = static_cast<T *>(c->real[9]);
    dst.jr = static_cast<T *>(c->real[6]);
    dst.jt = static_cast<T *>(c->real[7]);
    dst.jz = static_cast<T *>(c->real[8]);
    // without a background the kernel never reads these
    bg.rho = static_cast<T *>(c->has_bg ? c->bg[0] : c->real[9]);
    bg.jr = static_cast<T *>(c->has_bg ? c->bg[1] : c->real[6]);
    bg.jt = static_cast<T *>(c->has_bg ? c->bg[2] : c->real[7]);
    bg.jz = static_cast<T *>(c->has_bg ? c->bg[3] : c->real[8]);
    const int64_t n = int64_t(c->d.nmodes) * c->d.nz * c->d.nr * 2;  // real values per array
    hipLaunchKernelGGL((k_qc_reset_sources<T>), dim3(unsigned((4 * n + 255) / 256)), dim3(256), 0,
                       c->stream, dst, bg, c->has_bg ? 1 : 0, n);
  });
}

// Reorder the particles along z (stable, in the caller's arrays), so that
// the deposit's chunks of consecutive particles cover few z planes.  On the
// host, at binding only.
template <typename T>
gp_status sort_particles_by_z(gp_qc_ctx *c) {
  const int64_t n = c->part.n;
  if (n < 2) return GP_OK;
  void *dev[6] = {c->part.x, c->part.y, c->part.z, c->part.ux, c->part.uy, c->part.uz};
  std::vector<std::vector<T>> h(6, std::vector<T>(static_cast<size_t>(n)));
  for (int a = 0; a < 6; ++a)
    if (hipMemcpyAsync(h[a].data(), dev[a], size_t(n) * sizeof(T), hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
      return qfail(GP_ERR_HIP, "particle download failed");
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "stream synchronize failed");
  std::vector<int64_t> idx(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) idx[size_t(i)] = i;
  const std::vector<T> &z = h[2];
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int64_t a, int64_t b) { return z[size_t(a)] < z[size_t(b)]; });
  std::vector<T> tmp(static_cast<size_t>(n));
  for (int a = 0; a < 6; ++a) {
    for (int64_t i = 0; i < n; ++i) tmp[size_t(i)] = h[a][size_t(idx[size_t(i)])];
    h[a].swap(tmp);
    if (hipMemcpyAsync(dev[a], h[a].data(), size_t(n) * sizeof(T), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess)
      return qfail(GP_ERR_HIP, "particle upload failed");
    if (hipStreamSynchronize(c->stream) != hipSuccess)  // before tmp is reused
      return qfail(GP_ERR_HIP, "stream synchronize failed");
  }
  return GP_OK;
}

// Windows above this take the plain kernel (gfx950 allows 160 KiB of LDS
// per workgroup; the attribute below lifts the 64 KiB default).
constexpr size_t kQcMaxWindow = 128 * 1024;

template <typename T, int O>
void launch_move_deposit_o(gp_qc_ctx *c, const QcSrc<T> &src, int move) {
  const size_t lds = size_t(4) * c->d.nmodes * qc_win<O>() * c->d.nr * 2 * sizeof(double);
  if (lds <= kQcMaxWindow) {
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_qc_move_deposit_tiled<T, O>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(kQcMaxWindow));
      attr_set = true;
    }
    if (c->dep_per == 0) {
      // particles per thread: the fewest of 2..4 whose workgroups fill the
      // device's resident slots (CUs x workgroups per CU) with the least
      // tail, i.e. the smallest ceil(workgroups / slots) x per
      int cus = 0, per_cu = 0;
      int dev = 0;
      (void)hipGetDevice(&dev);
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &per_cu, reinterpret_cast<const void *>(&k_qc_move_deposit_tiled<T, O>),
              kQcDepThreads, lds) != hipSuccess)
        per_cu = 0;
      (void)hipGetLastError();
      c->dep_per = 2;
      const int64_t slots = int64_t(cus) * per_cu;
      if (slots > 0) {
        int64_t best = -1;
        for (int per = 2; per <= 4; ++per) {
          const int64_t wgs = (c->part.n + int64_t(kQcDepThreads) * per - 1) /
                              (int64_t(kQcDepThreads) * per);
          const int64_t cost = (wgs + slots - 1) / slots * per;
          if (best < 0 || cost < best) {
            best = cost;
            c->dep_per = per;
          }
        }
      }
    }
    const int64_t chunk = int64_t(kQcDepThreads) * c->dep_per;
    hipLaunchKernelGGL((k_qc_move_deposit_tiled<T, O>),
                       dim3(unsigned((c->part.n + chunk - 1) / chunk)), dim3(kQcDepThreads), lds,
                       c->stream, qc_part<T>(c), qc_geo<T>(c), src, T(c->d.dt), T(c->vgal),
                       T(c->part.q * c->part.w), move, c->dep_per, c->zs_ctl);
  } else {
    hipLaunchKernelGGL((k_qc_move_deposit<T, O>), dim3(unsigned((c->part.n + 255) / 256)),
                       dim3(256), 0, c->stream, qc_part<T>(c), qc_geo<T>(c), src, T(c->d.dt),
                       T(c->vgal), T(c->part.q * c->part.w), move);
  }
}

// The re-sort along z, when the count of the deposits since the last
// decision calls for it (the kernels return at once otherwise).
template <typename T>
void launch_zsort(gp_qc_ctx *c) {
  if (c->part.n < 2 || !c->zs_ctl || !c->zs_tmp) return;
  const int64_t chunk = int64_t(kQcSortThreads) * kQcSortPer;
  const unsigned blocks = unsigned((c->part.n + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_qcz_decide, dim3(1), dim3(1), 0, c->stream, c->zs_ctl, c->part.n,
                     c->resort_div);
  hipLaunchKernelGGL((k_qcz_count<T>), dim3(blocks), dim3(kQcSortThreads), 0, c->stream,
                     qc_part<T>(c), qc_geo<T>(c), c->zs_ctl);
  hipLaunchKernelGGL(k_qcz_scan, dim3(1), dim3(kQcMaxNz), 0, c->stream, c->zs_ctl, c->d.nz);
  hipLaunchKernelGGL((k_qcz_scatter<T>), dim3(blocks), dim3(kQcSortThreads), 0, c->stream,
                     qc_part<T>(c), qc_geo<T>(c), c->zs_ctl, static_cast<T *>(c->zs_tmp));
  hipLaunchKernelGGL((k_qcz_copyback<T>), dim3(std::min(blocks * kQcSortPer, 4096u)), dim3(256),
                     0, c->stream, qc_part<T>(c), c->zs_ctl,
                     static_cast<const T *>(c->zs_tmp));
}

template <typename T>
void launch_move_deposit(gp_qc_ctx *c, int move) {
  if (c->part.n == 0) return;
  QcSrc<T> src;
  src.jr = static_cast<T *>(c->real[6]);
  src.jt = static_cast<T *>(c->real[7]);
  src.jz = static_cast<T *>(c->real[8]);
  src.rho = static_cast<T *>(c->real[9]);
  QStamp stamp(c, 5);
  // the decision every kQcResortEvery steps (its five launches cost more
  // than the check saves when taken every step; the order decays over
  // hundreds of steps)
  if (move && c->resort_div > 0 && ++c->zs_steps % kQcResortEvery == 0) launch_zsort<T>(c);
  if (c->order == 3)
    launch_move_deposit_o<T, 3>(c, src, move);
  else
    launch_move_deposit_o<T, 1>(c, src, move);
}

template <typename T>
void launch_gather_push(gp_qc_ctx *c) {
  if (c->part.n == 0) return;
  const T h = T(c->part.q * c->d.dt / (2.0 * c->part.m));
  QStamp stamp(c, 6);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(unsigned((c->part.n + 255) / 256)), dim3(256), 0, c->stream,
                       qc_part<T>(c), qc_geo<T>(c), static_cast<const T *>(c->real[0]),
                       static_cast<const T *>(c->real[1]), static_cast<const T *>(c->real[2]),
                       static_cast<const T *>(c->real[3]), static_cast<const T *>(c->real[4]),
                       static_cast<const T *>(c->real[5]), h);
  };
  if (c->order == 3)
    go(k_qc_gather_push<T, 3>);
  else
    go(k_qc_gather_push<T, 1>);
}

}  // namespace

gp_status gp_qc_init(const gp_qc_desc *d, void *hip_stream, gp_qc_ctx **out) {
  if (!d || !out) return qfail(GP_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (!is_pow2(d->nz) || d->nz < 8 || d->nz > 1024)
    return qfail(GP_ERR_ARG, "nz must be a power of two in [8, 1024]");
  if (d->nr < 4 || d->nr > 512)
    return qfail(GP_ERR_ARG, "nr must lie in [4, 512]");
  if (d->nmodes < 1 || d->nmodes > 8) return qfail(GP_ERR_ARG, "nmodes must lie in [1, 8]");
  if (!(d->dz > 0) || !(d->dr > 0) || !(d->dt > 0) || !std::isfinite(d->dz) ||
      !std::isfinite(d->dr) || !std::isfinite(d->dt))
    return qfail(GP_ERR_ARG, "dz, dr, dt must be positive and finite");
  if (d->precision != GP_FP64 && d->precision != GP_MIXED)
    return qfail(GP_ERR_ARG, "precision must be GP_FP64 or GP_MIXED");
  if (d->shape_order != 0 && d->shape_order != 1 && d->shape_order != 3)
    return qfail(GP_ERR_ARG, "shape_order must be 0 or 1 (linear) or 3 (cubic)");
  gp_qc_ctx *c = new gp_qc_ctx();
  c->d = *d;
  c->order = d->shape_order == 3 ? 3 : 1;
  c->real_size = d->precision == GP_FP64 ? 8 : 4;
  auto bail = [&](gp_status st) {
    std::string keep = gp_last_error();
    gp_qc_destroy(c);
    set_last_error(keep);
    return st;
  };
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess)
      return bail(qfail(GP_ERR_HIP, "hipStreamCreate failed"));
    c->own_stream = true;
  }
  const size_t fb = field_bytes(c);
  for (auto &p : c->real) {
    gp_status st = qalloc(c, fb, &p);
    if (st) return bail(st);
    if (hipMemsetAsync(p, 0, fb, c->stream) != hipSuccess)
      return bail(qfail(GP_ERR_HIP, "clear failed"));
  }
  for (auto &p : c->spec) {
    gp_status st = qalloc(c, fb, &p);
    if (st) return bail(st);
    if (hipMemsetAsync(p, 0, fb, c->stream) != hipSuccess)
      return bail(qfail(GP_ERR_HIP, "clear failed"));
  }
  for (auto &p : c->scr) {
    gp_status st = qalloc(c, fb, &p);
    if (st) return bail(st);
  }
  for (auto &p : c->coef) {
    gp_status st = qalloc(c, fb, &p);
    if (st) return bail(st);
  }
  {
    const size_t twb = 1024 * 2 * c->real_size;
    gp_status st = qalloc(c, twb, &c->tw);
    if (st) return bail(st);
    std::vector<char> host(twb);
    if (d->precision == GP_FP64)
      fill_twiddles<double>(reinterpret_cast<Cx<double> *>(host.data()));
    else
      fill_twiddles<float>(reinterpret_cast<Cx<float> *>(host.data()));
    if (hipMemcpyAsync(c->tw, host.data(), twb, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return bail(qfail(GP_ERR_HIP, "twiddle upload failed"));
  }
  gp_status st = d->precision == GP_FP64 ? build_transforms<double>(c)
                                         : build_transforms<float>(c);
  if (st) return bail(st);
  st = build_tables(c);
  if (st) return bail(st);
  st = gp_qc_set_v_gal(c, 0.0);
  if (st) return bail(st);
  *out = c;
  return GP_OK;
}

gp_status gp_qc_set_v_gal(gp_qc_ctx *c, double vz) {
  QTRY(qcheck_ctx(c));
  if (!std::isfinite(vz) || std::fabs(vz) >= 1.0)
    return qfail(GP_ERR_ARG, "|v_gal| must be finite and below c");
  // largest |k_z v_gal| dt over the non-Nyquist planes
  const double kzmax = 2.0 * kPi * double(c->d.nz / 2 - 1) / (c->d.nz * c->d.dz);
  if (std::fabs(vz) * kzmax * c->d.dt >= 2.0 * kPi * (1.0 - 1e-6))
    return qfail(GP_ERR_UNSTABLE, "some mode has |k_z v_gal| dt >= 2 pi");
  c->vgal = vz;
  // per mode: the Cartesian coefficient kernel with k_z on its "y" axis and
  // this mode's k_r on its "z" axis (v_gal along "y")
  std::vector<double> kt(1 + c->d.nz + c->d.nr);
  kt[0] = 0.0;
  for (int i = 0; i < c->d.nz; ++i) {
    const int s = i < c->d.nz / 2 ? i : i - c->d.nz;
    kt[1 + i] = 2.0 * kPi * double(s) / (c->d.nz * c->d.dz);
  }
  void *ktab = nullptr;
  QTRY(qalloc(c, kt.size() * sizeof(double) * c->d.nmodes, &ktab));
  std::vector<double> all(kt.size() * c->d.nmodes);
  std::vector<double> krh(size_t(c->d.nmodes) * c->d.nr);
  if (hipMemcpy(krh.data(), c->kr_d, krh.size() * sizeof(double), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return qfail(GP_ERR_HIP, "k_r download failed");
  for (int m = 0; m < c->d.nmodes; ++m) {
    std::copy(kt.begin(), kt.end(), all.begin() + m * kt.size());
    for (int i = 0; i < c->d.nr; ++i)
      all[m * kt.size() + 1 + c->d.nz + i] = krh[size_t(m) * c->d.nr + i];
  }
  if (hipMemcpyAsync(ktab, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "k table upload failed");
  const int64_t per = int64_t(c->d.nz) * c->d.nr;
  for (int m = 0; m < c->d.nmodes; ++m) {
    RunGeom g{};
    g.nx = 1;
    g.ny = c->d.nz;
    g.nz = 2 * (c->d.nr - 1);  // unused by the kernel beyond nzh
    g.nzh = c->d.nr;
    g.dt = c->d.dt;
    g.vgal[0] = 0.0;
    g.vgal[1] = vz;
    g.vgal[2] = 0.0;
    g.nmode = per;
    CoefPtrs cp;
    for (int k = 0; k < 6; ++k)
      cp.c[k] = static_cast<char *>(c->coef[k]) + size_t(m) * per * 2 * c->real_size;
    const double *kd = static_cast<const double *>(ktab) + m * kt.size();
    if (c->d.precision == GP_FP64)
      launch_coefficients<double>(g, kd, cp, c->stream);
    else
      launch_coefficients<float>(g, kd, cp, c->stream);
  }
  QTRY(qcheck("coefficients"));
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "stream synchronize failed");
  // the k table is not needed after the coefficients
  (void)hipFree(ktab);
  c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), ktab), c->allocs.end());
  c->coef_ready = true;
  return GP_OK;
}

gp_status gp_qc_write(gp_qc_ctx *c, int which, const void *src) {
  QTRY(qcheck_ctx(c));
  void *dst = slot_of(c, which);
  if (!dst || which >= GP_QC_COEF0) return qfail(GP_ERR_ARG, "bad field selector");
  if (!src) return qfail(GP_ERR_ARG, "source is NULL");
  if (hipMemcpyAsync(dst, src, field_bytes(c), hipMemcpyDefault, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "write failed");
  return GP_OK;
}

gp_status gp_qc_read(gp_qc_ctx *c, int which, void *dst) {
  QTRY(qcheck_ctx(c));
  void *src = slot_of(c, which);
  if (!src) return qfail(GP_ERR_ARG, "bad field selector");
  if (!dst) return qfail(GP_ERR_ARG, "destination is NULL");
  if (hipMemcpyAsync(dst, src, field_bytes(c), hipMemcpyDefault, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "read failed");
  return GP_OK;
}

gp_status gp_qc_fields_fwd(gp_qc_ctx *c) {
  QTRY(qcheck_ctx(c));
  return qdispatch(c, [&](auto t) { enqueue_fields_fwd<decltype(t)>(c); });
}

gp_status gp_qc_sources_fwd(gp_qc_ctx *c) {
  QTRY(qcheck_ctx(c));
  return qdispatch(c, [&](auto t) { enqueue_sources_fwd<decltype(t)>(c); });
}

gp_status gp_qc_init_rho(gp_qc_ctx *c) {
  QTRY(qcheck_ctx(c));
  // transform rho into rho^{n+1}, then make it rho^n
  QTRY(qdispatch(c, [&](auto t) {
    using T = decltype(t);
    z_transform<T>(c, kFsFwdSrc, 4, false);
    hankel<T, kScalarFwd>(c, c->rho_old == 9 ? kQsRho1 : kQsRho0, 1, c->fmat);
  }));
  c->rho_old = c->rho_old == 9 ? 10 : 9;
  return GP_OK;
}

gp_status gp_qc_update(gp_qc_ctx *c) {
  QTRY(qcheck_ctx(c));
  return qdispatch(c, [&](auto t) { enqueue_update<decltype(t)>(c); });
}

gp_status gp_qc_fields_inv(gp_qc_ctx *c) {
  QTRY(qcheck_ctx(c));
  return qdispatch(c, [&](auto t) { enqueue_fields_inv<decltype(t)>(c); });
}

gp_status gp_qc_step(gp_qc_ctx *c, int nsteps) {
  QTRY(qcheck_ctx(c));
  if (nsteps < 0) return qfail(GP_ERR_ARG, "nsteps must be >= 0");
  return qdispatch(c, [&](auto t) {
    using T = decltype(t);
    for (int s = 0; s < nsteps; ++s) {
      enqueue_sources_fwd<T>(c);
      enqueue_update<T>(c);
      enqueue_fields_inv<T>(c);
    }
  });
}

gp_status gp_qc_synchronize(gp_qc_ctx *c) {
  QTRY(qcheck_ctx(c));
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "stream synchronize failed");
  return GP_OK;
}

gp_status gp_qc_set_background(gp_qc_ctx *c, const void *rho, const void *jr, const void *jt,
                               const void *jz) {
  QTRY(qcheck_ctx(c));
  const void *src[4] = {rho, jr, jt, jz};
  if (!rho && !jr && !jt && !jz) {
    c->has_bg = false;  // the arrays stay allocated for a later call
    return GP_OK;
  }
  const size_t fb = field_bytes(c);
  for (int a = 0; a < 4; ++a)
    if (!c->bg[a]) QTRY(qalloc(c, fb, &c->bg[a]));
  for (int a = 0; a < 4; ++a) {
    const hipError_t e = src[a] ? hipMemcpyAsync(c->bg[a], src[a], fb, hipMemcpyDefault, c->stream)
                                : hipMemsetAsync(c->bg[a], 0, fb, c->stream);
    if (e != hipSuccess) return qfail(GP_ERR_HIP, "background upload failed");
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "stream synchronize failed");
  c->has_bg = true;
  return GP_OK;
}

gp_status gp_qc_bind_particles(gp_qc_ctx *c, const gp_qc_particles *p) {
  QTRY(qcheck_ctx(c));
  if (!p) return qfail(GP_ERR_ARG, "particles are NULL");
  if (p->n < 0 || p->n > (int64_t(1) << 40)) return qfail(GP_ERR_ARG, "bad particle count");
  if (!std::isfinite(p->q) || !std::isfinite(p->w) || !(p->m > 0) || !std::isfinite(p->m))
    return qfail(GP_ERR_ARG, "q, w must be finite and m positive");
  if (p->n > 0 && (!p->x || !p->y || !p->z || !p->ux || !p->uy || !p->uz))
    return qfail(GP_ERR_ARG, "a particle array is NULL");
  c->part = *p;
  c->bound = true;
  c->dep_per = 0;  // chosen again for the new particle count
  c->zs_steps = 0;
  if (!c->zs_ctl) {
    void *ctl = nullptr;
    QTRY(qalloc(c, size_t(2 + 2 * kQcMaxNz) * sizeof(int), &ctl));
    c->zs_ctl = static_cast<int *>(ctl);
  }
  if (hipMemsetAsync(c->zs_ctl, 0, size_t(2 + 2 * kQcMaxNz) * sizeof(int), c->stream) !=
      hipSuccess)
    return qfail(GP_ERR_HIP, "clearing the re-sort counters failed");
  if (p->n > c->zs_cap) {
    QTRY(qalloc(c, size_t(6) * size_t(p->n) * c->real_size, &c->zs_tmp));
    c->zs_cap = p->n;
  }
  QTRY(c->d.precision == GP_FP64 ? sort_particles_by_z<double>(c) : sort_particles_by_z<float>(c));
  QTRY(fill_sources(c));
  // rho^n of the particles (and the background), transformed into the
  // rho^{n+1} slot, which then becomes rho^n
  QTRY(qdispatch(c, [&](auto t) {
    using T = decltype(t);
    launch_move_deposit<T>(c, 0);
    z_transform<T>(c, kFsFwdSrc, 4, false);
    hankel<T, kScalarFwd>(c, c->rho_old == 9 ? kQsRho1 : kQsRho0, 1, c->fmat);
  }));
  c->rho_old = c->rho_old == 9 ? 10 : 9;
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "stream synchronize failed");
  return GP_OK;
}

gp_status gp_qc_set_resort(gp_qc_ctx *c, int div) {
  QTRY(qcheck_ctx(c));
  if (div < 0) return qfail(GP_ERR_ARG, "div must be >= 0");
  c->resort_div = div;
  return GP_OK;
}

gp_status gp_qc_electrostatic_fields(gp_qc_ctx *c) {
  QTRY(qcheck_ctx(c));
  return qdispatch(c, [&](auto t) {
    using T = decltype(t);
    const int64_t n = int64_t(c->d.nmodes) * c->d.nz * c->d.nr;
    hipLaunchKernelGGL((k_qc_electrostatic<T>), dim3(unsigned((n + 255) / 256)), dim3(256), 0,
                       c->stream, static_cast<Cx<T> *>(c->spec[0]),
                       static_cast<Cx<T> *>(c->spec[1]), static_cast<Cx<T> *>(c->spec[2]),
                       static_cast<const Cx<T> *>(c->spec[c->rho_old]),
                       static_cast<const T *>(c->kr_t), c->d.nmodes, c->d.nz, c->d.nr,
                       T(2.0 * kPi / (c->d.nz * c->d.dz)));
    enqueue_fields_inv<T>(c);
  });
}

gp_status gp_qc_particle_step(gp_qc_ctx *c, int nsteps) {
  QTRY(qcheck_ctx(c));
  if (!c->bound) return qfail(GP_ERR_STATE, "no particles bound");
  if (nsteps < 0) return qfail(GP_ERR_ARG, "nsteps must be >= 0");
  for (int s = 0; s < nsteps; ++s) {
    QTRY(fill_sources(c));
    QTRY(qdispatch(c, [&](auto t) {
      using T = decltype(t);
      launch_move_deposit<T>(c, 1);
      enqueue_sources_fwd<T>(c);
      enqueue_update<T>(c);
      enqueue_fields_inv<T>(c);
      launch_gather_push<T>(c);
    }));
  }
  return GP_OK;
}

gp_status gp_qc_stage_timing(gp_qc_ctx *c, int enable) {
  QTRY(qcheck_ctx(c));
  c->timing = enable != 0;
  return GP_OK;
}

gp_status gp_qc_stage_times(gp_qc_ctx *c, double *ms, int *count) {
  QTRY(qcheck_ctx(c));
  if (!ms || !count) return qfail(GP_ERR_ARG, "output pointer is NULL");
  for (int i = 0; i < GP_QC_N_STAGES; ++i) {
    ms[i] = 0.0;
    count[i] = 0;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return qfail(GP_ERR_HIP, "stream synchronize failed");
  gp_status st = GP_OK;
  for (const auto &rec : c->recs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, rec.a, rec.b) == hipSuccess) {
      ms[rec.stage] += t;
      count[rec.stage] += 1;
    } else {
      st = qfail(GP_ERR_HIP, "hipEventElapsedTime failed");
    }
    (void)hipEventDestroy(rec.a);
    (void)hipEventDestroy(rec.b);
  }
  c->recs.clear();
  return st;
}

gp_status gp_qc_destroy(gp_qc_ctx *c) {
  if (!c) return GP_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (const auto &rec : c->recs) {
    (void)hipEventDestroy(rec.a);
    (void)hipEventDestroy(rec.b);
  }
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return GP_OK;
}

gp_status gp_qc_wavenumbers(int m, int nr, double dr, double *kr) {
  if (!kr) return qfail(GP_ERR_ARG, "kr is NULL");
  if (m < 0 || m > 63 || nr < 1 || nr > 512 || !(dr > 0) || !std::isfinite(dr))
    return qfail(GP_ERR_ARG, "m must lie in [0, 63], nr in [1, 512], dr positive and finite");
  const std::vector<double> k = spectral_kr(m, nr, dr);
  std::copy(k.begin(), k.end(), kr);
  return GP_OK;
}

gp_status gp_qc_hankel_matrix(int p, int m, int nr, double dr, int forward, double *out) {
  if (!out) return qfail(GP_ERR_ARG, "out is NULL");
  if (m < 0 || m > 63 || p < -64 || p > 64 || nr < 1 || nr > 512 || !(dr > 0) ||
      !std::isfinite(dr))
    return qfail(GP_ERR_ARG,
                 "m must lie in [0, 63], p in [-64, 64], nr in [1, 512], dr positive and finite");
  std::vector<double> M = backward_hankel(p, m, spectral_kr(m, nr, dr), nr, dr);
  if (forward && !invert(M, nr))
    return qfail(GP_ERR_ARG, "the Hankel matrix of order " + std::to_string(p) +
                                 " is singular for this nr");
  std::copy(M.begin(), M.end(), out);
  return GP_OK;
}
