// Internal types shared by the gfx950 kernels and the C ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace galpic {

// Interleaved complex value; aligned so one element is one vector load.
template <typename T>
struct alignas(2 * sizeof(T)) Cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ Cx<T> cx(T re, T im) {
  Cx<T> r;
  r.re = re;
  r.im = im;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) {
  return cx(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) {
  return cx(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) {
  return cx(s * a.re, s * a.im);
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> conj(Cx<T> a) {
  return cx(a.re, -a.im);
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ Cx<T> mul_i(Cx<T> a) {
  return cx(-a.im, a.re);
}

// Geometry of one run as the kernels see it.
struct RunGeom {
  int nx, ny, nz, nzh;       // nzh = nz/2 + 1 (half-spectrum length)
  int lx, ly, lz;            // log2 of nx, ny, nz
  int order;                 // shape order, 1 or 3
  double dx, dy, dz, dt;
  double vgal[3];
  int64_t ncell;             // nx * ny * nz
  int64_t nmode;             // nx * ny * nzh
};

// Particle arrays of one run (layout decided by the precision).
struct PartPtrs {
  int64_t n;
  double q, m, w;
  void *x, *y, *z;           // FP64: double positions; MIXED: x = int32 cell
  void *ox, *oy, *oz;        // MIXED: float offsets
  void *ux, *uy, *uz;
  int64_t *id;
};

constexpr double kPi = 3.14159265358979323846;

// A pointer read from a table in memory is generic to the compiler, which
// then emits flat instructions for it.  Every device buffer of the library
// is global memory: rebuilding the pointer from its integer value as a
// global-space pointer lets the compiler emit global loads, stores and
// atomics (a direct cast round trip would be folded away).
template <typename P>
__device__ __forceinline__ P *global_ptr(P *p) {
  using G = __attribute__((address_space(1))) P;
  return (P *)(G *)(uintptr_t)p;
}

// gfx950 deals the workgroups of a launch out to its 8 XCDs in turn (the
// linear workgroup w to XCD w mod 8), and every XCD has an L2 of its own.
// Numbering the logical work so that each XCD takes one contiguous range of
// it keeps neighbouring tiles, whose reads and writes share cache lines, in
// one L2.  A bijection of [0, total).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_contiguous(unsigned w, unsigned total) {
  const unsigned q = total / kXcds, r = total % kXcds;
  const unsigned x = w % kXcds, slot = w / kXcds;
  return x * q + (x < r ? x : r) + slot;
}

}  // namespace galpic
