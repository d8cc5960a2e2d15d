// Copies of the slab field solve: windows of a run's real grids into its
// slabs' local grids (owned planes plus guard planes on each side, periodic
// in z), the grid sums whose means the sources lose, and the owned planes
// of the slabs' new E, B back into the run's grids.  Each thread of the
// copies takes kUnroll elements a grid stride apart per round and issues
// their loads before any store, so that their latencies overlap.
//
// The paper names domain decomposition with local transforms over
// subdomains padded by guard cells, made possible by finite-order solvers,
// as future work.  On one device the guard exchange between neighbouring
// slabs is a copy out of the run's global arrays.  All three kernels are
// streaming copies: HBM-bound, z contiguous on both sides.
#include "kernels.hpp"

namespace galpic {
namespace {

constexpr int kUnroll = 4;

// Workgroup row blockIdx.y = run * 4 + quantity.
template <typename T>
__global__ __launch_bounds__(256) void k_slab_sums(const SlabSum<T> *__restrict__ sums) {
  const SlabSum<T> &sm = sums[blockIdx.y >> 2];
  const int q = blockIdx.y & 3;
  const T *__restrict__ src = global_ptr(sm.src[q]);
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i0 < sm.ncell;
       i0 += kUnroll * stride) {
    T v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = i0 + u * stride < sm.ncell ? src[i0 + u * stride] : T(0);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += double(v[u]);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(global_ptr(sm.out) + q, acc);
}

// Workgroup row blockIdx.y = slab * nf + (field - f0).
template <typename T>
__global__ __launch_bounds__(256) void k_slab_window(const SlabCopy<T> *__restrict__ jobs, int f0,
                                                     int nf) {
  const SlabCopy<T> &jb = jobs[blockIdx.y / nf];
  const int f = f0 + int(blockIdx.y % nf);
  const T *__restrict__ src = global_ptr(jb.glob[f]);
  T *__restrict__ dst = global_ptr(jb.win[f]);
  const T mean = f >= 6 ? T(global_ptr(jb.sums)[f - 6] * jb.inv_ncell) : T(0);
  const int64_t n = int64_t(jb.nxy) * jb.nw;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e0 < n;
       e0 += kUnroll * stride) {
    T v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t e = e0 + u * stride;
      const int64_t xy = e / jb.nw;
      const int j = int(e - xy * jb.nw);
      const int z = (jb.first + j) & (jb.nz - 1);
      v[u] = e < n ? src[xy * jb.nz + z] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (e0 + u * stride < n) dst[e0 + u * stride] = v[u] - mean;
  }
}

// Workgroup row blockIdx.y = slab * 6 + field (E, B).
template <typename T>
__global__ __launch_bounds__(256) void k_slab_interior(const SlabCopy<T> *__restrict__ jobs) {
  const SlabCopy<T> &jb = jobs[blockIdx.y / 6];
  const int f = int(blockIdx.y % 6);
  const T *__restrict__ src = global_ptr(jb.win[f]);
  T *__restrict__ dst = global_ptr(jb.glob[f]);
  const int64_t n = int64_t(jb.nxy) * jb.ns;
  const int own0 = jb.first + jb.guard;  // global plane of owned plane 0 (in [0, nz))
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e0 < n;
       e0 += kUnroll * stride) {
    T v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t e = e0 + u * stride;
      const int64_t xy = e / jb.ns;
      const int i = int(e - xy * jb.ns);
      v[u] = e < n ? src[xy * jb.nw + jb.guard + i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t e = e0 + u * stride;
      if (e < n) {
        const int64_t xy = e / jb.ns;
        dst[xy * jb.nz + own0 + int(e - xy * jb.ns)] = v[u];
      }
    }
  }
}

unsigned blocks_for(int64_t n, int64_t cap) {
  int64_t b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return unsigned(b);
}

}  // namespace

template <typename T>
void launch_slab_sums(const SlabSum<T> *sums, int nruns, int64_t max_cells, hipStream_t s) {
  hipLaunchKernelGGL((k_slab_sums<T>), dim3(blocks_for(max_cells, 1024), unsigned(4 * nruns)),
                     dim3(256), 0, s, sums);
}

template <typename T>
void launch_slab_window(const SlabCopy<T> *jobs, int njobs, int f0, int nf, int64_t max_win,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_slab_window<T>), dim3(blocks_for(max_win, 2048), unsigned(njobs * nf)),
                     dim3(256), 0, s, jobs, f0, nf);
}

template <typename T>
void launch_slab_interior(const SlabCopy<T> *jobs, int njobs, int64_t max_owned,
                          hipStream_t s) {
  hipLaunchKernelGGL((k_slab_interior<T>), dim3(blocks_for(max_owned, 2048),
                                                unsigned(njobs * 6)),
                     dim3(256), 0, s, jobs);
}

template void launch_slab_sums<float>(const SlabSum<float> *, int, int64_t, hipStream_t);
template void launch_slab_sums<double>(const SlabSum<double> *, int, int64_t, hipStream_t);
template void launch_slab_window<float>(const SlabCopy<float> *, int, int, int, int64_t,
                                        hipStream_t);
template void launch_slab_window<double>(const SlabCopy<double> *, int, int, int, int64_t,
                                         hipStream_t);
template void launch_slab_interior<float>(const SlabCopy<float> *, int, int64_t, hipStream_t);
template void launch_slab_interior<double>(const SlabCopy<double> *, int, int64_t, hipStream_t);

}  // namespace galpic
