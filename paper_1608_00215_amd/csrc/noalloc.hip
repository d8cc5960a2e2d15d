// Field energy without any allocation, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The same quantity as gp_field_energy,
// W_E = 1/2 sum |E|^2 dV and W_B = 1/2 sum |B|^2 dV of one run's real
// fields, reduced in double in two passes through a file-scope device
// array: each workgroup of the first pass writes the sums of its own chunk
// of cells to its slot, the second pass adds the slots in a fixed order, so
// the result does not depend on scheduling and nothing needs clearing.
//
// The array is a host-side stand-in in host code: kernels get its device
// address, looked up once per device when a context is created there
// (noalloc_prepare) and kept per device.  Every call on a device shares
// that device's array: calls that overlap on one device race.
#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace galpic {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kChunk = 8192;         // cells per workgroup of the first pass
constexpr int kMaxChunks = 8192;         // slots of the array: up to 2^26 cells
static __device__ __align__(256) double scratch[2 * kMaxChunks];

std::mutex g_mu;
std::vector<double *> g_ptr;  // per device: the array's device address

template <typename T>
__global__ __launch_bounds__(kThreads) void k_energy_chunks(const T *__restrict__ e0,
                                                            const T *__restrict__ e1,
                                                            const T *__restrict__ e2,
                                                            const T *__restrict__ b0,
                                                            const T *__restrict__ b1,
                                                            const T *__restrict__ b2,
                                                            int64_t ncell, double *slots) {
  __shared__ double part[2][kThreads / 64];
  const int64_t lo = int64_t(blockIdx.x) * kChunk;
  const int64_t hi = lo + kChunk < ncell ? lo + kChunk : ncell;
  double se = 0.0, sb = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double x = e0[i], y = e1[i], z = e2[i];
    const double u = b0[i], v = b1[i], w = b2[i];
    se += x * x + y * y + z * z;
    sb += u * u + v * v + w * w;
  }
  for (int off = 32; off > 0; off >>= 1) {
    se += __shfl_down(se, off, 64);
    sb += __shfl_down(sb, off, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][wave] = se;
    part[1][wave] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double te = 0.0, tb = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) {
      te += part[0][k];
      tb += part[1][k];
    }
    slots[2 * blockIdx.x] = te;
    slots[2 * blockIdx.x + 1] = tb;
  }
}

// One workgroup: the slots in a fixed order, times dV / 2, into out[0..1].
__global__ __launch_bounds__(kThreads) void k_energy_total(const double *__restrict__ slots,
                                                           int nslots, double half_dv,
                                                           double *out) {
  __shared__ double part[2][kThreads];
  double se = 0.0, sb = 0.0;
  for (int k = threadIdx.x; k < nslots; k += kThreads) {
    se += slots[2 * k];
    sb += slots[2 * k + 1];
  }
  part[0][threadIdx.x] = se;
  part[1][threadIdx.x] = sb;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) {
      part[0][threadIdx.x] += part[0][threadIdx.x + h];
      part[1][threadIdx.x] += part[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = half_dv * part[0][0];
    out[1] = half_dv * part[1][0];
  }
}

}  // namespace

int64_t noalloc_max_cells() { return int64_t(kChunk) * kMaxChunks; }

hipError_t noalloc_prepare() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  if (dev < int(g_ptr.size()) && g_ptr[dev]) return hipSuccess;
  double *p = nullptr;
  e = hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (dev >= int(g_ptr.size())) g_ptr.resize(dev + 1, nullptr);
  g_ptr[dev] = p;
  return hipSuccess;
}

double *noalloc_scratch(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  return dev >= 0 && dev < int(g_ptr.size()) ? g_ptr[dev] : nullptr;
}

template <typename T>
void launch_energy_noalloc(const T *const E[3], const T *const B[3], int64_t ncell, double dv,
                           double *slots, double *out, hipStream_t s) {
  const int nchunks = int((ncell + kChunk - 1) / kChunk);
  if (nchunks > 0)
    hipLaunchKernelGGL((k_energy_chunks<T>), dim3(unsigned(nchunks)), dim3(kThreads), 0, s,
                       E[0], E[1], E[2], B[0], B[1], B[2], ncell, slots);
  hipLaunchKernelGGL(k_energy_total, dim3(1), dim3(kThreads), 0, s, slots, nchunks, 0.5 * dv,
                     out);
}

template void launch_energy_noalloc<float>(const float *const[3], const float *const[3],
                                           int64_t, double, double *, double *, hipStream_t);
template void launch_energy_noalloc<double>(const double *const[3], const double *const[3],
                                            int64_t, double, double *, double *, hipStream_t);

}  // namespace galpic
