// Hand-written 3D FFT for gfx950: three LDS-tiled passes per transform.
//
// Layout: real grids [x][y][z] (z contiguous), half spectra [x][y][nz/2+1].
// Forward kernel exp(-i k.x), unnormalised; the inverse applies 1/(nx ny nz)
// in its last (z) pass.
//
//  * z pass: a tile of CW whole z-lines is loaded with coalesced reads, each
//    real line of length nz is packed into nz/2 complex values, transformed,
//    and split into the nz/2+1 half-spectrum values (the standard real-FFT
//    packing identity).
//  * y and x passes: a tile of CW adjacent half-spectrum columns times the
//    whole line length L is loaded with row-contiguous (coalesced) reads of
//    CW complex values per row, transformed column by column in LDS, and
//    stored back the same way.  CW = 16 (float) or 8 (double) makes every row
//    segment 128 bytes.
//
// Inside a tile the transform is a Stockham autosort FFT: radix-8 passes and
// one radix-4 or radix-2 pass, all butterflies of all CW columns spread over
// the workgroup, two barriers per pass.  The LDS row stride is CW+1 complex
// values so column walks do not hit the same bank.
#include "kernels.hpp"

#include <cmath>

namespace galpic {
namespace {

constexpr int kTwN = 1024;  // twiddle table length; supports lines up to 1024

template <typename T>
struct TileCols;
template <>
struct TileCols<float> {
  static constexpr int value = 16;
};
template <>
struct TileCols<double> {
  static constexpr int value = 8;
};

// w^(m) for w = exp(-+2 pi i / N): the table holds exp(-2 pi i m / 1024).
template <typename T>
__device__ __forceinline__ Cx<T> twiddle(const Cx<T> *__restrict__ tw, int m, int logN,
                                         bool inverse) {
  Cx<T> w = tw[m << (10 - logN)];
  if (inverse) w.im = -w.im;
  return w;
}

// In-register DFTs of size 2, 4, 8 (sign -1 forward, +1 inverse).
template <typename T>
__device__ __forceinline__ void dft2(Cx<T> &a0, Cx<T> &a1) {
  Cx<T> t = a0 - a1;
  a0 = a0 + a1;
  a1 = t;
}

// multiply by -i (forward) or +i (inverse)
template <typename T>
__device__ __forceinline__ Cx<T> rot90(Cx<T> a, bool inverse) {
  return inverse ? cx(-a.im, a.re) : cx(a.im, -a.re);
}

template <typename T>
__device__ __forceinline__ void dft4(Cx<T> *a, bool inverse) {
  Cx<T> t0 = a[0] + a[2];
  Cx<T> t1 = a[0] - a[2];
  Cx<T> t2 = a[1] + a[3];
  Cx<T> t3 = rot90(a[1] - a[3], inverse);
  a[0] = t0 + t2;
  a[2] = t0 - t2;
  a[1] = t1 + t3;
  a[3] = t1 - t3;
}

template <typename T>
__device__ __forceinline__ void dft8(Cx<T> *a, bool inverse) {
  Cx<T> e[4] = {a[0], a[2], a[4], a[6]};
  Cx<T> o[4] = {a[1], a[3], a[5], a[7]};
  dft4(e, inverse);
  dft4(o, inverse);
  const T h = T(0.70710678118654752440);
  // w8^m, m = 0..3, w8 = exp(-+ i pi / 4)
  Cx<T> o1 = o[1];
  Cx<T> o2 = o[2];
  Cx<T> o3 = o[3];
  if (!inverse) {
    o1 = cx(h * (o1.re + o1.im), h * (o1.im - o1.re));
    o2 = cx(o2.im, -o2.re);
    o3 = cx(h * (o3.im - o3.re), -h * (o3.re + o3.im));
  } else {
    o1 = cx(h * (o1.re - o1.im), h * (o1.im + o1.re));
    o2 = cx(-o2.im, o2.re);
    o3 = cx(-h * (o3.re + o3.im), h * (o3.re - o3.im));
  }
  a[0] = e[0] + o[0];
  a[4] = e[0] - o[0];
  a[1] = e[1] + o1;
  a[5] = e[1] - o1;
  a[2] = e[2] + o2;
  a[6] = e[2] - o2;
  a[3] = e[3] + o3;
  a[7] = e[3] - o3;
}

template <typename T, int R>
__device__ __forceinline__ void dft_small(Cx<T> *a, bool inverse) {
  if constexpr (R == 8) {
    dft8(a, inverse);
  } else if constexpr (R == 4) {
    dft4(a, inverse);
  } else {
    dft2(a[0], a[1]);
  }
}

// Stockham FFT of CW columns of length L = 2^LOGL stored in LDS as
// lds[row * S + col].
template <typename T, int LOGL, int CW, int NT, int S>
struct TileFFT {
  static constexpr int L = 1 << LOGL;

  template <int R, int LOGNS>
  __device__ __forceinline__ static void pass(Cx<T> *lds, const Cx<T> *__restrict__ tw,
                                              int tid, bool inverse) {
    constexpr int NS = 1 << LOGNS;
    constexpr int LOGR = R == 8 ? 3 : (R == 4 ? 2 : 1);
    constexpr int ITEMS = CW * (L / R);
    constexpr int PER = (ITEMS + NT - 1) / NT;
    Cx<T> a[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int it = tid + p * NT;
      if (ITEMS % NT == 0 || it < ITEMS) {
        const int c = it % CW;
        const int j = it / CW;
#pragma unroll
        for (int r = 0; r < R; ++r) a[p][r] = lds[(j + r * (L / R)) * S + c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int it = tid + p * NT;
      if (ITEMS % NT == 0 || it < ITEMS) {
        const int c = it % CW;
        const int j = it / CW;
        const int k = j & (NS - 1);
        if (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r)
            a[p][r] = a[p][r] * twiddle(tw, k * r, LOGNS + LOGR, inverse);
        }
        dft_small<T, R>(a[p], inverse);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[(base + r * NS) * S + c] = a[p][r];
      }
    }
    __syncthreads();
  }

  template <int REM, int LOGNS>
  __device__ __forceinline__ static void passes(Cx<T> *lds, const Cx<T> *tw, int tid,
                                                bool inverse) {
    if constexpr (REM >= 3) {
      pass<8, LOGNS>(lds, tw, tid, inverse);
      passes<REM - 3, LOGNS + 3>(lds, tw, tid, inverse);
    } else if constexpr (REM == 2) {
      pass<4, LOGNS>(lds, tw, tid, inverse);
    } else if constexpr (REM == 1) {
      pass<2, LOGNS>(lds, tw, tid, inverse);
    }
  }

  __device__ __forceinline__ static void run(Cx<T> *lds, const Cx<T> *tw, int tid,
                                             bool inverse) {
    passes<LOGL, 0>(lds, tw, tid, inverse);
  }
};

constexpr int kThreads = 256;

// Items per thread whose global loads (or LDS reads) are issued together
// before any of their results is used: a rolled loop would wait for each
// load in turn, one memory latency per item.
template <typename T>
struct Chunk {
  static constexpr int value = sizeof(T) == 4 ? 16 : 8;
};

// Items it = tid, tid + kThreads, ... < ITEMS of a tile: get(it) for a chunk
// of them, then put(it, value) for the same chunk.  Moves a tile from
// global memory into LDS (get loads) or out of it (get reads LDS).
template <typename T, int ITEMS, class Get, class Put>
__device__ __forceinline__ void tile_items(int tid, Get get, Put put) {
  constexpr int PER = (ITEMS + kThreads - 1) / kThreads;
  constexpr int CH = PER < Chunk<T>::value ? PER : Chunk<T>::value;
  // every item of every chunk exists: no bound checks
  constexpr bool kExact = ITEMS % kThreads == 0 && PER % CH == 0;
  for (int p0 = 0; p0 < PER; p0 += CH) {
    Cx<T> v[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int it = tid + (p0 + q) * kThreads;
      if (kExact || it < ITEMS) v[q] = get(it);
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int it = tid + (p0 + q) * kThreads;
      if (kExact || it < ITEMS) put(it, v[q]);
    }
  }
}

// The workgroup's (x, y) in the launch grid, renumbered so that each XCD
// takes a contiguous range of tiles: neighbouring column tiles of the y and
// x passes share the cache lines at their edges (rows of nz/2 + 1 complex
// values are not line-aligned), which one L2 then fetches once.  (The z
// passes, whose tiles are whole contiguous lines, keep the plain order:
// measured no faster renumbered.)
struct Tile {
  unsigned x, y;
};
__device__ __forceinline__ Tile tile_xcd() {
  const unsigned w = blockIdx.x + blockIdx.y * gridDim.x;
  const unsigned l = xcd_contiguous(w, gridDim.x * gridDim.y);
  return Tile{l % gridDim.x, l / gridDim.x};
}

// ---- z pass, forward: real lines -> half spectra ---------------------------
template <typename T, int LOGM>
__global__ __launch_bounds__(kThreads) void k_r2c_z(const FieldSet *__restrict__ sets, int nf,
                                                    int64_t nlines,
                                                    const Cx<T> *__restrict__ tw) {
  constexpr int CW = TileCols<T>::value;
  constexpr int S = CW + 1;
  constexpr int M = 1 << LOGM;
  constexpr int NZH = M + 1;
  __shared__ Cx<T> lds[M * S];
  const FieldSet &fs = sets[blockIdx.y / nf];
  const int f = blockIdx.y % nf;
  const Cx<T> *__restrict__ in = static_cast<const Cx<T> *>(global_ptr(fs.in[f]));
  Cx<T> *__restrict__ out = static_cast<Cx<T> *>(global_ptr(fs.out[f]));
  const int64_t line0 = int64_t(blockIdx.x) * CW;
  const int tid = threadIdx.x;
  tile_items<T, CW * M>(
      tid,
      [&](int it) {
        const int64_t line = line0 + it / M;
        return line < nlines ? in[line * M + it % M] : cx(T(0), T(0));
      },
      [&](int it, Cx<T> v) { lds[(it % M) * S + it / M] = v; });
  __syncthreads();
  TileFFT<T, LOGM, CW, kThreads, S>::run(lds, tw, tid, false);
  tile_items<T, CW * NZH>(
      tid,
      [&](int it) {
        const int k = it % NZH;
        const int c = it / NZH;
        const Cx<T> zk = lds[(k & (M - 1)) * S + c];
        const Cx<T> zm = conj(lds[((M - k) & (M - 1)) * S + c]);
        const Cx<T> even = T(0.5) * (zk + zm);
        const Cx<T> d = zk - zm;
        const Cx<T> odd = cx(T(0.5) * d.im, T(-0.5) * d.re);  // (zk - zm) / (2i)
        const Cx<T> w = twiddle(tw, k, LOGM + 1, false);       // exp(-2 pi i k / nz)
        return even + w * odd;
      },
      [&](int it, Cx<T> v) {
        const int64_t line = line0 + it / NZH;
        if (line < nlines) out[line * NZH + it % NZH] = v;
      });
}

// ---- z pass, inverse: half spectra -> real lines, scaled -------------------
template <typename T, int LOGM>
__global__ __launch_bounds__(kThreads) void k_c2r_z(const FieldSet *__restrict__ sets, int nf,
                                                    int64_t nlines, T scale,
                                                    const Cx<T> *__restrict__ tw) {
  constexpr int CW = TileCols<T>::value;
  constexpr int S = CW + 1;
  constexpr int M = 1 << LOGM;
  constexpr int NZH = M + 1;
  __shared__ Cx<T> lds[M * S];
  const FieldSet &fs = sets[blockIdx.y / nf];
  const int f = blockIdx.y % nf;
  const Cx<T> *__restrict__ in = static_cast<const Cx<T> *>(global_ptr(fs.in[f]));
  Cx<T> *__restrict__ out = static_cast<Cx<T> *>(global_ptr(fs.out[f]));
  const int64_t line0 = int64_t(blockIdx.x) * CW;
  const int tid = threadIdx.x;
  tile_items<T, CW * M>(
      tid,
      [&](int it) {
        const int k = it % M;
        const int64_t line = line0 + it / M;
        // loads from a valid line in every case (no branch around them, so
        // a chunk's loads are all in flight together); a line past the
        // last gives zero
        const int64_t ln = line < nlines ? line : nlines - 1;
        Cx<T> xk = in[ln * NZH + k];
        Cx<T> xm = conj(in[ln * NZH + (M - k)]);
        if (k == 0) {
          // the k_z = 0 and Nyquist values of a real field are real after
          // the x and y passes: keeping their real parts takes the
          // Hermitian part of the spectrum (as a real inverse transform
          // does), whatever rounding left in the other part
          xk.im = T(0);
          xm.im = T(0);
        }
        const Cx<T> even = xk + xm;
        const Cx<T> odd = (xk - xm) * twiddle(tw, k, LOGM + 1, true);
        const Cx<T> z = even + mul_i(odd);
        return line < nlines ? z : cx(T(0), T(0));
      },
      [&](int it, Cx<T> v) { lds[(it % M) * S + it / M] = v; });
  __syncthreads();
  TileFFT<T, LOGM, CW, kThreads, S>::run(lds, tw, tid, true);
  tile_items<T, CW * M>(
      tid, [&](int it) { return lds[(it % M) * S + it / M]; },
      [&](int it, Cx<T> z) {
        const int64_t line = line0 + it / M;
        if (line < nlines) out[line * M + it % M] = cx(scale * z.re, scale * z.im);
      });
}

// ---- y / x passes: complex transforms along a strided axis -----------------
struct StridedGeom {
  int ncols;            // nz/2 + 1
  int col_tiles;        // ceil(ncols / CW)
  int64_t row_stride;   // distance between consecutive line elements
  int64_t outer_stride; // distance between consecutive outer indices
  // held-mode mask (forward x pass only; kMask*): row = ix, outer = iy,
  // col = iz
  int mask;
  int half_row, half_outer, half_col;
};

// CW columns per workgroup: TileCols<T> by default; fewer where that would
// leave the chip short of workgroups (few, long lines).
template <typename T, int LOGL, int CW = TileCols<T>::value>
__global__ __launch_bounds__(kThreads) void k_c2c_strided(const FieldSet *__restrict__ sets,
                                                          int nf, StridedGeom sg, int inverse,
                                                          const Cx<T> *__restrict__ tw) {
  constexpr int S = CW + 1;
  constexpr int L = 1 << LOGL;
  __shared__ Cx<T> lds[L * S];
  const Tile wg = tile_xcd();
  const FieldSet &fs = sets[wg.y / nf];
  const int f = wg.y % nf;
  const Cx<T> *__restrict__ in = static_cast<const Cx<T> *>(global_ptr(fs.in[f]));
  Cx<T> *__restrict__ out = static_cast<Cx<T> *>(global_ptr(fs.out[f]));
  const int outer = wg.x / sg.col_tiles;
  const int col0 = (wg.x % sg.col_tiles) * CW;
  const int64_t base = int64_t(outer) * sg.outer_stride + col0;
  const int tid = threadIdx.x;
  tile_items<T, CW * L>(
      tid,
      [&](int it) {
        const int c = it % CW;
        return col0 + c < sg.ncols ? in[base + (it / CW) * sg.row_stride + c] : cx(T(0), T(0));
      },
      [&](int it, Cx<T> v) { lds[(it / CW) * S + it % CW] = v; });
  __syncthreads();
  TileFFT<T, LOGL, CW, kThreads, S>::run(lds, tw, tid, inverse != 0);
  tile_items<T, CW * L>(
      tid, [&](int it) { return lds[(it / CW) * S + it % CW]; },
      [&](int it, Cx<T> v) {
        const int c = it % CW;
        const int j = it / CW;
        const int col = col0 + c;
        if (col >= sg.ncols) return;
        if (sg.mask) {
          const bool held = j == sg.half_row || outer == sg.half_outer || col == sg.half_col ||
                            (sg.mask == kMaskHeld && j == 0 && outer == 0 && col == 0);
          if (held) v = cx(T(0), T(0));
        }
        out[base + j * sg.row_stride + c] = v;
      });
}

// Workgroup row blockIdx.y = set * nf + field: one launch transforms nf
// fields of every run in the table.
template <typename T, int LOG>
void dispatch_r2c(const FieldSet *sets, int nsets, int nf, int64_t nlines, const Cx<T> *tw,
                  hipStream_t s) {
  constexpr int CW = TileCols<T>::value;
  dim3 grid(unsigned((nlines + CW - 1) / CW), unsigned(nf * nsets));
  hipLaunchKernelGGL((k_r2c_z<T, LOG>), grid, dim3(kThreads), 0, s, sets, nf, nlines, tw);
}

template <typename T, int LOG>
void dispatch_c2r(const FieldSet *sets, int nsets, int nf, int64_t nlines, T scale,
                  const Cx<T> *tw, hipStream_t s) {
  constexpr int CW = TileCols<T>::value;
  dim3 grid(unsigned((nlines + CW - 1) / CW), unsigned(nf * nsets));
  hipLaunchKernelGGL((k_c2r_z<T, LOG>), grid, dim3(kThreads), 0, s, sets, nf, nlines, scale,
                     tw);
}

template <typename T, int LOG, int CW = TileCols<T>::value>
void dispatch_c2c(const FieldSet *sets, int nsets, int nf, const StridedGeom &sg, int n_outer,
                  int inverse, const Cx<T> *tw, hipStream_t s) {
  dim3 grid(unsigned(n_outer * sg.col_tiles), unsigned(nf * nsets));
  hipLaunchKernelGGL((k_c2c_strided<T, LOG, CW>), grid, dim3(kThreads), 0, s, sets, nf, sg,
                     inverse, tw);
}

}  // namespace

template <typename T>
void fill_twiddles(Cx<T> *h) {
  for (int m = 0; m < kTwN; ++m) {
    // exact values on the axes and diagonals keep symmetric roundoff
    const double a = -2.0 * kPi * double(m) / double(kTwN);
    h[m] = cx(T(std::cos(a)), T(std::sin(a)));
  }
}

template <typename T>
void launch_r2c_z(const FieldSet *sets, int nsets, int nf, const RunGeom &g, const Cx<T> *tw,
                  hipStream_t s) {
  const int64_t nlines = int64_t(g.nx) * g.ny;
  switch (g.lz - 1) {
    case 2: dispatch_r2c<T, 2>(sets, nsets, nf, nlines, tw, s); break;
    case 3: dispatch_r2c<T, 3>(sets, nsets, nf, nlines, tw, s); break;
    case 4: dispatch_r2c<T, 4>(sets, nsets, nf, nlines, tw, s); break;
    case 5: dispatch_r2c<T, 5>(sets, nsets, nf, nlines, tw, s); break;
    case 6: dispatch_r2c<T, 6>(sets, nsets, nf, nlines, tw, s); break;
    case 7: dispatch_r2c<T, 7>(sets, nsets, nf, nlines, tw, s); break;
    case 8: dispatch_r2c<T, 8>(sets, nsets, nf, nlines, tw, s); break;
    case 9: dispatch_r2c<T, 9>(sets, nsets, nf, nlines, tw, s); break;
    default: break;  // sizes are validated by the caller
  }
}

template <typename T>
void launch_c2r_z(const FieldSet *sets, int nsets, int nf, const RunGeom &g, const Cx<T> *tw,
                  hipStream_t s) {
  const int64_t nlines = int64_t(g.nx) * g.ny;
  const T scale = T(1.0 / double(g.ncell));
  switch (g.lz - 1) {
    case 2: dispatch_c2r<T, 2>(sets, nsets, nf, nlines, scale, tw, s); break;
    case 3: dispatch_c2r<T, 3>(sets, nsets, nf, nlines, scale, tw, s); break;
    case 4: dispatch_c2r<T, 4>(sets, nsets, nf, nlines, scale, tw, s); break;
    case 5: dispatch_c2r<T, 5>(sets, nsets, nf, nlines, scale, tw, s); break;
    case 6: dispatch_c2r<T, 6>(sets, nsets, nf, nlines, scale, tw, s); break;
    case 7: dispatch_c2r<T, 7>(sets, nsets, nf, nlines, scale, tw, s); break;
    case 8: dispatch_c2r<T, 8>(sets, nsets, nf, nlines, scale, tw, s); break;
    case 9: dispatch_c2r<T, 9>(sets, nsets, nf, nlines, scale, tw, s); break;
    default: break;
  }
}

template <typename T>
void launch_c2c(const FieldSet *sets, int nsets, int nf, const RunGeom &g, int axis,
                bool inverse, int mask, const Cx<T> *tw, hipStream_t s) {
  constexpr int CW = TileCols<T>::value;
  StridedGeom sg;
  sg.ncols = g.nzh;
  sg.col_tiles = (g.nzh + CW - 1) / CW;
  sg.mask = mask;
  int logl, n_outer;
  if (axis == 1) {  // y lines: outer = x
    sg.row_stride = g.nzh;
    sg.outer_stride = int64_t(g.ny) * g.nzh;
    logl = g.ly;
    n_outer = g.nx;
    sg.half_row = g.ny / 2;
    sg.half_outer = g.nx / 2;
  } else {          // x lines: outer = y
    sg.row_stride = int64_t(g.ny) * g.nzh;
    sg.outer_stride = g.nzh;
    logl = g.lx;
    n_outer = g.ny;
    sg.half_row = g.nx / 2;
    sg.half_outer = g.ny / 2;
  }
  sg.half_col = g.nz / 2;
  const int inv = inverse ? 1 : 0;
  switch (logl) {
    case 3: dispatch_c2c<T, 3>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 4: dispatch_c2c<T, 4>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 5: dispatch_c2c<T, 5>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 6: dispatch_c2c<T, 6>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 7: dispatch_c2c<T, 7>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 8: dispatch_c2c<T, 8>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 9: dispatch_c2c<T, 9>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 10: dispatch_c2c<T, 10>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    default: break;
  }
}

template <typename T, int CW>
void lines_cw(const FieldSet *sets, int nsets, int nf, int log_len, const StridedGeom &sg,
              int n_outer, int inv, const Cx<T> *tw, hipStream_t s) {
  switch (log_len) {
    case 3: dispatch_c2c<T, 3, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 4: dispatch_c2c<T, 4, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 5: dispatch_c2c<T, 5, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 6: dispatch_c2c<T, 6, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 7: dispatch_c2c<T, 7, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 8: dispatch_c2c<T, 8, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 9: dispatch_c2c<T, 9, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    case 10: dispatch_c2c<T, 10, CW>(sets, nsets, nf, sg, n_outer, inv, tw, s); break;
    default: break;
  }
}

template <typename T>
void launch_c2c_lines(const FieldSet *sets, int nsets, int nf, int log_len, int ncols,
                      int64_t row_stride, int64_t outer_stride, int n_outer, bool inverse,
                      const Cx<T> *tw, hipStream_t s) {
  constexpr int CW = TileCols<T>::value;
  constexpr int kNarrow = 4;
  StridedGeom sg{};
  sg.ncols = ncols;
  sg.row_stride = row_stride;
  sg.outer_stride = outer_stride;
  sg.mask = 0;
  const int inv = inverse ? 1 : 0;
  // Narrow tiles when the default width gives fewer than two workgroups per CU.
  const int64_t wide = int64_t(n_outer) * ((ncols + CW - 1) / CW) * nf * nsets;
  if (wide < 512) {
    sg.col_tiles = (ncols + kNarrow - 1) / kNarrow;
    lines_cw<T, kNarrow>(sets, nsets, nf, log_len, sg, n_outer, inv, tw, s);
  } else {
    sg.col_tiles = (ncols + CW - 1) / CW;
    lines_cw<T, CW>(sets, nsets, nf, log_len, sg, n_outer, inv, tw, s);
  }
}

template void launch_c2c_lines<float>(const FieldSet *, int, int, int, int, int64_t, int64_t,
                                      int, bool, const Cx<float> *, hipStream_t);
template void launch_c2c_lines<double>(const FieldSet *, int, int, int, int, int64_t, int64_t,
                                       int, bool, const Cx<double> *, hipStream_t);
template void fill_twiddles<float>(Cx<float> *);
template void fill_twiddles<double>(Cx<double> *);
template void launch_r2c_z<float>(const FieldSet *, int, int, const RunGeom &, const Cx<float> *,
                                  hipStream_t);
template void launch_r2c_z<double>(const FieldSet *, int, int, const RunGeom &,
                                   const Cx<double> *, hipStream_t);
template void launch_c2r_z<float>(const FieldSet *, int, int, const RunGeom &, const Cx<float> *,
                                  hipStream_t);
template void launch_c2r_z<double>(const FieldSet *, int, int, const RunGeom &,
                                   const Cx<double> *, hipStream_t);
template void launch_c2c<float>(const FieldSet *, int, int, const RunGeom &, int, bool, int,
                                const Cx<float> *, hipStream_t);
template void launch_c2c<double>(const FieldSet *, int, int, const RunGeom &, int, bool, int,
                                 const Cx<double> *, hipStream_t);

}  // namespace galpic
