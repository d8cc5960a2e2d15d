// Lab-frame snapshots of a boosted run (back-transformed diagnostics).
//
// The boosted frame moves at +beta c along z relative to the lab and the
// grid is the Galilean one with v_gal = (0, 0, -beta c), in which the
// plasma at rest in the lab is at rest.  A grid node z'_k = k dz at boosted
// time t' is the lab event z_lab = gamma z'_k, t_lab = t'/gamma +
// gamma beta z'_k / c, so lab plane gamma z'_k of the snapshot at lab time
// t_j takes the fields of Galilean plane k at boosted time
//   t'_jk = gamma t_j - gamma^2 beta z'_k / c,
// linearly interpolated between the two stored levels t'_n < t'_jk <=
// t'_{n+1} (levels t'_n = t'_0 + n dt), after the Lorentz transformation
//   E_x = gamma (E'_x + beta c B'_y),   E_y = gamma (E'_y - beta c B'_x),
//   B_x = gamma (B'_x - beta E'_y / c), B_y = gamma (B'_y + beta E'_x / c),
//   E_z = E'_z, B_z = B'_z      (c = 1).
//
// On the fly: after each field cycle the real E, B are level m (a device
// counter, so graph replays advance it too).  Level m adds w T(F^m) to the
// planes with t'_jk in (t'_{m-1}, t'_m] and (1 - w) T(F^m) to those with
// t'_jk in (t'_m, t'_{m+1}], w being the plane's interpolation weight; a
// plane is complete once both levels around it have been seen.  Each
// launch touches the few planes per snapshot whose boosted time falls in
// the two steps around the level: the work is tiny next to the step, and
// spread over (x, y) tiles so that a touched plane is not a serial walk.
// The snapshots are stored plane by plane ([z][x][y] per field), so the
// writes of a plane are contiguous; its reads from the [x][y][z] fields
// take one cache line per node.
#include "kernels.hpp"

namespace galpic {
namespace {

constexpr int kThreads = 256;
constexpr int kNodesPerBlock = 4 * kThreads;  // (x, y) nodes of a plane per workgroup

// Workgroup (tile, snapshot j, job): the tile's (x, y) nodes of every plane
// that level m touches in snapshot j.  The candidate planes come from
// inverting t'_jk = gamma t_j - gamma^2 beta k dz over the two steps around
// level m (a handful of planes); the exact comparison then decides each.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_btd(const BtdJob<T> *__restrict__ jobs) {
  // the plane times decide which planes a level touches; computed without
  // contraction so that the decision is the plain double expression
#pragma clang fp contract(off)
  BtdJob<T> jb = jobs[blockIdx.z];
  const int j = blockIdx.y;
  const int64_t nxy = int64_t(jb.nx) * jb.ny;
  const int64_t xy0 = int64_t(blockIdx.x) * kNodesPerBlock;
  if (j >= jb.nsnap || xy0 >= nxy) return;
  for (int f = 0; f < 6; ++f) jb.F[f] = global_ptr(jb.F[f]);
  jb.out = global_ptr(jb.out);
  const int m = *global_ptr(jb.level);
  const double t_prev = jb.t0 + double(m - 1) * jb.dt;
  const double t_m = jb.t0 + double(m) * jb.dt;
  const double t_next = jb.t0 + double(m + 1) * jb.dt;
  const double tj = jb.t_lab0 + double(j) * jb.dt_lab;
  const double gt = jb.gamma * tj;
  const double g2b = jb.gamma * jb.gamma * jb.beta;
  // planes with t_prev < t'_jk <= t_next, widened by one on each side
  int kmin = 0, kmax = jb.nz - 1;
  const double s = g2b * jb.dz;
  const double ka = (gt - t_next) / s, kb = (gt - t_prev) / s;
  if (isfinite(ka) && isfinite(kb)) {
    const double lo = fmin(ka, kb), hi = fmax(ka, kb);
    if (hi < -1.0 || lo > double(jb.nz)) return;
    // clamped in double first: the quotients may exceed the int range
    kmin = max(0, int(fmax(floor(lo), -1.0)) - 1);
    kmax = min(jb.nz - 1, int(fmin(ceil(hi), double(jb.nz))) + 1);
  }
  const int64_t ncell = nxy * jb.nz;
  T *out = jb.out + int64_t(j) * 6 * ncell;
  const T g = T(jb.gamma), gb = T(jb.gamma * jb.beta);
  for (int k = kmin; k <= kmax; ++k) {
    const double tp = gt - g2b * (double(k) * jb.dz);
    double wgt;
    if (m >= 1 && tp > t_prev && tp <= t_m)
      wgt = (tp - t_prev) / jb.dt;
    else if (tp > t_m && tp <= t_next)
      wgt = 1.0 - (tp - t_m) / jb.dt;
    else
      continue;  // uniform over the workgroup
    const T w = T(wgt);
    for (int64_t xy = xy0 + threadIdx.x; xy < min(xy0 + kNodesPerBlock, nxy); xy += kThreads) {
      const int64_t idx = xy * jb.nz + k;
      const T ex = jb.F[0][idx], ey = jb.F[1][idx], ez = jb.F[2][idx];
      const T bx = jb.F[3][idx], by = jb.F[4][idx], bz = jb.F[5][idx];
      const T lab[6] = {g * ex + gb * by, g * ey - gb * bx, ez,
                        g * bx - gb * ey, g * by + gb * ex, bz};
#pragma unroll
      for (int f = 0; f < 6; ++f) out[f * ncell + int64_t(k) * nxy + xy] += w * lab[f];
    }
  }
}

// Particle records.  After a move the particle sits at x (in the box) with
// the momentum u that moved it by (v - v_gal) dt; its worldline over the
// step is the segment ending there, x(s) = x - (1 - s) (v - v_gal) dt at
// boosted time t_new - (1 - s) dt, along which the lab time
// t'/gamma + gamma beta z / c increases strictly.  A snapshot whose lab time
// lies in (t_lab(0), t_lab(1)] records the particle at that point: x, y,
// gamma z (lab plane), u_x, u_y, gamma (u_z + beta gamma_p).  Since
// |v| < c bounds the move, the end position's z alone rules out most
// particles in a step: only those whose possible lab-time window holds a
// snapshot time read their momentum.
template <typename T>
__device__ __forceinline__ double particle_z(const BtdJob<T> &jb, int64_t k) {
  if constexpr (sizeof(T) == 8) {
    return static_cast<const double *>(jb.p.z)[k];
  } else {
    const int iz = static_cast<const int *>(jb.p.x)[k] & (jb.nz - 1);
    return (double(iz) + double(static_cast<const float *>(jb.p.oz)[k])) * jb.dz;
  }
}

template <typename T>
__device__ __forceinline__ void particle_xy(const BtdJob<T> &jb, int64_t k, double x[2]) {
  if constexpr (sizeof(T) == 8) {
    x[0] = static_cast<const double *>(jb.p.x)[k];
    x[1] = static_cast<const double *>(jb.p.y)[k];
  } else {
    const int cell = static_cast<const int *>(jb.p.x)[k];
    const int iy = (cell >> jb.lz) & (jb.ny - 1);
    const int ix = cell >> (jb.lz + jb.ly);
    x[0] = (double(ix) + double(static_cast<const float *>(jb.p.ox)[k])) * jb.dx;
    x[1] = (double(iy) + double(static_cast<const float *>(jb.p.oy)[k])) * jb.dy;
  }
}

// snapshots j in [j0, j1] (clipped) may have t_lab0 + j dt_lab in (lo, hi]
// (inv_dt: 1 / dt_lab; the range is widened by one on each side, so its
// rounding does not matter: the callers test each candidate exactly)
__device__ __forceinline__ bool snapshot_range(double lo, double hi, double t_lab0, double inv_dt,
                                               int nsnap, int &j0, int &j1) {
  const double ja = (lo - t_lab0) * inv_dt, jb = (hi - t_lab0) * inv_dt;
  if (!(jb >= -1.0) || !(ja < double(nsnap))) return false;
  j0 = max(0, int(fmax(floor(ja), -1.0)));
  j1 = min(nsnap - 1, int(fmin(floor(jb), double(nsnap))) + 1);
  return j0 <= j1;
}

// The exact crossing test of particle k (end position z, lab time tb at
// the end of the step) against snapshots j0..j1, and its records.
template <typename T>
__device__ __forceinline__ void record_particle(const BtdJob<T> &jb, int64_t k, double z,
                                                double tb, double t_start, int j0, int j1,
                                                const double L[3]) {
#pragma clang fp contract(off)
  const double g = jb.gamma, gb = jb.gamma * jb.beta;
  const double u[3] = {double(static_cast<const T *>(jb.p.ux)[k]),
                       double(static_cast<const T *>(jb.p.uy)[k]),
                       double(static_cast<const T *>(jb.p.uz)[k])};
  const double gp = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  // (v - v_gal)_z with v_gal = (0, 0, -beta c); x and y only on a crossing
  const double step_z = (u[2] / gp + jb.beta) * jb.dt;
  const double ta = t_start + gb * (z - step_z);
  for (int j = j0; j <= j1; ++j) {
    const double tj = jb.t_lab0 + double(j) * jb.dt_lab;
    if (!(ta < tj && tj <= tb)) continue;
    const double step[3] = {u[0] / gp * jb.dt, u[1] / gp * jb.dt, step_z};
    const double s = (tj - ta) / (tb - ta);
    double x[3];
    particle_xy<T>(jb, k, x);
    x[2] = z;
    double q[3];
    for (int a = 0; a < 3; ++a) {
      q[a] = x[a] - (1.0 - s) * step[a];
      q[a] = q[a] - floor(q[a] / L[a]) * L[a];
    }
    const int slot = atomicAdd(jb.pcount + j, 1);
    if (slot >= jb.pcap) continue;
    T *o = jb.pvals + int64_t(j) * 6 * jb.pcap + slot;
    o[0] = T(q[0]);
    o[jb.pcap] = T(q[1]);
    o[2 * int64_t(jb.pcap)] = T(g * q[2]);
    o[3 * int64_t(jb.pcap)] = T(u[0]);
    o[4 * int64_t(jb.pcap)] = T(u[1]);
    o[5 * int64_t(jb.pcap)] = T(g * (u[2] + jb.beta * gp));
    if (jb.pids) jb.pids[int64_t(j) * jb.pcap + slot] = jb.p.id[k];
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_btd_particles(const BtdJob<T> *__restrict__ jobs) {
  // the crossing decisions are the plain double expressions
#pragma clang fp contract(off)
  BtdJob<T> jb = jobs[blockIdx.y];
  if (jb.pcap <= 0) return;
  jb.p.x = global_ptr(jb.p.x);
  jb.p.y = global_ptr(jb.p.y);
  jb.p.z = global_ptr(jb.p.z);
  jb.p.ox = global_ptr(jb.p.ox);
  jb.p.oy = global_ptr(jb.p.oy);
  jb.p.oz = global_ptr(jb.p.oz);
  jb.p.ux = global_ptr(jb.p.ux);
  jb.p.uy = global_ptr(jb.p.uy);
  jb.p.uz = global_ptr(jb.p.uz);
  jb.p.id = global_ptr(jb.p.id);
  jb.pvals = global_ptr(jb.pvals);
  jb.pids = global_ptr(jb.pids);
  jb.pcount = global_ptr(jb.pcount);
  const int m = *global_ptr(jb.level);
  const double t_new = jb.t0 + double(m) * jb.dt;
  const double g = jb.gamma, gb = jb.gamma * jb.beta;
  const double L[3] = {jb.nx * jb.dx, jb.ny * jb.dy, jb.nz * jb.dz};
  // |v| < c bounds the z move: gb (v_z + beta) dt lies below reach
  const double reach = fmax(gb * (jb.beta + 1.0), gb * (jb.beta - 1.0)) * jb.dt;
  const double inv_dt_lab = 1.0 / jb.dt_lab;
  const double t_end = t_new / g, t_start = (t_new - jb.dt) / g;
  // four particles per pass, their position loads issued together (the
  // prefilter is a few flops per particle: the pass waits on memory); the
  // few that pass the prefilter are compacted per wave in LDS, so that the
  // exact test runs with full lanes instead of a few lanes per pass
  constexpr int kBatch = 4;
  __shared__ int64_t cand_k[kThreads / 64][kBatch * 64];
  __shared__ double cand_z[kThreads / 64][kBatch * 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  // every lane of a wave runs the same number of passes (the compaction
  // needs all lanes): the loop bound is the wave's first lane's
  const int64_t first = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63);
  for (int64_t w0 = first; w0 < jb.p.n; w0 += kBatch * stride) {
    const int64_t k0 = w0 + lane;
    // unconditional loads (index clamped to the last particle), so that
    // all of them are in flight before the first is used
    double zs[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) zs[i] = particle_z<T>(jb, min(k0 + i * stride, jb.p.n - 1));
    int count = 0;
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int64_t k = k0 + i * stride;
      const double z = zs[i];
      const double tb = t_end + gb * z;
      // prefilter on z alone: no snapshot in (lowest possible t_lab(0), tb]
      const double ta_lo = t_start + gb * z - reach;
      bool pass = false;
      int j0, j1;
      if (k < jb.p.n && snapshot_range(ta_lo, tb, jb.t_lab0, inv_dt_lab, jb.nsnap, j0, j1)) {
        for (int j = j0; j <= j1; ++j) {
          const double tj = jb.t_lab0 + double(j) * jb.dt_lab;
          pass = pass || (ta_lo < tj && tj <= tb);
        }
      }
      const uint64_t mask = __ballot(pass);
      if (pass) {
        const int at = count + __popcll(mask & below);
        cand_k[wave][at] = k;
        cand_z[wave][at] = z;
      }
      count += __popcll(mask);
    }
    __builtin_amdgcn_wave_barrier();
    for (int c = lane; c < count; c += 64) {
      const double z = cand_z[wave][c];
      const double tb = t_end + gb * z;
      int j0, j1;
      snapshot_range(t_start + gb * z - reach, tb, jb.t_lab0, inv_dt_lab, jb.nsnap, j0, j1);
      record_particle<T>(jb, cand_k[wave][c], z, tb, t_start, j0, j1, L);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <typename T>
__global__ void k_btd_advance(const BtdJob<T> *__restrict__ jobs, int njobs) {
  for (int i = threadIdx.x; i < njobs; i += blockDim.x) *global_ptr(jobs[i].level) += 1;
}

}  // namespace

template <typename T>
void launch_btd(const BtdJob<T> *jobs, int njobs, int max_snap, int64_t max_nxy, hipStream_t s) {
  if (njobs <= 0 || max_snap <= 0) return;
  const unsigned tiles = unsigned((max_nxy + kNodesPerBlock - 1) / kNodesPerBlock);
  hipLaunchKernelGGL((k_btd<T>), dim3(tiles, unsigned(max_snap), unsigned(njobs)),
                     dim3(kThreads), 0, s, jobs);
  hipLaunchKernelGGL((k_btd_advance<T>), dim3(1), dim3(64), 0, s, jobs, njobs);
}

template <typename T>
void launch_btd_particles(const BtdJob<T> *jobs, int njobs, int64_t max_n, hipStream_t s) {
  if (njobs <= 0 || max_n <= 0) return;
  int64_t blocks = (max_n + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_btd_particles<T>), dim3(unsigned(blocks), unsigned(njobs)),
                     dim3(kThreads), 0, s, jobs);
}

template void launch_btd_particles<float>(const BtdJob<float> *, int, int64_t, hipStream_t);
template void launch_btd_particles<double>(const BtdJob<double> *, int, int64_t, hipStream_t);
template void launch_btd<float>(const BtdJob<float> *, int, int, int64_t, hipStream_t);
template void launch_btd<double>(const BtdJob<double> *, int, int, int64_t, hipStream_t);

}  // namespace galpic
