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

template void launch_btd<float>(const BtdJob<float> *, int, int, int64_t, hipStream_t);
template void launch_btd<double>(const BtdJob<double> *, int, int, int64_t, hipStream_t);

}  // namespace galpic
