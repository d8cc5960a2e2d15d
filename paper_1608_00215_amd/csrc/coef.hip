// Galilean-PSATD coefficient table, built once per v_gal in double precision.
//
// Per half-spectrum mode with k != 0 (c = eps0 = 1), from the paper's
// coefficient block (C = cos(k dt), S = sin(k dt), nu = k.v_gal / k,
// theta = exp(i k.v_gal dt / 2), chi_1, chi_2, chi_3):
//
//   c0 = theta^2 C                         multiplies E and B
//   c1 = theta^2 S / k                     B gets -c1 ik x E, E gets +c1 ik x B
//   c2 = theta chi_1 / k^2                 multiplies ik x J in B
//   c3 = (i nu theta chi_1 - theta^2 S)/k  multiplies J in E
//   c4 = -chi_2 / k^2                      multiplies rho^{n+1} ik in E
//   c5 = +theta^2 chi_3 / k^2              multiplies rho^n ik in E
//
// The printed closed forms divide by 1 - nu^2 and by theta* - theta, which is
// 0/0 on every mode with k.v_gal = 0 and loses most digits when k is nearly
// parallel to a relativistic v_gal.  The same quantities are integrals over
// one step of the vacuum propagator against exp(i nu y), y = k tau in
// [0, phi = k dt] (the current is constant in the Galilean coordinates):
//
//   theta chi_1                 = int sin(y) e^{i nu y} dy
//   i nu theta chi_1 - theta^2 S = -int cos(y) e^{i nu y} dy
//   chi_2 D                     = int 2 sin^2(y/2) e^{i nu y} dy
//   chi_3 D                     = -int 2 (sin^2(phi/2) - sin^2(y/2)) e^{i nu y} dy
//   D                           = int e^{i nu y} dy
//
// Their integrands have no cancelling differences, so composite
// Gauss-Legendre quadrature (16 nodes per panel of length <= 1 in y) gives
// them to double rounding.  The 16-node rule is computed on the host by
// Newton iteration on the Legendre recurrence.
#include "kernels.hpp"

#include <cmath>

namespace galpic {
namespace {

constexpr int kGL = 16;

struct GLRule {
  double t[kGL];  // nodes on [0, 1]
  double w[kGL];  // weights on [0, 1]
};

GLRule make_rule() {
  GLRule r;
  const int n = kGL;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n + 0.5));  // initial guess
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    const double w = 2.0 / ((1.0 - x * x) * dp * dp);
    // map [-1, 1] -> [0, 1]
    r.t[i] = 0.5 * (1.0 - x);
    r.t[n - 1 - i] = 0.5 * (1.0 + x);
    r.w[i] = 0.5 * w;
    r.w[n - 1 - i] = 0.5 * w;
  }
  return r;
}

struct Cd {
  double re, im;
};
__device__ __forceinline__ Cd cmul(Cd a, Cd b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cd cdiv(Cd a, Cd b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

template <typename T>
__global__ __launch_bounds__(256) void k_coefficients(RunGeom g, const double *__restrict__ kt,
                                                      GLRule gl, CoefPtrs cp) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= g.nmode) return;
  const int iz = int(idx % g.nzh);
  const int iy = int((idx / g.nzh) % g.ny);
  const int ix = int(idx / (int64_t(g.nzh) * g.ny));
  const double kx = kt[ix];
  const double ky = kt[g.nx + iy];
  const double kz = kt[g.nx + g.ny + iz];
  const double k2 = kx * kx + ky * ky + kz * kz;
  const double dt = g.dt;
  Cd c[6];
  if (k2 == 0.0) {
    c[0] = {1.0, 0.0};
    c[1] = {dt, 0.0};
    c[2] = {0.5 * dt * dt, 0.0};
    c[3] = {-dt, 0.0};
    c[4] = {-dt * dt / 6.0, 0.0};
    c[5] = {-dt * dt / 3.0, 0.0};
  } else {
    const double k = sqrt(k2);
    const double kv = kx * g.vgal[0] + ky * g.vgal[1] + kz * g.vgal[2];
    const double phi = k * dt;
    const double nu = kv / k;
    const int panels = max(1, int(ceil(phi)));
    const double h = phi / panels;
    double sh_phi, ch_phi;
    sincos(0.5 * phi, &sh_phi, &ch_phi);
    const double s2phi = sh_phi * sh_phi;
    Cd A1 = {0, 0}, A2 = {0, 0}, A3 = {0, 0}, A4 = {0, 0}, D = {0, 0};
    for (int p = 0; p < panels; ++p) {
#pragma unroll 4
      for (int q = 0; q < kGL; ++q) {
        const double y = h * (double(p) + gl.t[q]);
        const double wq = h * gl.w[q];
        double sn, cn, sh, ch;
        sincos(nu * y, &sn, &cn);
        sincos(0.5 * y, &sh, &ch);
        const double siny = 2.0 * sh * ch;
        const double sh2 = sh * sh;
        const double cosy = 1.0 - 2.0 * sh2;
        const double f3 = 2.0 * sh2;
        const double f4 = 2.0 * (s2phi - sh2);
        const double er = wq * cn, ei = wq * sn;
        A1.re += siny * er; A1.im += siny * ei;
        A2.re += cosy * er; A2.im += cosy * ei;
        A3.re += f3 * er;   A3.im += f3 * ei;
        A4.re += f4 * er;   A4.im += f4 * ei;
        D.re += er;         D.im += ei;
      }
    }
    double st, ct;
    sincos(kv * dt, &st, &ct);
    const Cd theta2 = {ct, st};
    double S, C;
    sincos(phi, &S, &C);
    const Cd chi2 = cdiv(A3, D);
    const Cd chi3 = cdiv(A4, D);  // = -chi_3
    c[0] = {theta2.re * C, theta2.im * C};
    c[1] = {theta2.re * S / k, theta2.im * S / k};
    c[2] = {A1.re / k2, A1.im / k2};
    c[3] = {-A2.re / k, -A2.im / k};
    c[4] = {-chi2.re / k2, -chi2.im / k2};
    const Cd t3 = cmul(theta2, chi3);
    c[5] = {-t3.re / k2, -t3.im / k2};
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
    static_cast<Cx<T> *>(cp.c[i])[idx] = cx(T(c[i].re), T(c[i].im));
}

}  // namespace

template <typename T>
void launch_coefficients(const RunGeom &g, const double *kt, const CoefPtrs &cp, hipStream_t s) {
  static const GLRule rule = make_rule();
  const unsigned blocks = unsigned((g.nmode + 255) / 256);
  hipLaunchKernelGGL((k_coefficients<T>), dim3(blocks), dim3(256), 0, s, g, kt, rule, cp);
}

template void launch_coefficients<float>(const RunGeom &, const double *, const CoefPtrs &,
                                         hipStream_t);
template void launch_coefficients<double>(const RunGeom &, const double *, const CoefPtrs &,
                                          hipStream_t);

}  // namespace galpic
