// C ABI of the Galilean-PSATD step (declared in include/galpic.h).
//
// Host-side orchestration only: validation, device allocation, the order of
// kernel launches, the rho^n / rho^{n+1} buffer rotation, per-kernel event
// timing and HIP graph capture.  All arithmetic of the step runs in the
// kernels.
#include "galpic.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace galpic;

namespace {

thread_local std::string g_err;

gp_status fail(gp_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

}  // namespace

void galpic::set_last_error(const std::string &msg) { g_err = msg; }

namespace {

#define GP_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(GP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define GP_TRY(expr)              \
  do {                            \
    gp_status st_ = (expr);       \
    if (st_ != GP_OK) return st_; \
  } while (0)

gp_status check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return GP_OK;
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Kernel stages of a step (names: gp_stage_name).
enum {
  kStZero = 0, kStSort, kStDeposit, kStFused, kStFwdZ, kStFwdY, kStFwdX, kStUpdate, kStInvX,
  kStInvY, kStInvZ, kStGather, kStBtd, kStSlab, kStSlabEB, kStReduce, kNStages
};
static_assert(kNStages == GP_N_STAGES, "stage count");
const char *const kStageNames[kNStages] = {
    "zero_sources", "sort",      "deposit",   "fused_push_deposit", "fft_fwd_z", "fft_fwd_y",
    "fft_fwd_x",    "update",    "fft_inv_x", "fft_inv_y",          "fft_inv_z", "gather_push",
    "btd",          "slab_copy", "slab_fft_fwd_eb", "region_reduce"};

enum { kReal = 10, kSpec = 11 };
// real[] slots: 0-2 E, 3-5 B, 6-8 J, 9 rho
// spec[] slots: 0-2 E^, 3-5 B^, 6-8 J^, 9-10 rho buffers (rotating)

struct Run {
  RunGeom g{};
  TileGeom tg{};
  void *real[kReal] = {};
  void *spec[kSpec] = {};
  void *coef[6] = {};
  void *scratch[6] = {};
  int stencil[3] = {};          // field-solve stencil order per axis (0: spectral)
  double *kd = nullptr;         // wavenumbers x | y | z (nx + ny + nz/2+1), double
  void *kt = nullptr;           // the same in the run's real type (kd for FP64)
  int rho_old = 9;              // spec slot holding rho^n; the other holds rho^{n+1}
  int resort_div = 64;          // re-sort when > n / resort_div particles went global
  int flush = 1;                // 1: tile regions by float atomics; 2: region buffer
  void *regbuf = nullptr;       // flush 2: tiles x 4 x region values (freed with the sort)
  PartPtrs parts{};
  bool bound = false;
  SortBufs sb{};
  std::vector<void *> sort_allocs;  // freed on re-binding
  bool src_real_ready = false;  // J, rho deposited since the last forward FFT
  bool src_spec_ready = false;  // J^, rho^{n+1} ready for the update
  bool eb_real_ready = true;    // real E, B match the spectral state
  // lab-frame snapshots (off while btd_nsnap == 0)
  int btd_nsnap = 0;
  double btd_t_lab0 = 0, btd_dt_lab = 0, btd_t0 = 0;
  void *btd_out = nullptr;      // caller's buffer
  int btd_pcap = 0;             // particle records per snapshot (0: off)
  void *btd_pvals = nullptr;    // caller's buffers for them
  int64_t *btd_pids = nullptr;
  int *btd_pcount = nullptr;
};

struct StageRec {
  int stage;
  hipEvent_t a, b;
};

// Device tables of the batched launches.  FieldSet tables hold one entry per
// run in class order: runs of one grid shape sit next to each other, so one
// launch covers a class (a slice of the table) and a set-up call covers one
// run (a slice of one).
enum {
  kTabFwdZ0, kTabFwdZ1,           // real J, rho -> J^, rho^{n+1} (per rho parity)
  kTabFwdYX0, kTabFwdYX1,         // in place on J^, rho^{n+1}
  kTabInvX, kTabInvY, kTabInvZ,   // E^, B^ -> scratch -> scratch -> real E, B
  kTabEBZ, kTabEBYX,              // real E, B -> E^, B^ (setting fields)
  kTabRhoZ0, kTabRhoZ1,           // real rho -> rho^n (binding particles)
  kTabRhoYX0, kTabRhoYX1,
  kNTab
};

struct Class {
  RunGeom g;  // grid shape and spacing shared by the class
  int first;  // first class-order position
  int count;
};

struct Tables {
  void *dev = nullptr;                // one device allocation ...
  std::vector<unsigned char> host;    // ... mirrored on the host
  size_t fs[kNTab] = {};              // byte offsets of the FieldSet tables
  size_t upd[2] = {};                 // UpdatePtrs per rho parity (class order)
  size_t zero = 0;                    // ZeroSeg of J and rho (four per run)
  size_t jobs = 0;                    // PartJob per run (run order)
  size_t btd = 0;                     // BtdJob of the recording runs (compact)
  size_t bytes = 0;
  std::vector<Class> classes;
  std::vector<int> pos;               // run -> class-order position
  size_t max_zero16 = 0;
  PartBatch batch{};
  int btd_count = 0;                  // recording runs
  int btd_max_snap = 0;
  int64_t btd_max_nxy = 0;
  int btd_pjobs = 0;                  // recording runs that also record particles
  int64_t btd_max_n = 0;
  std::vector<int> btd_pos;           // run -> position in the BtdJob table, or -1
  int *btd_level = nullptr;           // device level counters, one per run
};

}  // namespace

struct gp_ctx {
  int precision = GP_FP64;
  int order = 1;
  size_t real_size = 8;  // bytes of one real value
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<Run> runs;
  std::vector<void *> allocs;
  void *tw = nullptr;
  double *d_sum = nullptr;
  // captured graphs: first deposit; per rho parity: field cycle + fused
  // particle pass; field cycle + final gather-push
  hipGraphExec_t g_first = nullptr;
  hipGraphExec_t g_mid[2] = {nullptr, nullptr};
  hipGraphExec_t g_last[2] = {nullptr, nullptr};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  bool stage_timing = false;
  std::vector<StageRec> stage_recs;
  Tables tab;
  bool current_correction = false;
  // slab field solve (gp_set_local_slabs): the slabs' local grids are the
  // runs of a context of their own, slab s of run r at r * n_slabs + s
  gp_ctx *slab = nullptr;
  gp_ctx *timing_parent = nullptr;  // a slab context records its stages there
  int n_slabs = 0;
  int guard = 0;
  int src_mask = kMaskHeld;  // x-pass mask of the sources' forward transform
  bool no_hold = false;      // the update advances every mode
  std::vector<void *> slab_allocs;
  void *slab_copy = nullptr;  // SlabCopy<T>[runs * n_slabs]
  void *slab_sum = nullptr;   // SlabSum<T>[runs]
  double *slab_sums = nullptr;
  int64_t slab_max_cells = 0, slab_max_win = 0, slab_max_owned = 0;
  int device = 0;  // the device current at gp_init_grid
};

namespace {

gp_status dev_alloc(std::vector<void *> &list, size_t bytes, void **out) {
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(GP_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  list.push_back(p);
  *out = p;
  return GP_OK;
}

void drop_graphs(gp_ctx *c) {
  auto drop = [](hipGraphExec_t &gx) {
    if (gx) (void)hipGraphExecDestroy(gx);
    gx = nullptr;
  };
  drop(c->g_first);
  for (int k = 0; k < 2; ++k) {
    drop(c->g_mid[k]);
    drop(c->g_last[k]);
  }
}

size_t real_bytes(const gp_ctx *c, const Run &r) { return size_t(r.g.ncell) * c->real_size; }
size_t spec_bytes(const gp_ctx *c, const Run &r) {
  return size_t(r.g.nmode) * 2 * c->real_size;
}

gp_status validate_desc(const gp_grid_desc &d, int i) {
  const std::string w = "run " + std::to_string(i) + ": ";
  if (!is_pow2(d.nx) || !is_pow2(d.ny) || !is_pow2(d.nz))
    return fail(GP_ERR_ARG, w + "nx, ny, nz must be powers of two");
  if (d.nx < 8 || d.ny < 8 || d.nz < 8 || d.nx > 1024 || d.ny > 1024 || d.nz > 1024)
    return fail(GP_ERR_ARG, w + "nx, ny, nz must lie in [8, 1024]");
  if (!(d.dx > 0) || !(d.dy > 0) || !(d.dz > 0) || !(d.dt > 0) || !std::isfinite(d.dx) ||
      !std::isfinite(d.dy) || !std::isfinite(d.dz) || !std::isfinite(d.dt))
    return fail(GP_ERR_ARG, w + "dx, dy, dz, dt must be positive and finite");
  if (d.shape_order != 1 && d.shape_order != 3)
    return fail(GP_ERR_ARG, w + "shape_order must be 1 or 3");
  if (d.precision != GP_FP64 && d.precision != GP_MIXED)
    return fail(GP_ERR_ARG, w + "precision must be GP_FP64 or GP_MIXED");
  if (int64_t(d.nx) * d.ny * d.nz > (int64_t(1) << 30))
    return fail(GP_ERR_ARG, w + "grid too large (at most 2^30 cells)");
  const int n[3] = {d.nx, d.ny, d.nz};
  for (int a = 0; a < 3; ++a)
    if (d.tile[a] != 0 && (!is_pow2(d.tile[a]) || d.tile[a] > 8 || d.tile[a] > n[a]))
      return fail(GP_ERR_ARG, w + "tile sizes must be 0 or powers of two <= min(8, grid)");
  if (d.resort_div < 0) return fail(GP_ERR_ARG, w + "resort_div must be >= 0");
  if (d.flush < 0 || d.flush > 2) return fail(GP_ERR_ARG, w + "flush must be 0, 1 or 2");
  for (int a = 0; a < 3; ++a)
    if (d.stencil[a] != 0 && (d.stencil[a] < 2 || d.stencil[a] > 64 || d.stencil[a] % 2))
      return fail(GP_ERR_ARG, w + "stencil orders must be 0 or even in [2, 64]");
  return GP_OK;
}

// Wavenumbers of one axis in transform index order (index n/2 stands for
// -n/2; its modes are held at zero): the exact k = 2 pi s / (n d), or for
// an even stencil order p = 2M the symbol of the centered difference
// (D f)_i = (1/d) sum_{l=1}^{M} a_l (f_{i+l} - f_{i-l}) acting on exp(ikx),
// [k] = (2/d) sum_l a_l sin(l k d), with the weights that make it exact for
// polynomials of degree 2M: a_l = (-1)^(l+1) r_l / l,
// r_l = (M!)^2 / ((M-l)! (M+l)!) = prod_{j<l} (M - j) / (M + 1 + j).
void axis_wavenumbers(int n, double d, int order, int count, double *out) {
  const int M = order / 2;
  std::vector<double> a(M + 1, 0.0);
  double r = 1.0;
  for (int l = 1; l <= M; ++l) {
    r *= double(M - (l - 1)) / double(M + l);
    a[l] = (l % 2 ? 1.0 : -1.0) * r / double(l);
  }
  for (int i = 0; i < count; ++i) {
    const int s = i < n / 2 ? i : i - n;
    const double k = 2.0 * kPi * double(s) / (double(n) * d);
    if (order == 0) {
      out[i] = k;
      continue;
    }
    double sum = 0.0;
    for (int l = M; l >= 1; --l) sum += a[l] * std::sin(double(l) * k * d);
    out[i] = 2.0 * sum / d;
  }
}

// The run's wavenumber tables on the device (double, and float for the
// mixed update).  Synchronising.
gp_status upload_wavenumbers(gp_ctx *c, Run &r) {
  const RunGeom &g = r.g;
  const int cnt = g.nx + g.ny + g.nzh;
  std::vector<double> kd(cnt);
  axis_wavenumbers(g.nx, g.dx, r.stencil[0], g.nx, kd.data());
  axis_wavenumbers(g.ny, g.dy, r.stencil[1], g.ny, kd.data() + g.nx);
  axis_wavenumbers(g.nz, g.dz, r.stencil[2], g.nzh, kd.data() + g.nx + g.ny);
  const size_t dbytes = size_t(cnt) * sizeof(double);
  const bool mixed = c->precision != GP_FP64;
  std::vector<float> kf(mixed ? cnt : 0);
  for (int i = 0; i < int(kf.size()); ++i) kf[i] = float(kd[i]);
  void *p = nullptr;
  GP_TRY(dev_alloc(c->allocs, dbytes + kf.size() * sizeof(float), &p));
  r.kd = static_cast<double *>(p);
  r.kt = mixed ? static_cast<void *>(static_cast<char *>(p) + dbytes) : p;
  if (hipMemcpyAsync(r.kd, kd.data(), dbytes, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      (mixed && hipMemcpyAsync(r.kt, kf.data(), kf.size() * sizeof(float),
                               hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(GP_ERR_HIP, "wavenumber upload failed");
  return GP_OK;
}

template <typename T>
Cx<T> *S(const Run &r, int slot) {
  return static_cast<Cx<T> *>(r.spec[slot]);
}
template <typename T>
T *R(const Run &r, int slot) {
  return static_cast<T *>(r.real[slot]);
}

template <typename T>
GridPtrs<T> grid_ptrs(const Run &r) {
  GridPtrs<T> g;
  for (int a = 0; a < 3; ++a) {
    g.E[a] = R<T>(r, a);
    g.B[a] = R<T>(r, 3 + a);
    g.J[a] = R<T>(r, 6 + a);
  }
  g.rho = R<T>(r, 9);
  return g;
}

// Records device events around one stage when timing is on.
struct Stamp {
  gp_ctx *c;  // the context whose record list takes the stage
  hipStream_t stream;
  StageRec rec{};
  bool on;
  Stamp(gp_ctx *ctx, int stage)
      : c(ctx->timing_parent ? ctx->timing_parent : ctx), stream(ctx->stream),
        on(c->stage_timing) {
    if (!on) return;
    rec.stage = stage;
    if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess) {
      on = false;
      return;
    }
    (void)hipEventRecord(rec.a, stream);
  }
  ~Stamp() {
    if (!on) return;
    (void)hipEventRecord(rec.b, stream);
    c->stage_recs.push_back(rec);
  }
};

// ---- device tables ---------------------------------------------------------
const FieldSet *fs_tab(gp_ctx *c, int kind, int pos) {
  return reinterpret_cast<const FieldSet *>(static_cast<char *>(c->tab.dev) + c->tab.fs[kind]) +
         pos;
}
template <typename T>
const UpdatePtrs<T> *upd_tab(gp_ctx *c, int parity, int pos) {
  return reinterpret_cast<const UpdatePtrs<T> *>(static_cast<char *>(c->tab.dev) +
                                                 c->tab.upd[parity]) +
         pos;
}
template <typename T>
const PartJob<T> *job_tab(gp_ctx *c) {
  return reinterpret_cast<const PartJob<T> *>(static_cast<char *>(c->tab.dev) + c->tab.jobs);
}
const ZeroSeg *zero_tab(gp_ctx *c) {
  return reinterpret_cast<const ZeroSeg *>(static_cast<char *>(c->tab.dev) + c->tab.zero);
}

template <typename V>
V *host_at(gp_ctx *c, size_t off, int i) {
  return reinterpret_cast<V *>(c->tab.host.data() + off) + i;
}

size_t align16(size_t n) { return (n + 15) & ~size_t(15); }

bool same_class(const RunGeom &a, const RunGeom &b) {
  return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.dx == b.dx && a.dy == b.dy &&
         a.dz == b.dz;
}

// Classes, table layout and the grid-side tables (fixed once the grids are
// allocated); the particle jobs are filled when particles are bound.
template <typename T>
gp_status build_tables(gp_ctx *c) {
  Tables &t = c->tab;
  const int n = int(c->runs.size());
  t.classes.clear();
  t.pos.assign(n, -1);
  std::vector<int> order;
  for (int i = 0; i < n; ++i) {
    if (t.pos[i] >= 0) continue;
    Class k{c->runs[i].g, int(order.size()), 0};
    for (int j = i; j < n; ++j)
      if (t.pos[j] < 0 && same_class(c->runs[j].g, c->runs[i].g)) {
        t.pos[j] = int(order.size());
        order.push_back(j);
        ++k.count;
      }
    t.classes.push_back(k);
  }
  size_t off = 0;
  for (int k = 0; k < kNTab; ++k) {
    t.fs[k] = off;
    off = align16(off + size_t(n) * sizeof(FieldSet));
  }
  for (int k = 0; k < 2; ++k) {
    t.upd[k] = off;
    off = align16(off + size_t(n) * sizeof(UpdatePtrs<T>));
  }
  t.zero = off;
  off = align16(off + size_t(4 * n) * sizeof(ZeroSeg));
  t.jobs = off;
  off = align16(off + size_t(n) * sizeof(PartJob<T>));
  t.btd = off;
  off = align16(off + size_t(n) * sizeof(BtdJob<T>));
  t.bytes = off;
  t.host.assign(off, 0);
  GP_TRY(dev_alloc(c->allocs, off, &t.dev));
  {
    void *lv = nullptr;
    GP_TRY(dev_alloc(c->allocs, size_t(n) * sizeof(int), &lv));
    t.btd_level = static_cast<int *>(lv);
    t.btd_pos.assign(n, -1);
  }
  t.max_zero16 = 0;
  for (int i = 0; i < n; ++i) {
    const Run &r = c->runs[i];
    const int q = t.pos[i];
    auto set = [&](int kind, int nf, auto in, auto out) {
      FieldSet *fs = host_at<FieldSet>(c, t.fs[kind], q);
      for (int f = 0; f < nf; ++f) {
        fs->in[f] = in(f);
        fs->out[f] = out(f);
      }
    };
    for (int par = 0; par < 2; ++par) {
      // parity par: rho^n in spec slot 9 + par, rho^{n+1} in the other
      void *src[4] = {r.spec[6], r.spec[7], r.spec[8], r.spec[10 - par]};
      set(kTabFwdZ0 + par, 4, [&](int f) { return r.real[6 + f]; },
          [&](int f) { return src[f]; });
      set(kTabFwdYX0 + par, 4, [&](int f) { return src[f]; }, [&](int f) { return src[f]; });
      set(kTabRhoZ0 + par, 1, [&](int) { return r.real[9]; },
          [&](int) { return r.spec[9 + par]; });
      set(kTabRhoYX0 + par, 1, [&](int) { return r.spec[9 + par]; },
          [&](int) { return r.spec[9 + par]; });
      UpdatePtrs<T> *u = host_at<UpdatePtrs<T>>(c, t.upd[par], q);
      for (int a = 0; a < 3; ++a) {
        u->E[a] = S<T>(r, a);
        u->B[a] = S<T>(r, 3 + a);
        u->J[a] = S<T>(r, 6 + a);
      }
      u->rho_old = S<T>(r, 9 + par);
      u->rho_new = S<T>(r, 10 - par);
      for (int k = 0; k < 6; ++k) u->coef[k] = static_cast<const Cx<T> *>(r.coef[k]);
      const T *kt = static_cast<const T *>(r.kt);
      u->k[0] = kt;
      u->k[1] = kt + r.g.nx;
      u->k[2] = kt + r.g.nx + r.g.ny;
    }
    set(kTabInvX, 6, [&](int f) { return r.spec[f]; }, [&](int f) { return r.scratch[f]; });
    set(kTabInvY, 6, [&](int f) { return r.scratch[f]; }, [&](int f) { return r.scratch[f]; });
    set(kTabInvZ, 6, [&](int f) { return r.scratch[f]; }, [&](int f) { return r.real[f]; });
    set(kTabEBZ, 6, [&](int f) { return r.real[f]; }, [&](int f) { return r.spec[f]; });
    set(kTabEBYX, 6, [&](int f) { return r.spec[f]; }, [&](int f) { return r.spec[f]; });
    for (int q = 0; q < 4; ++q) {  // J and rho
      ZeroSeg *z = host_at<ZeroSeg>(c, t.zero, 4 * i + q);
      z->p = r.real[6 + q];
      z->n16 = real_bytes(c, r) / 16;
      if (z->n16 > t.max_zero16) t.max_zero16 = z->n16;
    }
  }
  return GP_OK;
}

// Per-run scalars of the update tables (v_gal, dt, correction flag).
template <typename T>
void fill_update_scalars(gp_ctx *c) {
  for (size_t i = 0; i < c->runs.size(); ++i) {
    const Run &r = c->runs[i];
    for (int par = 0; par < 2; ++par) {
      UpdatePtrs<T> *u = host_at<UpdatePtrs<T>>(c, c->tab.upd[par], c->tab.pos[i]);
      for (int a = 0; a < 3; ++a) u->vgal[a] = r.g.vgal[a];
      u->dt = r.g.dt;
      u->correct = c->current_correction ? 1 : 0;
      u->no_hold = c->no_hold ? 1 : 0;
    }
  }
}

// Per-run particle jobs (pointers, geometry with v_gal, sort buffers).
template <typename T>
void fill_jobs(gp_ctx *c) {
  Tables &t = c->tab;
  PartBatch &b = t.batch;
  b = PartBatch{};
  b.order = c->order;
  b.njobs = int(c->runs.size());
  b.fixed_geom = c->order == 3 ? 1 : 0;
  for (size_t i = 0; i < c->runs.size(); ++i) {
    const Run &r = c->runs[i];
    PartJob<T> *j = host_at<PartJob<T>>(c, t.jobs, int(i));
    j->g = r.g;
    j->tg = r.tg;
    j->p = r.parts;
    j->gr = grid_ptrs<T>(r);
    j->sb = r.sb;
    j->block0 = b.nblocks;
    j->regbuf = static_cast<T *>(r.regbuf);
    j->resort_threshold = int(r.parts.n / r.resort_div);
    b.nblocks += r.tg.n_tiles;
    if (r.parts.n > b.max_n) b.max_n = r.parts.n;
    const int64_t cells = int64_t(r.tg.n_tiles) << r.tg.lcpt;
    if (cells > b.max_cells) b.max_cells = cells;
    if (r.tg.n_tiles > b.max_tiles) b.max_tiles = r.tg.n_tiles;
    if (r.regbuf) b.any_regbuf = 1;
    if (!default_cubic_tiles(r.tg, sizeof(T))) b.fixed_geom = 0;
    for (int m = 0; m < 4; ++m) {
      const size_t l = particle_lds_bytes<T>(m, r.tg);
      if (l > b.lds[m]) b.lds[m] = l;
    }
  }
}

// BtdJob entries of the runs that record lab-frame snapshots.
template <typename T>
void fill_btd_jobs(gp_ctx *c) {
  Tables &t = c->tab;
  t.btd_count = 0;
  t.btd_max_snap = 0;
  t.btd_max_nxy = 0;
  t.btd_pjobs = 0;
  t.btd_max_n = 0;
  for (size_t i = 0; i < c->runs.size(); ++i) {
    Run &r = c->runs[i];
    t.btd_pos[i] = -1;
    if (r.btd_nsnap <= 0) continue;
    BtdJob<T> *b = host_at<BtdJob<T>>(c, t.btd, t.btd_count);
    for (int f = 0; f < 6; ++f) b->F[f] = static_cast<const T *>(r.real[f]);
    b->out = static_cast<T *>(r.btd_out);
    b->level = t.btd_level + i;
    b->nx = r.g.nx;
    b->ny = r.g.ny;
    b->nz = r.g.nz;
    b->nsnap = r.btd_nsnap;
    b->t_lab0 = r.btd_t_lab0;
    b->dt_lab = r.btd_dt_lab;
    b->t0 = r.btd_t0;
    b->dt = r.g.dt;
    b->dz = r.g.dz;
    b->beta = -r.g.vgal[2];
    b->gamma = 1.0 / std::sqrt(1.0 - b->beta * b->beta);
    b->p = r.parts;
    b->lx = r.g.lx;
    b->ly = r.g.ly;
    b->lz = r.g.lz;
    b->dx = r.g.dx;
    b->dy = r.g.dy;
    b->pcap = r.bound ? r.btd_pcap : 0;
    b->pvals = static_cast<T *>(r.btd_pvals);
    b->pids = r.btd_pids;
    b->pcount = r.btd_pcount;
    if (b->pcap > 0) {
      ++t.btd_pjobs;
      t.btd_max_n = std::max(t.btd_max_n, r.parts.n);
    }
    t.btd_pos[i] = t.btd_count++;
    t.btd_max_snap = std::max(t.btd_max_snap, r.btd_nsnap);
    t.btd_max_nxy = std::max(t.btd_max_nxy, int64_t(r.g.nx) * r.g.ny);
  }
}

template <typename T>
const BtdJob<T> *btd_tab(gp_ctx *c, int pos) {
  return reinterpret_cast<const BtdJob<T> *>(static_cast<char *>(c->tab.dev) + c->tab.btd) + pos;
}

gp_status upload_tables(gp_ctx *c) {
  GP_HIP(hipMemcpyAsync(c->tab.dev, c->tab.host.data(), c->tab.bytes, hipMemcpyHostToDevice,
                        c->stream));
  GP_HIP(hipStreamSynchronize(c->stream));
  return GP_OK;
}

// ---- launch sequences --------------------------------------------------------
// Forward 3D FFT of the run at class-order position pos (or a whole class:
// count runs) through a pair of tables.
template <typename T>
void fft_forward(gp_ctx *c, int tab_z, int tab_yx, int nf, int pos, int count,
                 const RunGeom &g, int mask = kMaskHeld) {
  const Cx<T> *tw = static_cast<const Cx<T> *>(c->tw);
  launch_r2c_z<T>(fs_tab(c, tab_z, pos), count, nf, g, tw, c->stream);
  launch_c2c<T>(fs_tab(c, tab_yx, pos), count, nf, g, 1, false, kMaskNone, tw, c->stream);
  launch_c2c<T>(fs_tab(c, tab_yx, pos), count, nf, g, 0, false, mask, tw, c->stream);
}

// Inverse 3D FFT of E^, B^ into real E, B (via the scratch spectra).
template <typename T>
void fft_inverse(gp_ctx *c, int pos, int count, const RunGeom &g) {
  const Cx<T> *tw = static_cast<const Cx<T> *>(c->tw);
  launch_c2c<T>(fs_tab(c, kTabInvX, pos), count, 6, g, 0, true, kMaskNone, tw, c->stream);
  launch_c2c<T>(fs_tab(c, kTabInvY, pos), count, 6, g, 1, true, kMaskNone, tw, c->stream);
  launch_c2r_z<T>(fs_tab(c, kTabInvZ, pos), count, 6, g, tw, c->stream);
}

// The lab-frame records of the particles the last particle pass moved.
template <typename T>
void enqueue_btd_particles(gp_ctx *c) {
  if (c->tab.btd_pjobs == 0) return;
  Stamp s(c, kStBtd);
  launch_btd_particles<T>(btd_tab<T>(c, 0), c->tab.btd_count, c->tab.btd_max_n, c->stream);
}

// Zero J and rho, sort if flagged, then deposit (mode kPartDeposit) or run
// the fused gather-push + deposit (kPartFused), for every run at once.
template <typename T>
void enqueue_sources(gp_ctx *c, int mode) {
  {
    Stamp s(c, kStZero);
    launch_zero_segments(zero_tab(c), 4 * int(c->runs.size()), c->tab.max_zero16, c->stream);
  }
  {
    Stamp s(c, kStSort);
    launch_sort<T>(job_tab<T>(c), c->tab.batch, c->stream);
  }
  {
    Stamp s(c, mode == kPartFused ? kStFused : kStDeposit);
    launch_particles<T>(mode, job_tab<T>(c), c->tab.batch, 1.0, c->stream);
  }
  if (c->tab.batch.any_regbuf) {
    Stamp s(c, kStReduce);
    launch_region_reduce<T>(job_tab<T>(c), c->tab.batch, c->stream);
  }
  enqueue_btd_particles<T>(c);
}

// all runs rotate their rho buffers together
int rho_parity(const gp_ctx *c) { return c->runs[0].rho_old - 9; }

// rho^n in slot 9 + par for every run of c and of its slab context
void set_rho_parity(gp_ctx *c, int par) {
  for (auto &r : c->runs) r.rho_old = 9 + par;
  if (c->slab)
    for (auto &r : c->slab->runs) r.rho_old = 9 + par;
}

template <typename T>
const SlabCopy<T> *slab_copy_tab(gp_ctx *c) {
  return static_cast<const SlabCopy<T> *>(c->slab_copy);
}
template <typename T>
const SlabSum<T> *slab_sum_tab(gp_ctx *c) {
  return static_cast<const SlabSum<T> *>(c->slab_sum);
}

// Slab solve: the grid sums of J and rho, then the windows of fields
// f0 .. f0 + nf - 1 into the slabs (J and rho less their means).
template <typename T>
void slab_windows(gp_ctx *c, int f0, int nf) {
  Stamp s(c, kStSlab);
  launch_zero(c->slab_sums, 4 * c->runs.size() * sizeof(double), c->stream);
  launch_slab_sums<T>(slab_sum_tab<T>(c), int(c->runs.size()), c->slab_max_cells, c->stream);
  launch_slab_window<T>(slab_copy_tab<T>(c), int(c->slab->runs.size()), f0, nf,
                        c->slab_max_win, c->stream);
}

// Slab solve: rho^n of every slab from the runs' current real rho.
template <typename T>
void slab_init_rho(gp_ctx *c) {
  gp_ctx *sc = c->slab;
  slab_windows<T>(c, 9, 1);
  const int par = rho_parity(sc);
  for (const Class &k : sc->tab.classes)
    fft_forward<T>(sc, kTabRhoZ0 + par, kTabRhoYX0 + par, 1, k.first, k.count, k.g,
                   sc->src_mask);
}

template <typename T>
void enqueue_fft_fwd(gp_ctx *c);

// Slab solve, forward half: windows of E, B, J, rho, and their transforms on
// the slabs' local grids (E, B with nothing held, the sources with their
// Nyquist planes held).
template <typename T>
void slab_forward(gp_ctx *c) {
  gp_ctx *sc = c->slab;
  slab_windows<T>(c, 0, 10);
  {
    Stamp s(c, kStSlabEB);
    for (const Class &k : sc->tab.classes)
      fft_forward<T>(sc, kTabEBZ, kTabEBYX, 6, k.first, k.count, k.g, kMaskNone);
  }
  enqueue_fft_fwd<T>(sc);
}

template <typename T>
void enqueue_fft_fwd(gp_ctx *c) {
  if (c->slab) {
    slab_forward<T>(c);
    return;
  }
  const Cx<T> *tw = static_cast<const Cx<T> *>(c->tw);
  const int par = rho_parity(c);
  {
    Stamp s(c, kStFwdZ);
    for (const Class &k : c->tab.classes)
      launch_r2c_z<T>(fs_tab(c, kTabFwdZ0 + par, k.first), k.count, 4, k.g, tw, c->stream);
  }
  {
    Stamp s(c, kStFwdY);
    for (const Class &k : c->tab.classes)
      launch_c2c<T>(fs_tab(c, kTabFwdYX0 + par, k.first), k.count, 4, k.g, 1, false, kMaskNone, tw,
                    c->stream);
  }
  {
    Stamp s(c, kStFwdX);
    for (const Class &k : c->tab.classes)
      launch_c2c<T>(fs_tab(c, kTabFwdYX0 + par, k.first), k.count, 4, k.g, 0, false, c->src_mask, tw,
                    c->stream);
  }
}

template <typename T>
void enqueue_update(gp_ctx *c) {
  if (c->slab) {  // the slabs' update; the run's rho roles turn with theirs
    enqueue_update<T>(c->slab);
    for (auto &r : c->runs) r.rho_old = r.rho_old == 9 ? 10 : 9;
    return;
  }
  Stamp s(c, kStUpdate);
  const int par = rho_parity(c);
  for (const Class &k : c->tab.classes)
    launch_update<T>(k.g, upd_tab<T>(c, par, k.first), k.count, c->stream);
  for (auto &r : c->runs) r.rho_old = r.rho_old == 9 ? 10 : 9;
}

template <typename T>
void enqueue_fft_inv(gp_ctx *c) {
  if (c->slab) {  // the slabs' inverse, then their owned planes into E, B
    enqueue_fft_inv<T>(c->slab);
    Stamp s(c, kStSlab);
    launch_slab_interior<T>(slab_copy_tab<T>(c), int(c->slab->runs.size()), c->slab_max_owned,
                            c->stream);
    return;
  }
  const Cx<T> *tw = static_cast<const Cx<T> *>(c->tw);
  {
    Stamp s(c, kStInvX);
    for (const Class &k : c->tab.classes)
      launch_c2c<T>(fs_tab(c, kTabInvX, k.first), k.count, 6, k.g, 0, true, kMaskNone, tw,
                    c->stream);
  }
  {
    Stamp s(c, kStInvY);
    for (const Class &k : c->tab.classes)
      launch_c2c<T>(fs_tab(c, kTabInvY, k.first), k.count, 6, k.g, 1, true, kMaskNone, tw,
                    c->stream);
  }
  {
    Stamp s(c, kStInvZ);
    for (const Class &k : c->tab.classes)
      launch_c2r_z<T>(fs_tab(c, kTabInvZ, k.first), k.count, 6, k.g, tw, c->stream);
  }
}

template <typename T>
void enqueue_push(gp_ctx *c, double dt_factor) {
  Stamp s(c, kStGather);
  launch_particles<T>(kPartPush, job_tab<T>(c), c->tab.batch, dt_factor, c->stream);
}

// The current real E, B of every recording run as its next level.
template <typename T>
void enqueue_btd(gp_ctx *c) {
  if (c->tab.btd_count == 0) return;
  Stamp s(c, kStBtd);
  launch_btd<T>(btd_tab<T>(c, 0), c->tab.btd_count, c->tab.btd_max_snap, c->tab.btd_max_nxy,
                c->stream);
}

template <typename T>
void enqueue_field_cycle(gp_ctx *c) {
  enqueue_fft_fwd<T>(c);
  enqueue_update<T>(c);
  enqueue_fft_inv<T>(c);
  enqueue_btd<T>(c);
}

// nsteps whole steps; the gather-push of each step is fused with the
// deposit of the next.
template <typename T>
void enqueue_run(gp_ctx *c, int nsteps) {
  if (nsteps <= 0) return;
  enqueue_sources<T>(c, kPartDeposit);
  for (int s = 0; s + 1 < nsteps; ++s) {
    enqueue_field_cycle<T>(c);
    enqueue_sources<T>(c, kPartFused);
  }
  enqueue_field_cycle<T>(c);
  enqueue_push<T>(c, 1.0);
}

gp_status check_particles(gp_ctx *c, const gp_particles *p) {
  if (!p) return fail(GP_ERR_ARG, "particles pointer is NULL");
  for (size_t i = 0; i < c->runs.size(); ++i) {
    const gp_particles &q = p[i];
    const std::string w = "run " + std::to_string(i) + ": ";
    if (q.n < 0 || q.n > (int64_t(1) << 31) - 1)
      return fail(GP_ERR_ARG, w + "n must lie in [0, 2^31)");
    if (q.n == 0) continue;
    if (!q.x || !q.ux || !q.uy || !q.uz) return fail(GP_ERR_ARG, w + "NULL particle array");
    if (c->precision == GP_FP64 && (!q.y || !q.z))
      return fail(GP_ERR_ARG, w + "NULL position array");
    if (c->precision == GP_MIXED && (!q.off_x || !q.off_y || !q.off_z))
      return fail(GP_ERR_ARG, w + "NULL offset array");
    if (!(q.m > 0) || !(q.w >= 0) || !std::isfinite(q.q) || !std::isfinite(q.m) ||
        !std::isfinite(q.w))
      return fail(GP_ERR_ARG, w + "mass must be > 0 and weight >= 0, all finite");
  }
  return GP_OK;
}

PartPtrs to_parts(const gp_particles &q) {
  PartPtrs p;
  p.n = q.n;
  p.q = q.q;
  p.m = q.m;
  p.w = q.w;
  p.x = q.x;
  p.y = q.y;
  p.z = q.z;
  p.ox = q.off_x;
  p.oy = q.off_y;
  p.oz = q.off_z;
  p.ux = q.ux;
  p.uy = q.uy;
  p.uz = q.uz;
  p.id = q.id;
  return p;
}

bool same_parts(const PartPtrs &a, const gp_particles &b) {
  return a.n == b.n && a.x == b.x && a.y == b.y && a.z == b.z && a.ox == b.off_x &&
         a.oy == b.off_y && a.oz == b.off_z && a.ux == b.ux && a.uy == b.uy && a.uz == b.uz &&
         a.id == b.id && a.q == b.q && a.m == b.m && a.w == b.w;
}

gp_status require_bound(gp_ctx *c, const gp_particles *p) {
  if (!p) return fail(GP_ERR_ARG, "particles pointer is NULL");
  for (size_t i = 0; i < c->runs.size(); ++i) {
    if (!c->runs[i].bound)
      return fail(GP_ERR_STATE, "particles not bound (call gp_bind_particles first)");
    if (!same_parts(c->runs[i].parts, p[i]))
      return fail(GP_ERR_STATE, "run " + std::to_string(i) +
                                    ": particle arrays differ from the bound ones");
  }
  return GP_OK;
}

gp_status require_eb(gp_ctx *c, const char *who) {
  for (auto &r : c->runs)
    if (!r.eb_real_ready) return fail(GP_ERR_STATE, std::string(who) + " needs real E and B");
  return GP_OK;
}

gp_status check_ctx(gp_ctx *c) {
  if (!c) return fail(GP_ERR_ARG, "context is NULL");
  return GP_OK;
}

template <typename F>
gp_status dispatch(gp_ctx *c, F &&f) {
  if (c->precision == GP_FP64)
    f(double{});
  else
    f(float{});
  return check_launch("kernel launch");
}

void *field_slot(gp_ctx *c, Run &r, int which, size_t *bytes) {
  if (which >= GP_EX && which <= GP_RHO) {
    *bytes = real_bytes(c, r);
    return r.real[which - GP_EX];
  }
  if (which >= GP_EX_HAT && which <= GP_JZ_HAT) {
    *bytes = spec_bytes(c, r);
    return r.spec[which - GP_EX_HAT];
  }
  if (which == GP_RHO_HAT_OLD) {
    *bytes = spec_bytes(c, r);
    return r.spec[r.rho_old];
  }
  if (which == GP_RHO_HAT_NEW) {
    *bytes = spec_bytes(c, r);
    return r.spec[r.rho_old == 9 ? 10 : 9];
  }
  if (which >= GP_COEF0 && which <= GP_COEF5) {
    *bytes = spec_bytes(c, r);
    return r.coef[which - GP_COEF0];
  }
  return nullptr;
}

void free_sort(Run &r) {
  for (void *p : r.sort_allocs) (void)hipFree(p);
  r.sort_allocs.clear();
}

gp_status alloc_sort(gp_ctx *c, Run &r) {
  free_sort(r);
  const size_t nt = size_t(r.tg.n_tiles) + 1;
  const size_t ncell = size_t(r.tg.n_tiles) << r.tg.lcpt;
  const size_t n = size_t(r.parts.n);
  void *p = nullptr;
  GP_TRY(dev_alloc(r.sort_allocs, ncell * sizeof(int), &p));
  r.sb.cell_count = static_cast<int *>(p);
  GP_TRY(dev_alloc(r.sort_allocs, ncell * sizeof(int), &p));
  r.sb.cell_off = static_cast<int *>(p);
  GP_TRY(dev_alloc(r.sort_allocs, nt * sizeof(int), &p));
  r.sb.tile_total = static_cast<int *>(p);
  GP_TRY(dev_alloc(r.sort_allocs, nt * sizeof(int), &p));
  r.sb.start = static_cast<int *>(p);
  GP_TRY(dev_alloc(r.sort_allocs, n * sizeof(int), &p));
  r.sb.key = static_cast<int *>(p);
  GP_TRY(dev_alloc(r.sort_allocs, n * sizeof(int), &p));
  r.sb.rank = static_cast<int *>(p);
  GP_TRY(dev_alloc(r.sort_allocs, 4 * sizeof(int), &p));
  r.sb.state = static_cast<int *>(p);
  const int ncol = c->precision == GP_FP64 ? 6 : 7;
  for (int k = 0; k < 8; ++k) r.sb.tmp[k] = nullptr;
  for (int k = 0; k < ncol; ++k) {
    GP_TRY(dev_alloc(r.sort_allocs, n * c->real_size, &p));
    r.sb.tmp[k] = p;
  }
  if (r.parts.id) {
    GP_TRY(dev_alloc(r.sort_allocs, n * sizeof(int64_t), &p));
    r.sb.tmp[ncol] = p;
  }
  r.regbuf = nullptr;
  if (r.flush == 2) {
    GP_TRY(dev_alloc(r.sort_allocs,
                     size_t(r.tg.n_tiles) * 4 * size_t(r.tg.region) * c->real_size, &p));
    r.regbuf = p;
  }
  // a sort is forced at the first decision; the tile table starts empty
  const int init[4] = {0, 0, 0, 1};
  GP_HIP(hipMemcpyAsync(r.sb.state, init, sizeof(init), hipMemcpyHostToDevice, c->stream));
  launch_zero(r.sb.start, nt * sizeof(int), c->stream);
  launch_zero(r.sb.cell_count, ncell * sizeof(int), c->stream);
  GP_HIP(hipStreamSynchronize(c->stream));
  return GP_OK;
}

gp_status capture(gp_ctx *c, hipGraphExec_t *out, void (*body)(gp_ctx *)) {
  hipGraph_t graph = nullptr;
  GP_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  body(c);
  hipError_t le = hipGetLastError();
  hipError_t ee = hipStreamEndCapture(c->stream, &graph);
  if (le != hipSuccess || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(GP_ERR_HIP, std::string("graph capture failed: ") +
                                hipGetErrorString(le != hipSuccess ? le : ee));
  }
  hipError_t ie = hipGraphInstantiateWithFlags(out, graph, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess)
    return fail(GP_ERR_HIP, std::string("graph instantiate failed: ") + hipGetErrorString(ie));
  return GP_OK;
}

template <typename T>
void body_first(gp_ctx *c) {
  enqueue_sources<T>(c, kPartDeposit);
}
template <typename T>
void body_mid(gp_ctx *c) {
  enqueue_field_cycle<T>(c);
  enqueue_sources<T>(c, kPartFused);
}
template <typename T>
void body_last(gp_ctx *c) {
  enqueue_field_cycle<T>(c);
  enqueue_push<T>(c, 1.0);
}

template <typename T>
gp_status build_graphs(gp_ctx *c) {
  const bool timing = c->stage_timing;
  c->stage_timing = false;
  std::vector<int> saved(c->runs.size());
  for (size_t i = 0; i < c->runs.size(); ++i) saved[i] = c->runs[i].rho_old;
  gp_status st = capture(c, &c->g_first, body_first<T>);
  for (int k = 0; k < 2 && st == GP_OK; ++k) {
    set_rho_parity(c, k);
    st = capture(c, &c->g_mid[k], body_mid<T>);
    if (st == GP_OK) {
      set_rho_parity(c, k);
      st = capture(c, &c->g_last[k], body_last<T>);
    }
  }
  for (size_t i = 0; i < c->runs.size(); ++i) c->runs[i].rho_old = saved[i];
  if (c->slab) set_rho_parity(c->slab, saved[0] - 9);
  c->stage_timing = timing;
  if (st != GP_OK) drop_graphs(c);
  return st;
}

// Device tables of the slab solve: one SlabSum per run, one SlabCopy per
// slab (run-major), and the sums they share.
template <typename T>
gp_status build_slab_tables(gp_ctx *c) {
  const int n = int(c->runs.size());
  const int S = c->n_slabs;
  std::vector<SlabSum<T>> sums(n);
  std::vector<SlabCopy<T>> jobs(size_t(n) * S);
  void *d = nullptr;
  GP_TRY(dev_alloc(c->slab_allocs, size_t(4 * n) * sizeof(double), &d));
  c->slab_sums = static_cast<double *>(d);
  c->slab_max_cells = c->slab_max_win = c->slab_max_owned = 0;
  for (int i = 0; i < n; ++i) {
    const Run &r = c->runs[i];
    for (int q = 0; q < 4; ++q) sums[i].src[q] = R<T>(r, 6 + q);
    sums[i].out = c->slab_sums + 4 * i;
    sums[i].ncell = r.g.ncell;
    const int ns = r.g.nz / S;
    const int nw = ns + 2 * c->guard;
    const int nxy = r.g.nx * r.g.ny;
    c->slab_max_cells = std::max(c->slab_max_cells, r.g.ncell);
    c->slab_max_win = std::max(c->slab_max_win, int64_t(nxy) * nw);
    c->slab_max_owned = std::max(c->slab_max_owned, int64_t(nxy) * ns);
    for (int sl = 0; sl < S; ++sl) {
      const Run &w = c->slab->runs[size_t(i) * S + sl];
      SlabCopy<T> &jb = jobs[size_t(i) * S + sl];
      for (int f = 0; f < 10; ++f) {
        jb.glob[f] = R<T>(r, f);
        jb.win[f] = R<T>(w, f);
      }
      jb.sums = c->slab_sums + 4 * i;
      jb.nxy = nxy;
      jb.nz = r.g.nz;
      jb.nw = nw;
      jb.first = sl * ns - c->guard;
      jb.ns = ns;
      jb.guard = c->guard;
      jb.inv_ncell = 1.0 / double(r.g.ncell);
    }
  }
  GP_TRY(dev_alloc(c->slab_allocs, sums.size() * sizeof(SlabSum<T>), &c->slab_sum));
  GP_TRY(dev_alloc(c->slab_allocs, jobs.size() * sizeof(SlabCopy<T>), &c->slab_copy));
  GP_HIP(hipMemcpyAsync(c->slab_sum, sums.data(), sums.size() * sizeof(SlabSum<T>),
                        hipMemcpyHostToDevice, c->stream));
  GP_HIP(hipMemcpyAsync(c->slab_copy, jobs.data(), jobs.size() * sizeof(SlabCopy<T>),
                        hipMemcpyHostToDevice, c->stream));
  GP_HIP(hipStreamSynchronize(c->stream));
  return GP_OK;
}

void mark_step_done(gp_ctx *c) {
  for (auto &r : c->runs) {
    r.src_real_ready = false;
    r.src_spec_ready = false;
    r.eb_real_ready = true;
  }
}

gp_status check_run(gp_ctx *c, int run) {
  GP_TRY(check_ctx(c));
  if (run < 0 || run >= int(c->runs.size())) return fail(GP_ERR_ARG, "run out of range");
  return GP_OK;
}

}  // namespace

extern "C" {

const char *gp_last_error(void) { return g_err.c_str(); }

const char *gp_stage_name(int i) { return (i >= 0 && i < kNStages) ? kStageNames[i] : ""; }

gp_status gp_stage_timing(gp_ctx *c, int enable) {
  GP_TRY(check_ctx(c));
  c->stage_timing = enable != 0;
  return GP_OK;
}

gp_status gp_stage_times(gp_ctx *c, double *ms, int *count) {
  GP_TRY(check_ctx(c));
  if (!ms || !count) return fail(GP_ERR_ARG, "output pointer is NULL");
  for (int i = 0; i < kNStages; ++i) {
    ms[i] = 0.0;
    count[i] = 0;
  }
  GP_HIP(hipStreamSynchronize(c->stream));
  gp_status st = GP_OK;
  for (const StageRec &rec : c->stage_recs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, rec.a, rec.b) == hipSuccess) {
      ms[rec.stage] += t;
      count[rec.stage] += 1;
    } else {
      st = fail(GP_ERR_HIP, "hipEventElapsedTime failed");
    }
    (void)hipEventDestroy(rec.a);
    (void)hipEventDestroy(rec.b);
  }
  c->stage_recs.clear();
  return st;
}

gp_status gp_synchronize(gp_ctx *c) {
  GP_TRY(check_ctx(c));
  GP_HIP(hipStreamSynchronize(c->stream));
  return GP_OK;
}

gp_status gp_destroy(gp_ctx *c) {
  if (!c) return GP_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (const StageRec &rec : c->stage_recs) {
    (void)hipEventDestroy(rec.a);
    (void)hipEventDestroy(rec.b);
  }
  for (auto &r : c->runs) free_sort(r);
  if (c->slab) gp_destroy(c->slab);
  for (void *p : c->slab_allocs) (void)hipFree(p);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return GP_OK;
}

gp_status gp_init_grid(const gp_grid_desc *runs, int n_runs, void *hip_stream, gp_ctx **out) {
  g_err.clear();
  if (!out) return fail(GP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!runs || n_runs < 1) return fail(GP_ERR_ARG, "need at least one run descriptor");
  for (int i = 0; i < n_runs; ++i) GP_TRY(validate_desc(runs[i], i));
  for (int i = 1; i < n_runs; ++i)
    if (runs[i].precision != runs[0].precision || runs[i].shape_order != runs[0].shape_order)
      return fail(GP_ERR_ARG, "all runs of a context must share precision and shape order");
  gp_ctx *c = new gp_ctx();
  c->precision = runs[0].precision;
  c->order = runs[0].shape_order;
  c->real_size = c->precision == GP_FP64 ? sizeof(double) : sizeof(float);
  auto bail = [&](gp_status st) {
    std::string keep = g_err;
    gp_destroy(c);
    g_err = keep;
    return st;
  };
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    const hipError_t e = hipStreamCreate(&c->stream);
    if (e != hipSuccess)
      return bail(fail(GP_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e)));
    c->own_stream = true;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
    return bail(fail(GP_ERR_HIP, "hipEventCreate failed"));
  if (hipGetDevice(&c->device) != hipSuccess)
    return bail(fail(GP_ERR_HIP, "hipGetDevice failed"));
  {
    const hipError_t e = noalloc_prepare();
    if (e != hipSuccess)
      return bail(fail(GP_ERR_HIP, std::string("hipGetSymbolAddress of the energy scratch: ") +
                                       hipGetErrorString(e)));
  }
  c->runs.resize(n_runs);
  for (int i = 0; i < n_runs; ++i) {
    const gp_grid_desc &d = runs[i];
    Run &r = c->runs[i];
    RunGeom &g = r.g;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    g.nzh = d.nz / 2 + 1;
    g.lx = ilog2(d.nx);
    g.ly = ilog2(d.ny);
    g.lz = ilog2(d.nz);
    g.order = d.shape_order;
    g.dx = d.dx;
    g.dy = d.dy;
    g.dz = d.dz;
    g.dt = d.dt;
    g.vgal[0] = g.vgal[1] = g.vgal[2] = 0.0;
    g.ncell = int64_t(d.nx) * d.ny * d.nz;
    g.nmode = int64_t(d.nx) * d.ny * g.nzh;
    r.tg = make_tile_geom(g, c->real_size, d.tile);
    r.resort_div = d.resort_div > 0 ? d.resort_div : 64;
    // region buffer only when asked for: measured, its per-node sum costs
    // more than the atomics it saves (256x256x512: 12.44 + 1.53 ms against
    // 13.47 ms per fused pass)
    r.flush = d.flush == 2 ? 2 : 1;
    for (int a = 0; a < 3; ++a) r.stencil[a] = d.stencil[a];
    {
      gp_status st = upload_wavenumbers(c, r);
      if (st) return bail(st);
    }
    // one allocation per grid: grids at power-of-two distances in one block
    // would send the gather's six same-node loads to the same HBM channel
    for (auto &p : r.real) {
      gp_status st = dev_alloc(c->allocs, real_bytes(c, r), &p);
      if (st) return bail(st);
      launch_zero(p, real_bytes(c, r), c->stream);
    }
    for (auto &p : r.spec) {
      gp_status st = dev_alloc(c->allocs, spec_bytes(c, r), &p);
      if (st) return bail(st);
      launch_zero(p, spec_bytes(c, r), c->stream);
    }
    for (auto &p : r.coef) {
      gp_status st = dev_alloc(c->allocs, spec_bytes(c, r), &p);
      if (st) return bail(st);
    }
    for (auto &p : r.scratch) {
      gp_status st = dev_alloc(c->allocs, spec_bytes(c, r), &p);
      if (st) return bail(st);
    }
  }
  {
    const size_t twb = 1024 * 2 * c->real_size;
    gp_status st = dev_alloc(c->allocs, twb, &c->tw);
    if (st) return bail(st);
    std::vector<char> host(twb);
    if (c->precision == GP_FP64)
      fill_twiddles<double>(reinterpret_cast<Cx<double> *>(host.data()));
    else
      fill_twiddles<float>(reinterpret_cast<Cx<float> *>(host.data()));
    if (hipMemcpyAsync(c->tw, host.data(), twb, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return bail(fail(GP_ERR_HIP, "twiddle upload failed"));
    if (hipStreamSynchronize(c->stream) != hipSuccess)
      return bail(fail(GP_ERR_HIP, "stream synchronize failed"));
    void *sum = nullptr;
    st = dev_alloc(c->allocs, 2 * sizeof(double), &sum);
    if (st) return bail(st);
    c->d_sum = static_cast<double *>(sum);
    st = c->precision == GP_FP64 ? build_tables<double>(c) : build_tables<float>(c);
    if (st) return bail(st);
    st = upload_tables(c);
    if (st) return bail(st);
  }
  for (int i = 0; i < n_runs; ++i) {
    gp_status st = gp_set_v_gal(c, i, 0.0, 0.0, 0.0);
    if (st) return bail(st);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(fail(GP_ERR_HIP, "stream synchronize failed"));
  *out = c;
  return GP_OK;
}

gp_status gp_set_v_gal(gp_ctx *c, int run, double vx, double vy, double vz) {
  GP_TRY(check_run(c, run));
  if (!std::isfinite(vx) || !std::isfinite(vy) || !std::isfinite(vz) ||
      vx * vx + vy * vy + vz * vz >= 1.0)
    return fail(GP_ERR_ARG, "|v_gal| must be finite and below c");
  Run &r = c->runs[run];
  RunGeom &g = r.g;
  if (r.btd_nsnap > 0)
    return fail(GP_ERR_STATE, "turn the run's lab-frame snapshots off before changing v_gal");
  // bound on |k.v_gal| dt over the non-Nyquist modes: sum over the axes of
  // |v_a| max |k_a| (k exact or the stencil's symbol)
  const int n[3] = {g.nx, g.ny, g.nz};
  const double d[3] = {g.dx, g.dy, g.dz};
  const double v[3] = {vx, vy, vz};
  double phase = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int cnt = a < 2 ? n[a] : g.nzh;
    std::vector<double> k(cnt);
    axis_wavenumbers(n[a], d[a], r.stencil[a], cnt, k.data());
    double kmax = 0.0;
    for (int i = 0; i < cnt; ++i)
      if (i != n[a] / 2) kmax = std::max(kmax, std::fabs(k[i]));
    phase += std::fabs(v[a]) * kmax;
  }
  phase *= g.dt;
  if (phase >= 2.0 * kPi * (1.0 - 1e-6))
    return fail(GP_ERR_UNSTABLE, "some mode has |k.v_gal| dt >= 2 pi; the update is singular");
  g.vgal[0] = vx;
  g.vgal[1] = vy;
  g.vgal[2] = vz;
  CoefPtrs cp;
  for (int i = 0; i < 6; ++i) cp.c[i] = r.coef[i];
  if (c->precision == GP_FP64)
    launch_coefficients<double>(g, r.kd, cp, c->stream);
  else
    launch_coefficients<float>(g, r.kd, cp, c->stream);
  GP_TRY(check_launch("coefficients"));
  drop_graphs(c);
  if (c->tab.dev) {  // the update tables and particle jobs carry v_gal
    if (c->precision == GP_FP64) {
      fill_update_scalars<double>(c);
      if (r.bound) fill_jobs<double>(c);
    } else {
      fill_update_scalars<float>(c);
      if (r.bound) fill_jobs<float>(c);
    }
    GP_TRY(upload_tables(c));
  }
  if (c->slab)
    for (int s = 0; s < c->n_slabs; ++s)
      GP_TRY(gp_set_v_gal(c->slab, run * c->n_slabs + s, vx, vy, vz));
  return GP_OK;
}

gp_status gp_set_current_correction(gp_ctx *c, int enable) {
  GP_TRY(check_ctx(c));
  if (enable != 0 && enable != 1) return fail(GP_ERR_ARG, "enable must be 0 or 1");
  if (enable && c->slab)
    return fail(GP_ERR_STATE, "the slab solve does not take the current correction");
  c->current_correction = enable != 0;
  drop_graphs(c);
  if (c->precision == GP_FP64)
    fill_update_scalars<double>(c);
  else
    fill_update_scalars<float>(c);
  GP_TRY(upload_tables(c));
  return GP_OK;
}

gp_status gp_set_local_slabs(gp_ctx *c, int n_slabs, int guard) {
  GP_TRY(check_ctx(c));
  if (c->timing_parent) return fail(GP_ERR_ARG, "a slab context cannot be split again");
  if (n_slabs < 0 || guard < 0) return fail(GP_ERR_ARG, "n_slabs and guard must be >= 0");
  if (n_slabs > 0 && c->current_correction)
    return fail(GP_ERR_STATE, "the slab solve does not take the current correction");
  for (auto &r : c->runs)
    if (!r.eb_real_ready)
      return fail(GP_ERR_STATE, "the real E, B must be current (run gp_fft_inv first)");
  if (n_slabs > 0) {
    for (size_t i = 0; i < c->runs.size(); ++i) {
      const Run &r = c->runs[i];
      const std::string who = "run " + std::to_string(i) + ": ";
      if (r.stencil[2] == 0)
        return fail(GP_ERR_ARG, who + "local transforms need a finite-order stencil along z");
      if (r.g.nz % n_slabs != 0)
        return fail(GP_ERR_ARG, who + "nz must be a multiple of n_slabs");
      const int nw = r.g.nz / n_slabs + 2 * guard;
      if (nw < 8 || nw > r.g.nz || (nw & (nw - 1)) != 0)
        return fail(GP_ERR_ARG, who + "nz / n_slabs + 2 guard must be a power of two in "
                                      "[8, nz]");
    }
  }
  drop_graphs(c);
  GP_HIP(hipStreamSynchronize(c->stream));
  if (c->slab) {  // back to the global solve first
    gp_destroy(c->slab);
    c->slab = nullptr;
    for (void *p : c->slab_allocs) (void)hipFree(p);
    c->slab_allocs.clear();
    c->slab_copy = c->slab_sum = nullptr;
    c->slab_sums = nullptr;
    c->n_slabs = c->guard = 0;
    // the global solve's state from the real E, B and rho
    GP_TRY(dispatch(c, [&](auto t) {
      using T = decltype(t);
      const int par = rho_parity(c);
      for (const Class &k : c->tab.classes) {
        fft_forward<T>(c, kTabEBZ, kTabEBYX, 6, k.first, k.count, k.g);
        fft_forward<T>(c, kTabRhoZ0 + par, kTabRhoYX0 + par, 1, k.first, k.count, k.g);
      }
    }));
    GP_HIP(hipStreamSynchronize(c->stream));
  }
  for (auto &r : c->runs) {
    r.src_real_ready = false;
    r.src_spec_ready = false;
  }
  if (n_slabs == 0) return GP_OK;
  std::vector<gp_grid_desc> descs;
  for (const Run &r : c->runs)
    for (int s = 0; s < n_slabs; ++s) {
      gp_grid_desc d{};
      d.nx = r.g.nx;
      d.ny = r.g.ny;
      d.nz = r.g.nz / n_slabs + 2 * guard;
      d.dx = r.g.dx;
      d.dy = r.g.dy;
      d.dz = r.g.dz;
      d.dt = r.g.dt;
      d.shape_order = c->order;
      d.precision = c->precision;
      for (int a = 0; a < 3; ++a) d.stencil[a] = r.stencil[a];
      descs.push_back(d);
    }
  gp_ctx *sc = nullptr;
  GP_TRY(gp_init_grid(descs.data(), int(descs.size()), c->stream, &sc));
  sc->timing_parent = c;
  sc->src_mask = kMaskNyquist;
  sc->no_hold = true;
  c->slab = sc;
  c->n_slabs = n_slabs;
  c->guard = guard;
  auto undo = [&](gp_status st) {
    std::string keep = g_err;
    gp_destroy(sc);
    c->slab = nullptr;
    for (void *p : c->slab_allocs) (void)hipFree(p);
    c->slab_allocs.clear();
    c->n_slabs = c->guard = 0;
    g_err = keep;
    return st;
  };
  for (size_t i = 0; i < c->runs.size(); ++i)
    for (int s = 0; s < n_slabs; ++s) {
      const double *v = c->runs[i].g.vgal;
      gp_status st = gp_set_v_gal(sc, int(i) * n_slabs + s, v[0], v[1], v[2]);
      if (st) return undo(st);
    }
  {
    gp_status st = c->precision == GP_FP64 ? build_slab_tables<double>(c)
                                           : build_slab_tables<float>(c);
    if (st) return undo(st);
  }
  set_rho_parity(c, rho_parity(c));
  gp_status st = dispatch(c, [&](auto t) {
    using T = decltype(t);
    slab_init_rho<T>(c);
  });
  if (st) return undo(st);
  return GP_OK;
}

gp_status gp_btd_configure(gp_ctx *c, int run, int n_snap, double t_lab0, double dt_lab,
                           double t_boost0, void *out) {
  GP_TRY(check_run(c, run));
  Run &r = c->runs[run];
  if (n_snap < 0 || n_snap > 65535) return fail(GP_ERR_ARG, "n_snap must lie in [0, 65535]");
  if (n_snap > 0) {
    if (!out) return fail(GP_ERR_ARG, "snapshot buffer is NULL");
    if (!std::isfinite(t_lab0) || !std::isfinite(dt_lab) || !std::isfinite(t_boost0))
      return fail(GP_ERR_ARG, "t_lab0, dt_lab, t_boost0 must be finite");
    if (r.g.vgal[0] != 0.0 || r.g.vgal[1] != 0.0)
      return fail(GP_ERR_ARG, "lab-frame snapshots need v_gal = (0, 0, -beta c)");
    if (!r.eb_real_ready) return fail(GP_ERR_STATE, "gp_btd_configure needs real E and B");
  }
  drop_graphs(c);
  GP_HIP(hipStreamSynchronize(c->stream));
  r.btd_nsnap = n_snap;
  r.btd_t_lab0 = t_lab0;
  r.btd_dt_lab = dt_lab;
  r.btd_t0 = t_boost0;
  r.btd_out = n_snap > 0 ? out : nullptr;
  // new snapshots: particle records start off (gp_btd_particles)
  r.btd_pcap = 0;
  r.btd_pvals = nullptr;
  r.btd_pids = nullptr;
  r.btd_pcount = nullptr;
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    fill_btd_jobs<T>(c);
  }));
  GP_TRY(upload_tables(c));
  if (n_snap == 0) return GP_OK;
  // clear the snapshots, start at level 0 and record the current fields
  launch_zero(out, size_t(6) * n_snap * size_t(r.g.ncell) * c->real_size, c->stream);
  launch_zero(c->tab.btd_level + run, sizeof(int), c->stream);
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    launch_btd<T>(btd_tab<T>(c, c->tab.btd_pos[run]), 1, n_snap, int64_t(r.g.nx) * r.g.ny,
                  c->stream);
  }));
  return check_launch("btd");
}

gp_status gp_btd_particles(gp_ctx *c, int run, int cap, void *vals, int64_t *ids,
                           int *counts) {
  GP_TRY(check_run(c, run));
  Run &r = c->runs[run];
  if (cap < 0) return fail(GP_ERR_ARG, "cap must be >= 0");
  if (cap > 0) {
    if (r.btd_nsnap <= 0)
      return fail(GP_ERR_STATE, "particle records need the run's snapshots (gp_btd_configure)");
    if (!(r.btd_dt_lab > 0)) return fail(GP_ERR_ARG, "particle records need dt_lab > 0");
    if (!r.bound) return fail(GP_ERR_STATE, "particle records need bound particles");
    if (!vals || !counts) return fail(GP_ERR_ARG, "record buffers are NULL");
    if (ids && !r.parts.id) return fail(GP_ERR_ARG, "the run's particles carry no ids");
    if (int64_t(cap) * 6 * r.btd_nsnap > (int64_t(1) << 40))
      return fail(GP_ERR_ARG, "cap too large");
  }
  drop_graphs(c);
  GP_HIP(hipStreamSynchronize(c->stream));
  r.btd_pcap = cap;
  r.btd_pvals = cap > 0 ? vals : nullptr;
  r.btd_pids = cap > 0 ? ids : nullptr;
  r.btd_pcount = cap > 0 ? counts : nullptr;
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    fill_btd_jobs<T>(c);
  }));
  GP_TRY(upload_tables(c));
  if (cap > 0) launch_zero(counts, size_t(r.btd_nsnap) * sizeof(int), c->stream);
  return check_launch("btd particles");
}

gp_status gp_btd_record(gp_ctx *c) {
  GP_TRY(check_ctx(c));
  GP_TRY(require_eb(c, "gp_btd_record"));
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_btd<T>(c);
  }));
  return check_launch("btd");
}

gp_status gp_bind_particles(gp_ctx *c, const gp_particles *p) {
  GP_TRY(check_ctx(c));
  GP_TRY(check_particles(c, p));
  drop_graphs(c);
  GP_HIP(hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < c->runs.size(); ++i) {
    Run &r = c->runs[i];
    r.bound = false;
    r.parts = to_parts(p[i]);
    GP_TRY(alloc_sort(c, r));
    r.bound = true;
  }
  if (c->precision == GP_FP64) {
    fill_jobs<double>(c);
    fill_btd_jobs<double>(c);  // particle records follow the new arrays
  } else {
    fill_jobs<float>(c);
    fill_btd_jobs<float>(c);
  }
  GP_TRY(upload_tables(c));
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    for (auto &r : c->runs) launch_zero(r.real[9], real_bytes(c, r), c->stream);
    launch_sort<T>(job_tab<T>(c), c->tab.batch, c->stream);
    launch_particles<T>(kPartRho, job_tab<T>(c), c->tab.batch, 0.0, c->stream);
    const int par = rho_parity(c);
    for (const Class &k : c->tab.classes)
      fft_forward<T>(c, kTabRhoZ0 + par, kTabRhoYX0 + par, 1, k.first, k.count, k.g);
    if (c->slab) slab_init_rho<T>(c);
  }));
  for (auto &r : c->runs) {
    r.src_real_ready = false;
    r.src_spec_ready = false;
  }
  return GP_OK;
}

gp_status gp_deposit(gp_ctx *c, const gp_particles *p) {
  GP_TRY(check_ctx(c));
  GP_TRY(require_bound(c, p));
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_sources<T>(c, kPartDeposit);
  }));
  for (auto &r : c->runs) r.src_real_ready = true;
  return GP_OK;
}

gp_status gp_fft_fwd(gp_ctx *c) {
  GP_TRY(check_ctx(c));
  for (auto &r : c->runs) {
    if (!r.src_real_ready) return fail(GP_ERR_STATE, "gp_fft_fwd needs a deposit first");
    if (c->slab && !r.eb_real_ready)
      return fail(GP_ERR_STATE, "the slab solve transforms the real E, B: run gp_fft_inv first");
  }
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_fft_fwd<T>(c);
  }));
  for (auto &r : c->runs) {
    r.src_real_ready = false;
    r.src_spec_ready = true;
  }
  return GP_OK;
}

gp_status gp_galilean_psatd_update(gp_ctx *c) {
  GP_TRY(check_ctx(c));
  for (auto &r : c->runs)
    if (!r.src_spec_ready)
      return fail(GP_ERR_STATE, "gp_galilean_psatd_update needs gp_fft_fwd first");
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_update<T>(c);
  }));
  for (auto &r : c->runs) {
    r.src_spec_ready = false;
    r.eb_real_ready = false;
  }
  return GP_OK;
}

gp_status gp_fft_inv(gp_ctx *c) {
  GP_TRY(check_ctx(c));
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_fft_inv<T>(c);
  }));
  for (auto &r : c->runs) r.eb_real_ready = true;
  return GP_OK;
}

gp_status gp_gather_push(gp_ctx *c, const gp_particles *p) {
  GP_TRY(check_ctx(c));
  GP_TRY(require_bound(c, p));
  GP_TRY(require_eb(c, "gp_gather_push"));
  return dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_push<T>(c, 1.0);
  });
}

gp_status gp_gather_push_deposit(gp_ctx *c, const gp_particles *p) {
  GP_TRY(check_ctx(c));
  GP_TRY(require_bound(c, p));
  GP_TRY(require_eb(c, "gp_gather_push_deposit"));
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_sources<T>(c, kPartFused);
  }));
  for (auto &r : c->runs) r.src_real_ready = true;
  return GP_OK;
}

gp_status gp_half_push(gp_ctx *c, const gp_particles *p) {
  GP_TRY(check_ctx(c));
  GP_TRY(require_bound(c, p));
  GP_TRY(require_eb(c, "gp_half_push"));
  return dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_push<T>(c, 0.5);
  });
}

gp_status gp_step(gp_ctx *c, const gp_particles *p) { return gp_run(c, p, 1); }

gp_status gp_run(gp_ctx *c, const gp_particles *p, int nsteps) {
  GP_TRY(check_ctx(c));
  GP_TRY(require_bound(c, p));
  if (nsteps < 0) return fail(GP_ERR_ARG, "nsteps < 0");
  GP_TRY(require_eb(c, "gp_run"));
  if (nsteps == 0) return GP_OK;
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    enqueue_run<T>(c, nsteps);
  }));
  mark_step_done(c);
  return GP_OK;
}

gp_status gp_step_graph(gp_ctx *c, const gp_particles *p, int nsteps) {
  GP_TRY(check_ctx(c));
  GP_TRY(require_bound(c, p));
  if (nsteps < 0) return fail(GP_ERR_ARG, "nsteps < 0");
  GP_TRY(require_eb(c, "gp_step_graph"));
  if (nsteps == 0) return GP_OK;
  if (!c->g_first) {
    if (c->precision == GP_FP64)
      GP_TRY(build_graphs<double>(c));
    else
      GP_TRY(build_graphs<float>(c));
  }
  // all runs rotate their rho buffers together
  int par = c->runs[0].rho_old - 9;
  GP_HIP(hipEventRecord(c->ev0, c->stream));
  GP_HIP(hipGraphLaunch(c->g_first, c->stream));
  for (int s = 0; s + 1 < nsteps; ++s) {
    GP_HIP(hipGraphLaunch(c->g_mid[par], c->stream));
    par ^= 1;
  }
  GP_HIP(hipGraphLaunch(c->g_last[par], c->stream));
  par ^= 1;
  GP_HIP(hipEventRecord(c->ev1, c->stream));
  c->timed = true;
  set_rho_parity(c, par);
  mark_step_done(c);
  return GP_OK;
}

gp_status gp_last_graph_ms(gp_ctx *c, double *ms) {
  GP_TRY(check_ctx(c));
  if (!ms) return fail(GP_ERR_ARG, "ms is NULL");
  if (!c->timed) return fail(GP_ERR_STATE, "no graph replay recorded");
  GP_HIP(hipEventSynchronize(c->ev1));
  float t = 0.f;
  GP_HIP(hipEventElapsedTime(&t, c->ev0, c->ev1));
  *ms = t;
  return GP_OK;
}

gp_status gp_sort_count(gp_ctx *c, int run, int *sorts) {
  GP_TRY(check_run(c, run));
  if (!sorts) return fail(GP_ERR_ARG, "sorts is NULL");
  Run &r = c->runs[run];
  if (!r.bound) return fail(GP_ERR_STATE, "particles not bound");
  int st[4];
  GP_HIP(hipMemcpyAsync(st, r.sb.state, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  GP_HIP(hipStreamSynchronize(c->stream));
  *sorts = st[2];
  return GP_OK;
}

gp_status gp_set_fields(gp_ctx *c, int run, const void *const E[3], const void *const B[3],
                        int project_transverse) {
  GP_TRY(check_run(c, run));
  Run &r = c->runs[run];
  const size_t rb = real_bytes(c, r);
  for (int a = 0; a < 6; ++a) {
    const void *src = a < 3 ? (E ? E[a] : nullptr) : (B ? B[a - 3] : nullptr);
    if (src)
      GP_HIP(hipMemcpyAsync(r.real[a], src, rb, hipMemcpyDefault, c->stream));
    else
      launch_zero(r.real[a], rb, c->stream);
  }
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    const int pos = c->tab.pos[run];
    fft_forward<T>(c, kTabEBZ, kTabEBYX, 6, pos, 1, r.g);
    const T *kt = static_cast<const T *>(r.kt);
    launch_project<T>(r.g, kt, S<T>(r, 0), S<T>(r, 1), S<T>(r, 2), project_transverse != 0,
                      c->stream);
    launch_project<T>(r.g, kt, S<T>(r, 3), S<T>(r, 4), S<T>(r, 5), project_transverse != 0,
                      c->stream);
    fft_inverse<T>(c, pos, 1, r.g);
  }));
  GP_HIP(hipStreamSynchronize(c->stream));
  r.eb_real_ready = true;
  return GP_OK;
}

gp_status gp_read_field(gp_ctx *c, int run, int which, void *dst) {
  GP_TRY(check_run(c, run));
  if (!dst) return fail(GP_ERR_ARG, "dst is NULL");
  size_t bytes = 0;
  void *src = field_slot(c, c->runs[run], which, &bytes);
  if (!src) return fail(GP_ERR_ARG, "unknown field selector");
  GP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, c->stream));
  GP_HIP(hipStreamSynchronize(c->stream));
  return GP_OK;
}

gp_status gp_write_field(gp_ctx *c, int run, int which, const void *src) {
  GP_TRY(check_run(c, run));
  if (!src) return fail(GP_ERR_ARG, "src is NULL");
  if (which >= GP_COEF0 && which <= GP_COEF5)
    return fail(GP_ERR_ARG, "coefficient tables are read-only");
  Run &r = c->runs[run];
  size_t bytes = 0;
  void *dst = field_slot(c, r, which, &bytes);
  if (!dst) return fail(GP_ERR_ARG, "unknown field selector");
  GP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, c->stream));
  GP_HIP(hipStreamSynchronize(c->stream));
  if (which >= GP_JX && which <= GP_RHO) r.src_real_ready = true;
  if ((which >= GP_JX_HAT && which <= GP_JZ_HAT) || which == GP_RHO_HAT_NEW)
    r.src_spec_ready = true;
  if (which >= GP_EX && which <= GP_BZ) r.eb_real_ready = true;
  return GP_OK;
}

gp_status gp_field_ptr(gp_ctx *c, int run, int which, void **dev_ptr) {
  GP_TRY(check_run(c, run));
  if (!dev_ptr) return fail(GP_ERR_ARG, "dev_ptr is NULL");
  size_t bytes = 0;
  void *p = field_slot(c, c->runs[run], which, &bytes);
  if (!p) return fail(GP_ERR_ARG, "unknown field selector");
  *dev_ptr = p;
  return GP_OK;
}

gp_status gp_field_energy(gp_ctx *c, int run, double *we, double *wb) {
  GP_TRY(check_run(c, run));
  if (!we || !wb) return fail(GP_ERR_ARG, "output pointer is NULL");
  Run &r = c->runs[run];
  launch_zero(c->d_sum, 2 * sizeof(double), c->stream);
  GP_TRY(dispatch(c, [&](auto t) {
    using T = decltype(t);
    launch_sum_squares<T>(R<T>(r, 0), R<T>(r, 1), R<T>(r, 2), r.g.ncell, c->d_sum, c->stream);
    launch_sum_squares<T>(R<T>(r, 3), R<T>(r, 4), R<T>(r, 5), r.g.ncell, c->d_sum + 1,
                          c->stream);
  }));
  double h[2];
  GP_HIP(hipMemcpyAsync(h, c->d_sum, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  GP_HIP(hipStreamSynchronize(c->stream));
  const double dv = r.g.dx * r.g.dy * r.g.dz;
  *we = 0.5 * dv * h[0];
  *wb = 0.5 * dv * h[1];
  return GP_OK;
}

gp_status gp_field_energy_noalloc(gp_ctx *c, int run, double *out) {
  GP_TRY(check_run(c, run));
  if (!out) return fail(GP_ERR_ARG, "out is NULL");
  const Run &r = c->runs[run];
  if (r.g.ncell > noalloc_max_cells())
    return fail(GP_ERR_ARG, "gp_field_energy_noalloc takes at most " +
                                std::to_string(noalloc_max_cells()) + " cells; the run has " +
                                std::to_string(r.g.ncell));
  double *slots = noalloc_scratch(c->device);
  if (!slots) return fail(GP_ERR_STATE, "no energy scratch on the context's device");
  const double dv = r.g.dx * r.g.dy * r.g.dz;
  return dispatch(c, [&](auto t) {
    using T = decltype(t);
    const T *E[3] = {R<T>(r, 0), R<T>(r, 1), R<T>(r, 2)};
    const T *B[3] = {R<T>(r, 3), R<T>(r, 4), R<T>(r, 5)};
    launch_energy_noalloc<T>(E, B, r.g.ncell, dv, slots, out, c->stream);
  });
}

}  // extern "C"
