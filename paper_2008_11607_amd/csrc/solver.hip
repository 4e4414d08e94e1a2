// Host driver of the REXII shifted-solve path and the C ABI entry points.
//
// One call of rexii_apply:
//   1. rho and the pole set (coeffs.cpp; eq. matrixAccuracyBound);
//   2. per-pole Helmholtz shifts and accumulation weights (kernels.h);
//   3. solves scheduled in batches of B concurrent slots, poles sorted by
//      their expected Krylov cost so that a batch finishes together;
//   4. per batch: a chunk of kernels (FP64 residual/refinement step, then C
//      inner COCG iterations) replayed from a HIP graph until every slot has
//      converged, then FP64 weighted accumulation (Sec. 2.2, reduced sum);
//   5. the output is rebuilt from the three accumulated fields.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "kernels.h"
#include "rexii_internal.h"

namespace rexii {

// ---------------------------------------------------------------------------
// error state
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

rexii_status set_error(rexii_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
rexii_status clear_error() {
  g_err.clear();
  return REXII_OK;
}

struct HipError {
  rexii_status st;
  std::string msg;
};

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw HipError{e_ == hipErrorOutOfMemory ? REXII_ERR_OOM : REXII_ERR_HIP,            \
                     std::string(#call) + ": " + hipGetErrorString(e_)};                   \
  } while (0)

using cd = std::complex<double>;

static inline double2 to_d2(cd c) { return make_double2(c.real(), c.imag()); }

// ---------------------------------------------------------------------------
// device memory: caller workspace or own allocation
// ---------------------------------------------------------------------------
class Arena {
 public:
  Arena(void* ws, size_t bytes) : base_(static_cast<char*>(ws)), cap_(bytes), own_(false) {}
  ~Arena() {
    if (own_ && base_) (void)hipFree(base_);
  }
  void reserve_own(size_t bytes) {
    own_ = true;
    cap_ = bytes;
    HIPCHK(hipMalloc(reinterpret_cast<void**>(&base_), bytes));
  }
  template <typename T>
  T* take(size_t count) {
    const size_t bytes = ((count * sizeof(T)) + 255) & ~size_t(255);
    if (off_ + bytes > cap_) throw HipError{REXII_ERR_WORKSPACE, "workspace too small"};
    T* p = reinterpret_cast<T*>(base_ + off_);
    off_ += bytes;
    return p;
  }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, off_ = 0;
  bool own_;
};

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// problem description
// ---------------------------------------------------------------------------
struct SolveDesc {
  cd zeta, a1, a2;     // Helmholtz shift and RHS coefficients
  cd c0, c1, c2;       // accumulation weights (A_j += Re(c_j y))
  cd inv_sigma, m1, m2;
  double cost;         // expected relative Krylov cost (for scheduling)
  int pole;            // first pole index this solve serves
};

struct Plan {
  int nx, ny;
  double g, H, fc, t;
  double h, tol, rho, kappa, pole_tol;
  int M, N, P, m0;
  int precision;
  int max_iter;
  double inner_eta;
  bool paired;
  bool has_vel;
  int B;               // slots per batch
  int chunk;           // inner iterations per graph replay
  bool profile = false;
  std::vector<cd> z, w;
  std::vector<SolveDesc> solves;
  double S1 = 0, S2 = 0;
};

static Geo make_geo(int nx, int ny) {
  Geo g;
  g.nx = nx;
  g.ny = ny;
  g.tiles_x = (nx + kTX - 1) / kTX;
  g.tiles_y = (ny + kTY - 1) / kTY;
  g.nblk = g.tiles_x * g.tiles_y;
  g.cx = 0.25 * double(nx) * nx;
  g.cy = 0.25 * double(ny) * ny;
  return g;
}

static size_t inner_elem_bytes(int precision) { return precision == REXII_PREC_MIXED ? 8 : 16; }

// Chebyshev estimate of the COCG iteration count for (L - zeta) with the
// spectrum of L in [-lmax, 0]: the segment {-l - zeta} seen from 0.
static double cheb_cost(cd zeta, double lmax, double tol) {
  const cd w0 = -(1.0 + 2.0 * zeta / lmax);
  const cd s = std::sqrt(w0 * w0 - 1.0);
  const double R = std::max(std::abs(w0 + s), std::abs(w0 - s));
  if (!(R > 1.0 + 1e-15)) return 1e9;
  return std::log(2.0 / tol) / std::log(R);
}

static rexii_status validate_op(const rexii_swe_op* op) {
  if (!op) return set_error(REXII_ERR_INVALID_ARG, "op is NULL");
  if (op->nx < 4 || op->ny < 4) return set_error(REXII_ERR_INVALID_ARG, "nx and ny must be >= 4");
  if (size_t(op->nx) * size_t(op->ny) > (size_t(1) << 28))
    return set_error(REXII_ERR_INVALID_ARG, "grid too large");
  if (!(op->g > 0.0) || !std::isfinite(op->g)) return set_error(REXII_ERR_INVALID_ARG, "g must be > 0");
  if (!std::isfinite(op->f_cor)) return set_error(REXII_ERR_INVALID_ARG, "f_cor must be finite");
  if (!op->H_field && (!(op->H0 > 0.0) || !std::isfinite(op->H0)))
    return set_error(REXII_ERR_INVALID_ARG, "H0 must be > 0");
  return REXII_OK;
}

static rexii_opts resolve_opts(const rexii_opts* o) {
  rexii_opts r;
  rexii_default_opts(&r);
  if (o) r = *o;
  if (r.h <= 0.0) r.h = 0.5;
  if (r.tol <= 0.0) r.tol = (r.precision == REXII_PREC_MIXED) ? 1e-6 : 1e-10;
  if (r.max_iter <= 0) r.max_iter = 50000;
  if (r.inner_tol <= 0.0) r.inner_tol = 1e-4;
  return r;
}

// Pole set, shifts, weights and scheduling (host, FP64).
static rexii_status build_plan(const rexii_swe_op* op, double t, const rexii_opts& o, bool has_vel,
                               bool div_free, Plan& pl) {
  pl.nx = op->nx;
  pl.ny = op->ny;
  pl.g = op->g;
  pl.H = op->H0;
  pl.fc = op->f_cor;
  pl.t = t;
  pl.h = o.h;
  pl.tol = o.tol;
  pl.precision = o.precision;
  pl.max_iter = o.max_iter;
  pl.inner_eta = (o.precision == REXII_PREC_MIXED) ? o.inner_tol : 0.0;
  pl.has_vel = has_vel;
  pl.profile = (o.profile != 0);
  pl.paired = (o.pair_conjugate != 0) && div_free;
  if (!(o.h > 0.0 && o.h < M_PI)) return set_error(REXII_ERR_INVALID_ARG, "h must be in (0, pi)");
  if (!(o.tol > 0.0 && o.tol < 1.0)) return set_error(REXII_ERR_INVALID_ARG, "tol must be in (0, 1)");
  if (o.precision != REXII_PREC_FP64 && o.precision != REXII_PREC_MIXED)
    return set_error(REXII_ERR_INVALID_ARG, "unknown precision");
  pl.rho = (o.rho > 0.0) ? o.rho : rho_const(op->nx, op->ny, op->g, op->H0, op->f_cor);
  pl.m0 = (o.m0 >= 0) ? o.m0 : m0_from_tol(o.tol);
  const double Md = std::ceil(t * pl.rho / pl.h) + pl.m0;
  if (Md > 2.0e6) return set_error(REXII_ERR_INVALID_ARG, "t*rho/h too large for this library");
  pl.M = m_rule(t, pl.rho, pl.h, pl.m0);
  pl.N = pl.M + terms_L();
  std::vector<cplx> z, w;
  poles_weights(pl.M, pl.h, z, w);
  pl.P = int(z.size());
  pl.z.resize(pl.P);
  pl.w.resize(pl.P);
  for (int k = 0; k < pl.P; ++k) {
    pl.z[k] = cd(z[k].re, z[k].im);
    pl.w[k] = cd(w[k].re, w[k].im);
  }
  pl.kappa = kappa_sum(w, pl.h);
  pl.pole_tol = pl.tol / pl.kappa;

  const double g = op->g, H = op->H0, fc = op->f_cor;
  const double lmax = max_s2(op->nx) + max_s2(op->ny);  // max(s_x^2 + s_y^2)
  pl.S1 = pl.S2 = 0.0;
  std::vector<cd> m1(pl.P), m2(pl.P), sig(pl.P), zet(pl.P);
  for (int k = 0; k < pl.P; ++k) {
    const cd zk = pl.z[k];
    const cd den = zk * zk + t * t * fc * fc;
    m1[k] = -zk / den;
    m2[k] = -t * fc / den;
    sig[k] = t * t * g * H * zk / den;
    zet[k] = den / (t * t * g * H);
    pl.S1 += (pl.w[k] * m1[k]).real();
    pl.S2 += (pl.w[k] * m2[k]).real();
  }
  pl.solves.clear();
  if (pl.paired) {
    for (int n = 0; 2 * n < pl.P; ++n) {
      const int k = 2 * n;
      SolveDesc s;
      s.zeta = zet[k];
      s.a1 = t * H * m1[k];
      s.a2 = t * H * m2[k];
      const cd w1 = pl.w[k], w2c = std::conj(pl.w[k + 1]);
      s.inv_sigma = 1.0 / sig[k];
      s.m1 = m1[k];
      s.m2 = m2[k];
      s.c0 = (w1 - w2c) * s.inv_sigma;
      s.c1 = (w1 + w2c) * m1[k] * s.inv_sigma;
      s.c2 = (w1 - w2c) * m2[k] * s.inv_sigma;
      s.cost = cheb_cost(s.zeta, lmax, pl.pole_tol);
      s.pole = k;
      pl.solves.push_back(s);
    }
  } else {
    for (int k = 0; k < pl.P; ++k) {
      SolveDesc s;
      s.zeta = zet[k];
      s.a1 = t * H * m1[k];
      s.a2 = t * H * m2[k];
      s.inv_sigma = 1.0 / sig[k];
      s.m1 = m1[k];
      s.m2 = m2[k];
      s.c0 = pl.w[k] * s.inv_sigma;
      s.c1 = pl.w[k] * m1[k] * s.inv_sigma;
      s.c2 = pl.w[k] * m2[k] * s.inv_sigma;
      s.cost = cheb_cost(s.zeta, lmax, pl.pole_tol);
      s.pole = k;
      pl.solves.push_back(s);
    }
  }
  // most expensive first: batches of similar cost
  std::stable_sort(pl.solves.begin(), pl.solves.end(),
                   [](const SolveDesc& a, const SolveDesc& b) { return a.cost > b.cost; });
  const Geo geo = make_geo(op->nx, op->ny);
  int B = o.pole_batch;
  if (B <= 0) {
    B = (8192 + geo.nblk - 1) / geo.nblk;
    B = std::max(8, std::min(B, 512));
  }
  // keep a batch within 16 GiB
  const size_t per_slot = size_t(op->nx) * op->ny * (16 + 4 * inner_elem_bytes(o.precision));
  const size_t cap = size_t(16) << 30;
  B = int(std::max<size_t>(1, std::min<size_t>(size_t(B), cap / per_slot)));
  B = std::min<int>(B, int(pl.solves.size()));
  pl.B = std::max(1, B);
  pl.chunk = 16;
  return REXII_OK;
}

static size_t plan_bytes(const Plan& pl) {
  const size_t n = size_t(pl.nx) * pl.ny;
  const Geo geo = make_geo(pl.nx, pl.ny);
  const size_t eb = inner_elem_bytes(pl.precision);
  size_t b = 0;
  b += al256(2 * n * sizeof(double));      // D0, Z0
  b += al256(3 * n * sizeof(double));      // A
  b += al256(64 * sizeof(int));            // flags, counters
  b += al256(pl.B * sizeof(Slot));
  b += al256(pl.B * n * 16);               // x64
  b += 4 * al256(pl.B * n * eb);           // d, r, p0, p1
  b += 2 * al256(size_t(pl.B) * geo.nblk * 16) + al256(size_t(pl.B) * geo.nblk * 8);
  b += 6 * al256(pl.B * 16);               // c0..c2, inv_sigma, m1, m2
  return b;
}

// ---------------------------------------------------------------------------
// the batched solve engine
// ---------------------------------------------------------------------------
struct Engine {
  Plan& pl;
  hipStream_t st;
  Batch bt{};
  Rhs rhs{};
  double* A = nullptr;
  double2 *c0 = nullptr, *c1 = nullptr, *c2 = nullptr, *isg = nullptr, *dm1 = nullptr, *dm2 = nullptr;
  int* hcount = nullptr;   // pinned host mirror of the counters
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  // report
  int max_iters = 0, max_rounds = 0, not_conv = 0, breakdowns = 0;
  int64_t total_iters = 0;
  double max_rel_res = 0.0;
  int stagnated = 0;
  // profiling (opts.profile)
  std::vector<hipEvent_t> evs;
  int64_t mv_launches = 0, up_launches = 0;
  double mv_ms = 0.0, up_ms = 0.0;

  Engine(Plan& p, hipStream_t s) : pl(p), st(s) {}
  ~Engine() {
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (hcount) (void)hipHostFree(hcount);
  }

  void setup(Arena& ar, const double* f, double* DZ, int* small) {
    const size_t n = size_t(pl.nx) * pl.ny;
    const Geo geo = make_geo(pl.nx, pl.ny);
    const size_t eb = inner_elem_bytes(pl.precision);
    A = ar.take<double>(3 * n);
    bt.B = pl.B;
    bt.geo = geo;
    bt.slots = ar.take<Slot>(pl.B);
    bt.x64 = ar.take<double2>(size_t(pl.B) * n);
    bt.d = ar.take<char>(size_t(pl.B) * n * eb);
    bt.r = ar.take<char>(size_t(pl.B) * n * eb);
    bt.p0 = ar.take<char>(size_t(pl.B) * n * eb);
    bt.p1 = ar.take<char>(size_t(pl.B) * n * eb);
    bt.part_a = ar.take<double2>(size_t(pl.B) * geo.nblk);
    bt.part_b = ar.take<double2>(size_t(pl.B) * geo.nblk);
    bt.part_c = ar.take<double>(size_t(pl.B) * geo.nblk);
    bt.counter = small + 16;
    c0 = ar.take<double2>(pl.B);
    c1 = ar.take<double2>(pl.B);
    c2 = ar.take<double2>(pl.B);
    isg = ar.take<double2>(pl.B);
    dm1 = ar.take<double2>(pl.B);
    dm2 = ar.take<double2>(pl.B);
    rhs.eta0 = f;
    rhs.D0 = pl.has_vel ? DZ : nullptr;
    rhs.Z0 = pl.has_vel ? DZ + n : nullptr;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hcount), 64 * sizeof(int), hipHostMallocDefault));
    launch_fill_zero(A, 3 * n, st);
  }

  template <typename T>
  void enqueue_chunk() {
    launch_outer_update<T>(bt, st);
    launch_outer_residual<T>(bt, rhs, st);
    launch_scalars_outer(bt, st);
    for (int i = 0; i < pl.chunk; ++i) {
      launch_inner_mv<T>(bt, st);
      launch_scalars_mv(bt, st);
      launch_inner_up<T>(bt, st);
      launch_scalars_up(bt, st);
    }
    launch_count(bt, st);
    HIPCHK(hipMemcpyAsync(hcount, bt.counter, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  }

  // The same chunk, launched directly, with an event pair around every inner
  // kernel; elapsed times are collected after the chunk's host sync.
  template <typename T>
  void enqueue_chunk_profiled() {
    if (evs.empty()) {
      evs.resize(4 * pl.chunk);
      for (hipEvent_t& e : evs) HIPCHK(hipEventCreate(&e));
    }
    launch_outer_update<T>(bt, st);
    launch_outer_residual<T>(bt, rhs, st);
    launch_scalars_outer(bt, st);
    for (int i = 0; i < pl.chunk; ++i) {
      HIPCHK(hipEventRecord(evs[4 * i], st));
      launch_inner_mv<T>(bt, st);
      HIPCHK(hipEventRecord(evs[4 * i + 1], st));
      launch_scalars_mv(bt, st);
      HIPCHK(hipEventRecord(evs[4 * i + 2], st));
      launch_inner_up<T>(bt, st);
      HIPCHK(hipEventRecord(evs[4 * i + 3], st));
      launch_scalars_up(bt, st);
    }
    launch_count(bt, st);
    HIPCHK(hipMemcpyAsync(hcount, bt.counter, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  }
  void collect_profile() {
    for (int i = 0; i < pl.chunk; ++i) {
      float a = 0.f, b = 0.f;
      HIPCHK(hipEventElapsedTime(&a, evs[4 * i], evs[4 * i + 1]));
      HIPCHK(hipEventElapsedTime(&b, evs[4 * i + 2], evs[4 * i + 3]));
      mv_ms += a;
      up_ms += b;
    }
    mv_launches += pl.chunk;
    up_launches += pl.chunk;
  }

  template <typename T>
  void build_graph() {
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_chunk<T>();
    } catch (...) {
      hipGraph_t g2;
      (void)hipStreamEndCapture(st, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    HIPCHK(hipStreamEndCapture(st, &graph));
    HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
  }

  // Run all solves in batches; accumulate into A.  If xout != nullptr the
  // per-solve solutions are expanded into xout instead (shifted_solve).
  template <typename T>
  void run(const double* f, double2* xout) {
    const size_t n = size_t(pl.nx) * pl.ny;
    const int S = int(pl.solves.size());
    if (!pl.profile) build_graph<T>();
    std::vector<Slot> hs(pl.B);
    std::vector<double2> hc0(pl.B), hc1(pl.B), hc2(pl.B), his(pl.B), hm1(pl.B), hm2(pl.B);
    for (int s0 = 0; s0 < S; s0 += pl.B) {
      const int ns = std::min(pl.B, S - s0);
      for (int j = 0; j < pl.B; ++j) {
        Slot sl;
        std::memset(&sl, 0, sizeof(sl));
        if (j < ns) {
          const SolveDesc& d = pl.solves[s0 + j];
          sl.zeta = to_d2(d.zeta);
          sl.a1 = to_d2(d.a1);
          sl.a2 = to_d2(d.a2);
          sl.tol2 = pl.pole_tol * pl.pole_tol;
          sl.inner_eta2 = pl.inner_eta * pl.inner_eta;
          sl.status = kOuterPending;
          sl.max_iter = pl.max_iter;
          sl.pole = d.pole;
          hc0[j] = to_d2(d.c0);
          hc1[j] = to_d2(d.c1);
          hc2[j] = to_d2(d.c2);
          his[j] = to_d2(d.inv_sigma);
          hm1[j] = to_d2(d.m1);
          hm2[j] = to_d2(d.m2);
        } else {
          sl.status = kIdle;
          hc0[j] = hc1[j] = hc2[j] = his[j] = hm1[j] = hm2[j] = make_double2(0, 0);
        }
        hs[j] = sl;
      }
      HIPCHK(hipMemcpyAsync(bt.slots, hs.data(), pl.B * sizeof(Slot), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(c0, hc0.data(), pl.B * 16, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(c1, hc1.data(), pl.B * 16, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(c2, hc2.data(), pl.B * 16, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(isg, his.data(), pl.B * 16, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dm1, hm1.data(), pl.B * 16, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dm2, hm2.data(), pl.B * 16, hipMemcpyHostToDevice, st));
      launch_fill_zero(reinterpret_cast<double*>(bt.x64), size_t(pl.B) * n * 2, st);
      // replay the chunk until no slot is working
      const int max_replays = pl.max_iter / pl.chunk + 64;
      for (int rep = 0; rep < max_replays; ++rep) {
        if (pl.profile) {
          enqueue_chunk_profiled<T>();
          HIPCHK(hipStreamSynchronize(st));
          collect_profile();
        } else {
          HIPCHK(hipGraphLaunch(gexec, st));
          HIPCHK(hipStreamSynchronize(st));
        }
        if (hcount[0] == 0) break;
      }
      if (xout) {
        launch_expand(bt, f, ns, isg, dm1, dm2, pl.t * pl.g, pl.has_vel ? 1 : 0,
                      xout + size_t(s0) * 3 * n, st);
      } else {
        launch_accumulate(bt, c0, c1, c2, ns, A, st);
      }
      HIPCHK(hipMemcpyAsync(hs.data(), bt.slots, pl.B * sizeof(Slot), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int j = 0; j < ns; ++j) {
        const Slot& sl = hs[j];
        max_iters = std::max(max_iters, sl.it_total);
        max_rounds = std::max(max_rounds, sl.rounds);
        total_iters += sl.it_total;
        if (sl.status == kFailMaxIter) not_conv++;
        if (sl.status == kFailBreakdown) breakdowns++;
        if (sl.status != kDone && sl.status != kFailMaxIter && sl.status != kFailBreakdown) not_conv++;
        stagnated += sl.stagnated;
        const double rel = sl.bn2 > 0 ? std::sqrt(sl.rn2 / sl.bn2) : 0.0;
        max_rel_res = std::max(max_rel_res, rel);
      }
    }
  }
};

static void fill_report(rexii_report* rep, const Plan& pl, const Engine* e, double secs) {
  if (!rep) return;
  std::memset(rep, 0, sizeof(*rep));
  rep->P = pl.P;
  rep->M = pl.M;
  rep->N = pl.N;
  rep->m0 = pl.m0;
  rep->solves = int(pl.solves.size());
  rep->h = pl.h;
  rep->t = pl.t;
  rep->rho = pl.rho;
  rep->kappa_sum = pl.kappa;
  rep->pole_tol = pl.pole_tol;
  rep->seconds = secs;
  if (e) {
    rep->max_iters = e->max_iters;
    rep->max_refine = e->max_rounds;
    rep->not_converged = e->not_conv;
    rep->total_iters = e->total_iters;
    rep->max_rel_residual = e->max_rel_res;
    const double eb = double(inner_elem_bytes(pl.precision));
    // inner iteration: mv reads r, p and writes p; up reads p, d, r and writes d, r
    rep->alg_bytes = double(e->total_iters) * double(pl.nx) * pl.ny * 8.0 * eb;
    rep->mv_launches = e->mv_launches;
    rep->up_launches = e->up_launches;
    rep->mv_ms = e->mv_ms;
    rep->up_ms = e->up_ms;
    rep->mv_bytes = double(e->total_iters) * double(pl.nx) * pl.ny * 3.0 * eb;
    rep->up_bytes = double(e->total_iters) * double(pl.nx) * pl.ny * 5.0 * eb;
  }
}

// Shared front end of apply / shifted_solve.
static rexii_status run_problem_on(const rexii_swe_op* op, const double* f, double* u, double t,
                                   const rexii_opts* opts_in, void* ws, size_t ws_bytes,
                                   hipStream_t stream, rexii_report* rep, const std::vector<cd>* shifts,
                                   double2* xout);

// The work runs on a private stream (graph capture needs a capturable
// stream; the caller's may be the null stream), ordered after the work
// already enqueued on the caller's stream and before anything enqueued on it
// later: the call returns only when its result is complete.
static rexii_status run_problem(const rexii_swe_op* op, const double* f, double* u, double t,
                                const rexii_opts* opts_in, void* ws, size_t ws_bytes,
                                hipStream_t stream, rexii_report* rep, const std::vector<cd>* shifts,
                                double2* xout) {
  {
    // argument checks that need no device
    rexii_status v = validate_op(op);
    if (v != REXII_OK) return v;
    if (!f || (!u && !xout)) return set_error(REXII_ERR_INVALID_ARG, "NULL state pointer");
    if (!(t >= 0.0) || !std::isfinite(t)) return set_error(REXII_ERR_INVALID_ARG, "t must be finite and >= 0");
    if (op->H_field) return set_error(REXII_ERR_INVALID_ARG, "variable depth is not supported by this entry point");
  }
  hipStream_t own = nullptr;
  hipEvent_t ev = nullptr;
  if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess)
    return set_error(REXII_ERR_HIP, "hipStreamCreateWithFlags failed");
  rexii_status st = REXII_OK;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, stream) != hipSuccess ||
      hipStreamWaitEvent(own, ev, 0) != hipSuccess) {
    st = set_error(REXII_ERR_HIP, "could not order the private stream after the caller's stream");
  } else {
    st = run_problem_on(op, f, u, t, opts_in, ws, ws_bytes, own, rep, shifts, xout);
  }
  const std::string msg = g_err;
  if (hipStreamSynchronize(own) != hipSuccess && st == REXII_OK) st = set_error(REXII_ERR_HIP, "stream sync failed");
  if (ev) (void)hipEventDestroy(ev);
  (void)hipStreamDestroy(own);
  if (st != REXII_OK) g_err = msg.empty() ? g_err : msg;
  return st;
}

static rexii_status run_problem_on(const rexii_swe_op* op, const double* f, double* u, double t,
                                   const rexii_opts* opts_in, void* ws, size_t ws_bytes,
                                   hipStream_t stream, rexii_report* rep, const std::vector<cd>* shifts,
                                   double2* xout) {
  const auto t0 = std::chrono::steady_clock::now();
  rexii_status st = validate_op(op);
  if (st != REXII_OK) return st;
  if (op->H_field) return set_error(REXII_ERR_INVALID_ARG, "variable depth is not supported by this entry point");
  if (!f || (!u && !xout)) return set_error(REXII_ERR_INVALID_ARG, "NULL state pointer");
  if (!(t >= 0.0) || !std::isfinite(t)) return set_error(REXII_ERR_INVALID_ARG, "t must be finite and >= 0");
  const size_t n = size_t(op->nx) * op->ny;
  if (u && (u < f + 3 * n && f < u + 3 * n)) return set_error(REXII_ERR_INVALID_ARG, "u overlaps f");
  rexii_opts o = resolve_opts(opts_in);
  try {
    if (t == 0.0 && !shifts) {
      launch_copy(f, u, 3 * n, stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(stream));
      if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->t = 0.0;
      }
      return clear_error();
    }
    // workspace: sized for the unpaired plan, an upper bound of every variant
    Plan pl;
    st = build_plan(op, t, o, true, false, pl);
    if (st != REXII_OK) return st;
    if (shifts) pl.B = std::max(1, std::min<int>(pl.B, int(shifts->size())));
    const size_t need = plan_bytes(pl);
    Arena ar(ws, ws_bytes);
    if (!ws) {
      ar.reserve_own(need);
    } else if (ws_bytes < need) {
      return set_error(REXII_ERR_WORKSPACE, "workspace smaller than rexii_workspace_size()");
    }
    double* DZ = ar.take<double>(2 * n);
    int* small = ar.take<int>(64);
    // input checks and velocity derivatives
    int* flags = nullptr;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&flags), 4 * sizeof(int), hipHostMallocDefault));
    struct FreeHost {
      int* p;
      ~FreeHost() { (void)hipHostFree(p); }
    } fh{flags};
    launch_fill_zero(reinterpret_cast<double*>(small), 8, stream);
    launch_prep(f, op->nx, op->ny, DZ, DZ + n, small, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(flags, small, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (flags[0] & 1) return set_error(REXII_ERR_NONFINITE, "non-finite value in f");
    const bool has_vel = (flags[0] & 2) != 0;
    const bool div_free = (flags[0] & 4) == 0;

    st = build_plan(op, t, o, has_vel, div_free && !shifts, pl);
    if (st != REXII_OK) return st;
    if (shifts) {
      // explicit shifts: one solve per shift, no weights
      pl.paired = false;
      pl.solves.clear();
      const double g = op->g, H = op->H0, fc = op->f_cor;
      for (size_t k = 0; k < shifts->size(); ++k) {
        const cd zk = (*shifts)[k];
        const cd den = zk * zk + t * t * fc * fc;
        SolveDesc s;
        s.m1 = -zk / den;
        s.m2 = -t * fc / den;
        const cd sig = t * t * g * H * zk / den;
        s.zeta = den / (t * t * g * H);
        s.a1 = t * H * s.m1;
        s.a2 = t * H * s.m2;
        s.inv_sigma = 1.0 / sig;
        s.c0 = s.c1 = s.c2 = 0.0;
        s.cost = 0.0;
        s.pole = int(k);
        pl.solves.push_back(s);
      }
      pl.B = std::max(1, std::min<int>(pl.B, int(pl.solves.size())));
      pl.pole_tol = o.tol;
    }
    Engine e(pl, stream);
    e.setup(ar, f, DZ, small);
    if (o.precision == REXII_PREC_MIXED)
      e.run<float>(f, xout);
    else
      e.run<double>(f, xout);
    if (!xout) {
      launch_reconstruct(f, e.A, op->nx, op->ny, pl.S1, pl.S2, t * op->g, pl.has_vel ? 1 : 0, u, stream);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_report(rep, pl, &e, secs);
    if (e.breakdowns > 0) return set_error(REXII_ERR_BREAKDOWN, "Krylov breakdown in a shifted solve");
    if (e.not_conv > 0) return set_error(REXII_ERR_NOT_CONVERGED, "a shifted solve reached max_iter");
    return clear_error();
  } catch (const HipError& he) {
    return set_error(he.st, he.msg);
  } catch (const std::bad_alloc&) {
    return set_error(REXII_ERR_OOM, "host allocation failed");
  }
}

}  // namespace rexii

using namespace rexii;

extern "C" {

void rexii_default_opts(rexii_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->h = 0.5;
  o->tol = 0.0;
  o->precision = REXII_PREC_FP64;
  o->max_iter = 50000;
  o->m0 = -1;
  o->rho = 0.0;
  o->pole_batch = 0;
  o->pair_conjugate = 1;
  o->inner_tol = 1e-4;
}

const char* rexii_last_error(void) { return g_err.c_str(); }

rexii_status rexii_rho(const rexii_swe_op* op, hipStream_t stream, double* rho) {
  (void)stream;
  rexii_status st = validate_op(op);
  if (st != REXII_OK) return st;
  if (!rho) return set_error(REXII_ERR_INVALID_ARG, "rho is NULL");
  if (op->H_field) return set_error(REXII_ERR_INVALID_ARG, "variable depth: not supported yet");
  *rho = rho_const(op->nx, op->ny, op->g, op->H0, op->f_cor);
  return clear_error();
}

rexii_status rexii_workspace_size(const rexii_swe_op* op, const rexii_opts* opts, double t, size_t* bytes) {
  rexii_status st = validate_op(op);
  if (st != REXII_OK) return st;
  if (!bytes) return set_error(REXII_ERR_INVALID_ARG, "bytes is NULL");
  if (!(t > 0.0)) {
    *bytes = 0;
    return clear_error();
  }
  rexii_opts o = resolve_opts(opts);
  Plan pl;
  // sized for the unpaired case (an upper bound)
  st = build_plan(op, t, o, true, false, pl);
  if (st != REXII_OK) return st;
  *bytes = plan_bytes(pl);
  return clear_error();
}

rexii_status rexii_apply(const rexii_swe_op* op, const double* f, double* u, double t, const rexii_opts* opts,
                         void* workspace, size_t ws_bytes, hipStream_t stream, rexii_report* rep) {
  return run_problem(op, f, u, t, opts, workspace, ws_bytes, stream, rep, nullptr, nullptr);
}

rexii_status rexii_shifted_solve(const rexii_swe_op* op, const double* f, double t, int32_t npoles, const double* z,
                                 double* x, const rexii_opts* opts, void* workspace, size_t ws_bytes,
                                 hipStream_t stream, rexii_report* rep) {
  if (npoles <= 0 || !z || !x) return set_error(REXII_ERR_INVALID_ARG, "need npoles > 0, z and x");
  if (!(t > 0.0)) return set_error(REXII_ERR_INVALID_ARG, "t must be > 0");
  std::vector<cd> sh(npoles);
  for (int k = 0; k < npoles; ++k) {
    sh[k] = cd(z[2 * k], z[2 * k + 1]);
    if (!(sh[k].real() != 0.0) || !std::isfinite(sh[k].real()) || !std::isfinite(sh[k].imag()))
      return set_error(REXII_ERR_INVALID_ARG, "shifts need a finite, non-zero real part");
  }
  return run_problem(op, f, nullptr, t, opts, workspace, ws_bytes, stream, rep, &sh,
                     reinterpret_cast<double2*>(x));
}

rexii_status rexii_apply_adjoint(const rexii_swe_op*, const double*, const double*, double*, double*, double,
                                 const rexii_opts*, void*, size_t, hipStream_t, rexii_report*) {
  return set_error(REXII_ERR_INVALID_ARG, "rexii_apply_adjoint: not implemented yet");
}

rexii_status rexii_apply_batched(int32_t, const rexii_swe_op*, const double* const*, double* const*, const double*,
                                 const rexii_opts*, void*, size_t, hipStream_t, rexii_report*) {
  return set_error(REXII_ERR_INVALID_ARG, "rexii_apply_batched: not implemented yet");
}

}  // extern "C"
