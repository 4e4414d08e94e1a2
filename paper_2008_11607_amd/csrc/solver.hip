// Host side of the REXII shifted-solve path and the C ABI entry points.
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
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "kernels_fft.h"
#include "kernels_lz.h"
#include "precond.h"
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
  // bytes handed out so far; reset(m) gives back everything taken after m
  size_t mark() const { return off_; }
  void reset(size_t m) { off_ = m; }
  size_t remaining() const { return cap_ - off_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, off_ = 0;
  bool own_;
};

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// Per-device resources reused across calls: the private stream the solver
// runs on (graph capture needs a capturable stream), an event that orders it
// after the caller's stream, pinned host buffers (device-to-host reads, the
// chunk counters) and the instantiated chunk graphs of recent calls.  One
// call holds a device's set at a time; a call that finds it busy (another
// host thread) creates and frees its own, as every call did before.  The
// sets live until the process ends.
// ---------------------------------------------------------------------------
struct DevCtx {
  std::mutex mu;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  void* pin = nullptr;         // staging of device-to-host reads
  size_t pin_bytes = 0;
  int* hcount = nullptr;       // 64 ints: counters the chunk graphs copy out
  char* dscr = nullptr;        // small device scratch (depth maximum)
  struct Graph {
    std::vector<char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::deque<Graph> graphs;    // most recent first
  static constexpr size_t kGraphs = 6;
  static constexpr size_t kScratch = 64 << 10;
};

static std::mutex g_ctx_mu;
static std::map<int, DevCtx*> g_ctx;
static thread_local DevCtx* tl_ctx = nullptr;   // the set the calling thread holds

static DevCtx* device_ctx() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  DevCtx*& c = g_ctx[dev];
  if (!c) c = new DevCtx();
  return c;
}

// Pinned host memory of at least `bytes` from the held set (grown on
// demand), or nullptr when the thread holds none.
static void* ctx_pinned(size_t bytes) {
  DevCtx* c = tl_ctx;
  if (!c) return nullptr;
  if (c->pin_bytes < bytes) {
    if (c->pin) (void)hipHostFree(c->pin);
    c->pin = nullptr;
    c->pin_bytes = 0;
    const size_t nb = std::max<size_t>(bytes, size_t(1) << 20);
    HIPCHK(hipHostMalloc(&c->pin, nb, hipHostMallocDefault));
    c->pin_bytes = nb;
  }
  return c->pin;
}

// Device-to-host read of `bytes` bytes ordered on `st`: through a pinned
// staging buffer, then the stream is drained (a copy into pageable memory
// followed by a stream synchronisation has returned stale data under the
// profiler's kernel tracing).
static void read_to_host(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  void* pin = ctx_pinned(bytes);
  void* own = nullptr;
  if (!pin) {
    HIPCHK(hipHostMalloc(&own, bytes, hipHostMallocDefault));
    pin = own;
  }
  struct Free {
    void* p;
    ~Free() {
      if (p) (void)hipHostFree(p);
    }
  } fr{own};
  HIPCHK(hipMemcpyAsync(pin, src, bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(dst, pin, bytes);
}

// Copies of a constant host table in device memory, one per device, made
// on first use (a synchronous upload).  When the table goes, its copies are
// only queued; the next call that makes a copy frees them, so a call that
// must not allocate or free (it never makes copies) frees none either.  The
// tables below live in caches that are never destroyed, so nothing is freed
// while the process exits.
class DevCopies {
 public:
  ~DevCopies() {
    std::lock_guard<std::mutex> lk(retired_mu());
    for (auto& kv : ptr_) retired().push_back(kv.second);
  }
  // the current device's copy of v (made now if there is none)
  const double* get(const std::vector<double>& v) const {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    {
      std::lock_guard<std::mutex> lk(retired_mu());
      for (void* p : retired()) (void)hipFree(p);
      retired().clear();
    }
    std::lock_guard<std::mutex> lk(mu_);
    auto it = ptr_.find(dev);
    if (it != ptr_.end()) return it->second;
    double* d = nullptr;
    HIPCHK(hipMalloc(reinterpret_cast<void**>(&d), std::max<size_t>(1, v.size()) * sizeof(double)));
    const hipError_t e = hipMemcpy(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      throw HipError{REXII_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e)};
    }
    ptr_.emplace(dev, d);
    return d;
  }

 private:
  static std::mutex& retired_mu() {
    static std::mutex& m = *new std::mutex();
    return m;
  }
  static std::vector<void*>& retired() {
    static std::vector<void*>& v = *new std::vector<void*>();
    return v;
  }
  mutable std::mutex mu_;
  mutable std::map<int, double*> ptr_;
};

// Axis symbols s(k) of a grid, x wavenumbers 0..nx/2 then y wavenumbers
// 0..ny-1, formed once per (nx, ny, derivative) and kept (8 most recent),
// with device copies made on demand.
struct SymTable {
  std::vector<double> s;
  DevCopies dev;
};

static std::shared_ptr<const SymTable> symbol_table(int nx, int ny, int deriv) {
  static std::mutex mu;
  using Entry = std::pair<std::tuple<int, int, int>, std::shared_ptr<const SymTable>>;
  static std::deque<Entry>& cache = *new std::deque<Entry>();
  const auto key = std::make_tuple(nx, ny, deriv);
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto it = cache.begin(); it != cache.end(); ++it)
      if (it->first == key) {
        auto hit = *it;
        cache.erase(it);
        cache.push_front(hit);
        return hit.second;
      }
  }
  auto st = std::make_shared<SymTable>();
  st->s.resize(size_t(nx / 2 + 1) + ny);
  for (int k = 0; k <= nx / 2; ++k) st->s[k] = axis_symbol(k, nx, deriv);
  for (int k = 0; k < ny; ++k) st->s[nx / 2 + 1 + k] = axis_symbol(k, ny, deriv);
  std::shared_ptr<const SymTable> out = st;
  std::lock_guard<std::mutex> lk(mu);
  for (auto it = cache.begin(); it != cache.end(); ++it)
    if (it->first == key) {
      cache.erase(it);
      break;
    }
  cache.push_front({key, out});
  while (cache.size() > 8) cache.pop_back();
  return out;
}

// ---------------------------------------------------------------------------
// problem description
// ---------------------------------------------------------------------------
struct SolveDesc {
  cd zeta, a1, a2;     // Helmholtz shift and RHS coefficients
  cd gamma = 0.0, sc = 1.0;  // flux-form (BiCGStab) path: cross-term factor, RHS scale
  cd c0, c1, c2;       // accumulation weights (A_j += Re(c_j y))
  cd inv_sigma, m1, m2;
  double cost;         // expected Krylov iterations at tol (Chebyshev estimate)
  double tol = 0.0;    // relative residual this solve is driven to
  // Error bound of the weighted sum (Theorem 1 with cond(V) = 1 in the W-norm,
  // every resolvent of norm <= 1/|h mu|): the solve contributes
  // wsum * sqrt(g) |r3| / |f|_W, wsum = sum of |w_k| / |h mu| over the poles
  // it serves and r3 = rscale * (the solver's residual) the eta-row residual of
  // the 3-field system (the velocity rows are exact).
  double wsum = 0.0;
  double rscale = 1.0;
  double ref2 = 0.0;   // stop-test reference (SolveDev::ref2)
  int yidx = -1;       // row of the kept solutions (-1: the queue position)
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
  bool bicg = false;   // flux-form operator solved by BiCGStab
  double hmax = 0.0;   // max depth (variable depth)
  int B;               // slots per batch
  int chunk;           // inner iterations per graph replay
  bool profile = false;
  std::vector<cd> z, w;
  std::vector<cd> w_fwd;   // forward weights (w holds the adjoint ones in adjoint plans)
  std::vector<SolveDesc> solves;
  double S1 = 0, S2 = 0;
  bool shifts = false;     // explicit shifts (resolvents), no weighted sum
};

struct GridGeo {
  int tiles_x, tiles_y, nblk;
};
// work items are kTX x th tiles (th = kTY for COCG; 16 or 32 for BiCGStab)
static GridGeo make_geo(int nx, int ny, int th) {
  GridGeo g;
  g.tiles_x = (nx + kTX - 1) / kTX;
  g.tiles_y = (ny + th - 1) / th;
  g.nblk = g.tiles_x * g.tiles_y;
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
  if (r.max_iter < 0) r.max_iter = 0;   // 0: caps per solve (Krylov paths), 50000 (shared-Krylov m)
  if (r.inner_tol <= 0.0) r.inner_tol = 1e-4;
  return r;
}

// Pole set, shifts, weights and scheduling (host, FP64).
static rexii_status build_plan(const rexii_swe_op* op, double t, const rexii_opts& o, bool has_vel,
                               bool div_free, Plan& pl, bool adjoint = false, double hmax = 0.0) {
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
  pl.bicg = (op->H_field != nullptr) || (o.method == 1) || (o.method == 2);
  pl.hmax = op->H_field ? hmax : op->H0;
  // the two poles of a term give conjugate systems only for the symmetric
  // constant-depth operator
  pl.paired = (o.pair_conjugate != 0) && div_free && !pl.bicg;
  if (!(o.h > 0.0 && o.h < M_PI)) return set_error(REXII_ERR_INVALID_ARG, "h must be in (0, pi)");
  if (!(o.tol > 0.0 && o.tol < 1.0)) return set_error(REXII_ERR_INVALID_ARG, "tol must be in (0, 1)");
  if (o.tile_rows != 0 && o.tile_rows != 16 && o.tile_rows != 32)
    return set_error(REXII_ERR_INVALID_ARG, "tile_rows must be 0, 16 or 32");
  if (o.scheme != REXII_SCHEME_REXII)
    return set_error(REXII_ERR_INVALID_ARG, "the REXI scheme is available on the Fourier path only");
  if (o.precision != REXII_PREC_FP64 && o.precision != REXII_PREC_MIXED)
    return set_error(REXII_ERR_INVALID_ARG, "unknown precision");
  if (o.method < 0 || o.method > 2) return set_error(REXII_ERR_INVALID_ARG, "unknown method");
  if (op->H_field && !(hmax > 0.0)) return set_error(REXII_ERR_INVALID_ARG, "variable depth needs max H > 0");
  pl.rho = (o.rho > 0.0) ? o.rho
           : (op->H_field ? rho_bound_var(op->nx, op->ny, op->g, hmax, op->f_cor)
                          : rho_const(op->nx, op->ny, op->g, op->H0, op->f_cor));
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
  pl.w_fwd = pl.w;
  if (adjoint) {
    // r(tA)^T = W Re sum_k w'_k (tA - z_k)^{-1} W^{-1}: with A^T = -W A W^{-1}
    // the transposed resolvent at z_k is -W (tA + z_k)^{-1} W^{-1}, and
    // -z_{n,1} = conj(z_{n,2}), so the same poles serve with
    // w'_{n,1} = -conj(w_{n,2}), w'_{n,2} = -conj(w_{n,1}).
    for (int k = 0; k + 1 < pl.P; k += 2) {
      const cd a = pl.w[k], b = pl.w[k + 1];
      pl.w[k] = -std::conj(b);
      pl.w[k + 1] = -std::conj(a);
    }
  }

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
  if (pl.bicg) {
    // flux form: (L_H + gamma C_H - zeta) eta = sc (eta0 + t m1 D_H + t m2 Z_H),
    // solved for eta itself (no 1/sigma scaling)
    for (int k = 0; k < pl.P; ++k) {
      const cd zk = pl.z[k];
      const cd den = zk * zk + t * t * fc * fc;
      SolveDesc s;
      s.zeta = den / (t * t * g);
      s.gamma = t * fc / zk;
      s.sc = s.zeta / zk;
      s.a1 = t * m1[k];
      s.a2 = t * m2[k];
      s.inv_sigma = 1.0;
      s.m1 = m1[k];
      s.m2 = m2[k];
      s.c0 = pl.w[k];
      s.c1 = pl.w[k] * m1[k];
      s.c2 = pl.w[k] * m2[k];
      s.cost = cheb_cost(s.zeta / pl.hmax, lmax, pl.pole_tol);
      s.pole = k;
      pl.solves.push_back(s);
    }
  } else if (pl.paired) {
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
  // Per-solve tolerances.  With a_s = (sum of |w_k| over the poles solve s
  // serves) / |h mu|, the error of the weighted sum is at most
  // sum_s a_s eps_s ||f|| (each resolvent has norm <= 1/|h mu|, A being
  // skew), so any eps_s with sum_s a_s eps_s <= tol meets tol.  The uniform
  // choice eps_s = tol / kappa_sum (kappa_sum = sum_s a_s) over-solves the
  // light poles (the two poles of a term differ ~160-fold in weight); an
  // equal share of the bound, eps_s = tol / (S a_s), minimises the total
  // digits sum_s log(1/eps_s) (Krylov work is about linear in digits),
  // capped at 1e-2.
  {
    const double hmu = std::abs(pl.h * mu());
    // iterations per e-fold of each solve (Chebyshev estimate), clamped to
    // [1/4, 4] x the median so that one badly estimated solve cannot take
    // the budget of the others
    std::vector<double> c(pl.solves.size());
    for (size_t i = 0; i < c.size(); ++i)
      c[i] = cheb_cost(pl.bicg ? pl.solves[i].zeta / pl.hmax : pl.solves[i].zeta, lmax, 2.0 / M_E);
    std::vector<double> cs = c;
    std::nth_element(cs.begin(), cs.begin() + cs.size() / 2, cs.end());
    const double cmed = cs.empty() ? 1.0 : std::min(cs[cs.size() / 2], 1e6);
    double csum = 0.0;
    for (double& ci : c) {
      ci = std::min(std::max(ci, 0.25 * cmed), 4.0 * cmed);
      csum += ci;
    }
    pl.pole_tol = 1.0;
    for (size_t i = 0; i < c.size(); ++i) {
      SolveDesc& sd = pl.solves[i];
      double a = std::abs(pl.w[sd.pole]) / hmu;
      if (pl.paired) a += std::abs(pl.w[sd.pole + 1]) / hmu;
      sd.tol = (a > 0.0) ? std::min(pl.tol * c[i] / (a * csum), 1e-2) : 1e-2;
      sd.wsum = a;
      // flux form: the solver's system is the eta row scaled by sc
      sd.rscale = pl.bicg ? 1.0 / std::abs(sd.sc) : 1.0;
      pl.pole_tol = std::min(pl.pole_tol, sd.tol);
      sd.cost = cheb_cost(pl.bicg ? sd.zeta / pl.hmax : sd.zeta, lmax, sd.tol);
    }
  }
  // most expensive first (longest-processing-time order for the slot queue)
  std::stable_sort(pl.solves.begin(), pl.solves.end(),
                   [](const SolveDesc& a, const SolveDesc& b) { return a.cost > b.cost; });
  pl.B = o.pole_batch;
  pl.chunk = 16;
  return REXII_OK;
}

// Slots for a set of problems: enough tiles to fill the chip several times
// over, within a memory budget, never more than the number of solves.
// Slots: by default enough for about 16384 work items (tiles) per pass,
// counted with the solve-weighted mean tile count when problems differ in
// size; at most a 24 GiB engine.
static int choose_slots(int requested, size_t max_points, double mean_nblk, size_t nsolves, int precision, int nvec) {
  int B = requested;
  if (B <= 0) {
    B = int(std::ceil(16384.0 / std::max(1.0, mean_nblk)));
    B = std::max(8, std::min(B, 1024));
  }
  B = std::min(B, kMaxSlots);
  const size_t per_slot = max_points * (16 + nvec * inner_elem_bytes(precision));
  const size_t budget = size_t(24) << 30;
  B = int(std::max<size_t>(1, std::min<size_t>(size_t(B), budget / per_slot)));
  B = int(std::min<size_t>(size_t(B), std::max<size_t>(1, nsolves)));
  return B;
}

// ---------------------------------------------------------------------------
// the slot engine (one or several problems)
// ---------------------------------------------------------------------------
struct Problem {
  Plan pl;
  const double* f = nullptr;   // device [3][ny][nx]
  double* DZ = nullptr;        // device div / curl of the initial velocity
  double* A = nullptr;         // device accumulators [3][ny][nx]
  const double* H = nullptr;   // device depth field (flux-form path)
  const void* Hin = nullptr;   // the depth in the inner-iteration type
  double fw2 = 0.0;            // ||f||_W^2, W = diag(g, H, H)
  size_t n() const { return size_t(pl.nx) * pl.ny; }
};

struct EngineSize {
  int B = 1, cap = 0, cap_blk = 0, S = 0, ninst = 0;
  int method = 0;   // 0 COCG, 1 BiCGStab
  int th = kTY;     // rows of a work tile
  int nvec = 5;     // inner-precision vectors per slot
  size_t eb = 16;
};

static EngineSize engine_size(const std::vector<Problem*>& probs, int requested_B, int precision,
                              int tile_rows) {
  EngineSize z;
  size_t maxp = 0;
  int min_nb = 0;
  z.method = 0;
  for (Problem* p : probs) z.method = std::max(z.method, p->pl.bicg ? 1 : 0);
  // BiCGStab default tile: 64 x 32 in mixed precision, 64 x 16 in FP64 (its
  // FP64 tiles need twice the LDS and registers; measured at 2048^2: 32 rows
  // 7% faster in mixed precision, 16 rows 7% faster in FP64)
  const int th_default = (precision == REXII_PREC_MIXED) ? kTYB : 16;
  z.th = (z.method == 1) ? ((tile_rows == 16 || tile_rows == 32) ? tile_rows : th_default) : kTY;
  for (Problem* p : probs) {
    maxp = std::max(maxp, p->n());
    const int nb = make_geo(p->pl.nx, p->pl.ny, z.th).nblk;
    z.cap_blk = std::max(z.cap_blk, nb);
    z.S += int(p->pl.solves.size());
    min_nb = (min_nb == 0) ? nb : std::min(min_nb, nb);
  }
  // the smallest problem's tile count, in units of kTX x kTY tiles: slots
  // enough to fill the GPU while only the smallest problems are left (the
  // queue runs the most expensive solves first); memory caps the count
  const double mean_nblk = double(std::max(1, min_nb)) * double(z.th) / kTY;
  z.cap = int(maxp);
  z.ninst = int(probs.size());
  z.eb = inner_elem_bytes(precision);
  z.nvec = z.method ? 8 : 5;
  z.B = choose_slots(requested_B, maxp, mean_nblk, size_t(z.S), precision, z.nvec);
  return z;
}

// device bytes of the engine (problem arrays D0/Z0 and A and the kept
// solutions are counted by the caller)
static size_t engine_bytes(const EngineSize& z) {
  size_t b = 0;
  b += al256(z.B * sizeof(Slot)) + al256(z.ninst * sizeof(Inst));
  b += al256(z.S * sizeof(SolveDev)) + al256(z.S * sizeof(SolveStat));
  b += al256(sizeof(int)) + al256((z.B + 2) * sizeof(int)) + al256(4 * sizeof(int));
  b += al256(size_t(z.B) * z.cap_blk * kNDots * sizeof(double));
  b += al256(size_t(z.B) * (z.cap_blk + 7) * sizeof(int2));
  b += al256(size_t(z.B) * z.cap * 16);
  b += size_t(z.nvec) * al256(size_t(z.B) * z.cap * z.eb);
  b += al256(16 * sizeof(int));
  return b;
}

// Iteration cap of one solve: opts.max_iter if set, else from its Chebyshev
// estimate: 4x in FP32 inner arithmetic (a mixed-precision solve past it is
// re-run in FP64), 20x in FP64.
static int solve_cap(double cost, int precision, int user_max_iter) {
  if (user_max_iter > 0) return user_max_iter;
  const double c = std::isfinite(cost) ? std::max(cost, 0.0) : 1e9;
  const double cap = (precision == REXII_PREC_MIXED) ? 4.0 * c + 2000.0 : 20.0 * c + 5000.0;
  return int(std::min(cap, 1.0e9));
}

// D/Z, A, a small block, a constant depth field when a constant-depth
// problem runs through the flux-form path, and an FP32 copy of the depth
// for the mixed-precision inner iterations
static size_t problem_bytes(const Problem& p) {
  return al256(2 * p.n() * 8) + al256(3 * p.n() * 8) + al256((8 + 256) * 8) + al256(p.n() * 8) + al256(p.n() * 4);
}

struct Engine {
  hipStream_t st;
  EngineSize z;
  int precision = 0, chunk = 16, grid = 0;
  bool profile = false;
  Eng e{};
  int* hcount = nullptr;   // pinned host mirror of the counters
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<SolveStat> stats;
  std::vector<int> solve_inst;    // instance of each queued solve
  std::vector<int> solve_index;   // index of the solve within its instance
  // profiling (opts.profile)
  std::vector<hipEvent_t> evs;
  int64_t launches = 0;
  double kernel_ms = 0.0;
  static constexpr int kBcgEvents = 7;   // around the 6 kernels of a BiCGStab step
  double step_ms[kBcgEvents - 1] = {};
  double u1_bytes = 0.0;
  double pass_bytes = 0.0;
  std::vector<size_t> inst_points;
  std::vector<char> inst_vel;
  std::vector<const Plan*> plans;  // plan of each instance
  int max_cap = 0;                // largest per-solve iteration cap
  std::vector<char> retried;      // per queued solve: re-run in FP64
  double solve_seconds = 0.0;     // host wall time of run()

  bool graph_shared = false;    // gexec / graph belong to the device set's cache
  bool hcount_shared = false;   // hcount belongs to the device set

  explicit Engine(hipStream_t s) : st(s) {
    // every byte of e (padding included) is defined: e keys the graph cache
    std::memset(static_cast<void*>(&e), 0, sizeof(e));
  }
  ~Engine() {
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    if (!graph_shared) {
      if (gexec) (void)hipGraphExecDestroy(gexec);
      if (graph) (void)hipGraphDestroy(graph);
    }
    if (hcount && !hcount_shared) (void)hipHostFree(hcount);
  }

  // yout: device [rows][ystride] complex128 kept solutions (row
  // SolveDesc::yidx, or the queue position when that is -1) or nullptr to
  // accumulate only.
  void setup(Arena& ar, const std::vector<Problem*>& probs, const EngineSize& zs, int prec, int user_max_iter,
             double inner_eta, bool prof, double2* yout, int ystride) {
    z = zs;
    precision = prec;
    profile = prof;
    e.B = z.B;
    e.S = z.S;
    e.method = z.method;
    e.th = z.th;
    e.d_is_f32 = (prec == REXII_PREC_MIXED) ? 1 : 0;
    e.retry = e.d_is_f32;
    e.cap = z.cap;
    e.cap_blk = z.cap_blk;
    e.inner_eta2 = inner_eta * inner_eta;
    e.slots = ar.take<Slot>(z.B);
    Inst* dinst = ar.take<Inst>(z.ninst);
    SolveDev* dsol = ar.take<SolveDev>(z.S);
    e.inst = dinst;
    e.solves = dsol;
    e.stats = ar.take<SolveStat>(z.S);
    e.next = ar.take<int>(1);
    e.work = ar.take<int>(z.B + 2);
    e.counter = ar.take<int>(4);
    e.items = ar.take<int2>(size_t(z.B) * (z.cap_blk + 7));   // 8 band lists of sum ceil(nb / 8) entries
    e.part = ar.take<double>(size_t(z.B) * z.cap_blk * kNDots);
    e.x64 = ar.take<double2>(size_t(z.B) * z.cap);
    e.d = ar.take<char>(size_t(z.B) * z.cap * z.eb);
    e.r0 = ar.take<char>(size_t(z.B) * z.cap * z.eb);
    e.r1 = ar.take<char>(size_t(z.B) * z.cap * z.eb);
    e.p0 = ar.take<char>(size_t(z.B) * z.cap * z.eb);
    e.p1 = ar.take<char>(size_t(z.B) * z.cap * z.eb);
    if (z.method == 1) {
      e.v0 = ar.take<char>(size_t(z.B) * z.cap * z.eb);
      e.v1 = ar.take<char>(size_t(z.B) * z.cap * z.eb);
      e.rh = ar.take<char>(size_t(z.B) * z.cap * z.eb);
    }
    e.yout = yout;
    e.ystride = ystride;
    e.dbg = ar.take<int>(16);

    plans.clear();
    for (Problem* p : probs) plans.push_back(&p->pl);
    // problem table
    std::vector<Inst> hinst(z.ninst);
    inst_points.resize(z.ninst);
    inst_vel.resize(z.ninst);
    for (int i = 0; i < z.ninst; ++i) {
      inst_points[i] = probs[i]->n();
      inst_vel[i] = probs[i]->pl.has_vel ? 1 : 0;
    }
    for (int i = 0; i < z.ninst; ++i) {
      const Plan& pl = probs[i]->pl;
      const GridGeo g = make_geo(pl.nx, pl.ny, z.th);
      Inst I;
      I.nx = pl.nx;
      I.ny = pl.ny;
      I.tiles_x = g.tiles_x;
      I.nblk = g.nblk;
      I.cx = 0.25 * double(pl.nx) * pl.nx;
      I.cy = 0.25 * double(pl.ny) * pl.ny;
      I.cxy = 0.25 * double(pl.nx) * pl.ny;
      I.H = probs[i]->H;
      I.Hin = probs[i]->Hin;
      I.eta0 = probs[i]->f;
      I.D0 = pl.has_vel ? probs[i]->DZ : nullptr;
      I.Z0 = pl.has_vel ? probs[i]->DZ + probs[i]->n() : nullptr;
      I.A = probs[i]->A;
      hinst[i] = I;
    }
    // solve queue: all problems' solves, most expensive first
    struct Q {
      double cost;
      int inst, idx;
    };
    std::vector<Q> q;
    for (int i = 0; i < z.ninst; ++i)
      for (size_t k = 0; k < probs[i]->pl.solves.size(); ++k) q.push_back({probs[i]->pl.solves[k].cost, i, int(k)});
    std::stable_sort(q.begin(), q.end(), [](const Q& a, const Q& b) { return a.cost > b.cost; });
    std::vector<SolveDev> hs(z.S);
    solve_inst.resize(z.S);
    solve_index.resize(z.S);
    for (int j = 0; j < z.S; ++j) {
      const Plan& pl = probs[q[j].inst]->pl;
      const SolveDesc& d = pl.solves[q[j].idx];
      SolveDev D;
      D.zeta = to_d2(d.zeta);
      D.a1 = to_d2(d.a1);
      D.a2 = to_d2(d.a2);
      D.c0 = to_d2(d.c0);
      D.c1 = to_d2(d.c1);
      D.c2 = to_d2(d.c2);
      D.gamma = to_d2(d.gamma);
      D.sc = to_d2(d.sc);
      D.tol2 = d.tol * d.tol;
      D.ref2 = d.ref2;
      D.inst = q[j].inst;
      D.max_it = solve_cap(d.cost, prec, user_max_iter);
      D.yidx = (d.yidx >= 0) ? d.yidx : j;
      D.pad = 0;
      max_cap = std::max(max_cap, D.max_it);
      hs[j] = D;
      solve_inst[j] = q[j].inst;
      solve_index[j] = q[j].idx;
    }
    HIPCHK(hipMemcpyAsync(dinst, hinst.data(), z.ninst * sizeof(Inst), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dsol, hs.data(), z.S * sizeof(SolveDev), hipMemcpyHostToDevice, st));
    // zero: slots (all idle), queue head, tile table, counters, x64
    launch_fill_zero(reinterpret_cast<double*>(e.slots), z.B * sizeof(Slot) / 8, st);
    launch_fill_zero(reinterpret_cast<double*>(e.next), 1, st);  // 8 bytes inside its 256-byte block
    launch_fill_zero(reinterpret_cast<double*>(e.work), (size_t(z.B + 2) * 4 + 7) / 8, st);
    launch_fill_zero(reinterpret_cast<double*>(e.counter), 2, st);
    launch_fill_zero(reinterpret_cast<double*>(e.dbg), 8, st);
    launch_fill_zero(reinterpret_cast<double*>(e.x64), size_t(z.B) * z.cap * 2, st);
    if (tl_ctx) {
      if (!tl_ctx->hcount)
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&tl_ctx->hcount), 64 * sizeof(int), hipHostMallocDefault));
      hcount = tl_ctx->hcount;
      hcount_shared = true;
    } else {
      HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hcount), 64 * sizeof(int), hipHostMallocDefault));
    }
    // persistent grid: every CU filled with as many blocks as fit
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int occ = (z.method == 1) ? bcg_occupancy(precision == REXII_PREC_MIXED ? 1 : 0, z.th)
                                    : pass_occupancy(precision == REXII_PREC_MIXED ? 1 : 0);
    // one work item (slot, tile) per block when every slot is live; never
    // fewer blocks than fill the chip
    const size_t items = size_t(z.B) * z.cap_blk;
    grid = int(std::max<size_t>(size_t(cus) * std::max(1, occ), items));
    grid = ((grid + 7) / 8) * 8;
    e.grid_small = ((cus * 4 + 7) / 8) * 8;
  }

  template <typename T>
  void enqueue_chunk(bool with_events) {
    launch_retire(e, st);
    launch_assign(e, st);
    for (int i = 0; i < chunk; ++i) {
      if (z.method == 1) {
        launch_bcg<T>(e, grid, st, with_events ? &evs[kBcgEvents * i] : nullptr);
      } else {
        if (with_events) HIPCHK(hipEventRecord(evs[2 * i], st));
        launch_pass<T>(e, grid, st);
        if (with_events) HIPCHK(hipEventRecord(evs[2 * i + 1], st));
        launch_pass_scalars(e, st);
      }
    }
    launch_count_finished(e, st);
    HIPCHK(hipMemcpyAsync(hcount, e.counter, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  }

  // The chunk's launches depend only on e (pointers, sizes, modes), the
  // grid, the chunk length, the inner type and the counter buffer: a graph
  // captured for the same values is replayed as it is.
  template <typename T>
  std::vector<char> graph_key() const {
    std::vector<char> k(sizeof(Eng) + 4 * sizeof(int) + sizeof(void*));
    char* p = k.data();
    std::memcpy(p, &e, sizeof(Eng));
    const int v[4] = {grid, chunk, int(sizeof(T)), z.method};
    std::memcpy(p + sizeof(Eng), v, sizeof(v));
    const void* hc = hcount;
    std::memcpy(p + sizeof(Eng) + sizeof(v), &hc, sizeof(void*));
    return k;
  }

  template <typename T>
  void build_graph() {
    DevCtx* c = tl_ctx;
    std::vector<char> key;
    if (c && hcount_shared) {
      key = graph_key<T>();
      for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it) {
        if (it->key == key) {
          DevCtx::Graph g = *it;
          c->graphs.erase(it);
          c->graphs.push_front(g);
          graph = g.graph;
          gexec = g.exec;
          graph_shared = true;
          return;
        }
      }
    }
    capture_graph<T>();
    if (c && hcount_shared) {
      // the set keeps the graph; the oldest beyond the limit is dropped (its
      // last replay belonged to an earlier, finished call)
      c->graphs.push_front(DevCtx::Graph{key, graph, gexec});
      graph_shared = true;
      while (c->graphs.size() > DevCtx::kGraphs) {
        DevCtx::Graph& old = c->graphs.back();
        (void)hipGraphExecDestroy(old.exec);
        (void)hipGraphDestroy(old.graph);
        c->graphs.pop_back();
      }
    }
  }

  template <typename T>
  void capture_graph() {
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_chunk<T>(false);
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(st, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    HIPCHK(hipStreamEndCapture(st, &graph));
    HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
  }

  // Runs the chunks until the queue drains (or max_chunks > 0 chunks have
  // run).  With max_chunks > 0 the time of chunks 2..max_chunks is returned
  // (ms, HIP events on the engine's stream) and no statistics are read.
  template <typename T>
  double run(int max_chunks = 0) {
    if (max_chunks > 0) {
      build_graph<T>();
      hipEvent_t a = nullptr, b = nullptr;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&b));
      HIPCHK(hipGraphLaunch(gexec, st));
      HIPCHK(hipEventRecord(a, st));
      for (int c = 1; c < max_chunks; ++c) HIPCHK(hipGraphLaunch(gexec, st));
      HIPCHK(hipEventRecord(b, st));
      HIPCHK(hipStreamSynchronize(st));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, a, b));
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      return double(ms);
    }
    if (profile) {
      evs.resize((z.method == 1 ? kBcgEvents : 2) * chunk);
      for (hipEvent_t& ev : evs) HIPCHK(hipEventCreate(&ev));
    } else {
      build_graph<T>();
    }
    const auto w0 = std::chrono::steady_clock::now();
    // $REXII_PROGRESS = seconds: a progress line on stderr at that interval
    // (long calls, e.g. large batches, report how far the queue has got)
    double every = 0.0;
    if (const char* pv = std::getenv("REXII_PROGRESS")) every = std::atof(pv);
    auto last = w0;
    // enough replays for every solve to run to its iteration cap in turn
    const int64_t per_slot = (int64_t(z.S) + z.B - 1) / z.B;
    const int64_t max_replays = per_slot * (int64_t(max_cap) / chunk + 8) + 8;
    for (int64_t rep = 0; rep < max_replays; ++rep) {
      if (profile) {
        enqueue_chunk<T>(true);
        HIPCHK(hipStreamSynchronize(st));
        for (int i = 0; i < chunk; ++i) {
          float ms = 0.f;
          if (z.method == 1) {
            const hipEvent_t* ev = &evs[kBcgEvents * i];
            for (int k = 0; k + 1 < kBcgEvents; ++k) {
              HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
              step_ms[k] += ms;
            }
            HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[kBcgEvents - 1]));
          } else {
            HIPCHK(hipEventElapsedTime(&ms, evs[2 * i], evs[2 * i + 1]));
          }
          kernel_ms += ms;
        }
        launches += chunk;
      } else {
        HIPCHK(hipGraphLaunch(gexec, st));
        HIPCHK(hipStreamSynchronize(st));
      }
      if (hcount[0] == 0) break;
      if (every > 0.0) {
        const auto now = std::chrono::steady_clock::now();
        if (std::chrono::duration<double>(now - last).count() >= every) {
          last = now;
          std::fprintf(stderr, "rexii: %d of %d solves started, %d slots working, %.0f s\n", hcount[1], z.S,
                       hcount[0], std::chrono::duration<double>(now - w0).count());
          std::fflush(stderr);
        }
      }
    }
    stats.resize(z.S);
    read_to_host(stats.data(), e.stats, z.S * sizeof(SolveStat), st);
    solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
#ifdef REXII_DEBUG_CHECKS
    int dbg[16];
    HIPCHK(hipMemcpy(dbg, e.dbg, sizeof(dbg), hipMemcpyDeviceToHost));
    fprintf(stderr, "rexii debug: nonuniform=%d fin_mismatch=%d missed_retire=%d nonzero_x0=%d stale_total=%d bad_tile=%d\n",
            dbg[0], dbg[1], dbg[2], dbg[3], dbg[4], dbg[5]);
#endif
    // algorithmic bytes of all pass launches (per point of the solve's grid)
    pass_bytes = 0.0;
    u1_bytes = 0.0;
    for (int j = 0; j < z.S; ++j) {
      const double pts = double(inst_points[solve_inst[j]]);
      if (z.method == 1) {
        // BiCGStab iteration: pass U2 reads p' and r_hat and writes v;
        // pass S reads r, v and r_hat; pass U1 reads r, v, p and d and
        // writes d, r and p (13 complex values); each pass reads the depth
        // in the inner type (hb).  Per inner solve, its first U1 reads no
        // d and its last reads no depth and writes only d; every inner
        // solve after the first starts by moving d into x64 (d read, x64
        // read and write).  A residual round reads eta0 (and D0, Z0 with
        // an initial velocity) and writes r, p and r_hat; after the first
        // it also reads x64, d and the FP64 depth.
        const double eb = double(z.eb), hb = (z.eb == 8) ? 4.0 : 8.0;
        const double dz = inst_vel[solve_inst[j]] ? 16.0 : 0.0;
        const int R = stats[j].rounds, solves_in = std::max(0, R - 1);
        pass_bytes += pts * (stats[j].it_total * (13.0 * eb + 3.0 * hb) - solves_in * (3.0 * eb + hb) +
                             std::max(0, R - 2) * (eb + 32.0) + (8.0 + dz + 3.0 * eb) +
                             solves_in * (32.0 + dz + 4.0 * eb));
        u1_bytes += pts * (stats[j].it_total * (7.0 * eb + hb) - solves_in * (3.0 * eb + hb) +
                           std::max(0, R - 2) * (eb + 32.0));
      } else {
        // COCG: an inner step reads d, r, p and writes them (6 complex
        // values; 4 in a step that leaves d alone); a residual step reads
        // x64 (16 B), d and eta0 (8 B) and writes r and p (the first reads
        // only eta0); each restart's prime step reads r; the first inner
        // step of every later round moves d into x64 (32 B instead of a d
        // read)
        const double eb = double(z.eb);
        const int R = stats[j].rounds;
        pass_bytes += pts * (6.0 * eb * stats[j].it_total - 2.0 * eb * stats[j].skips + (8.0 + 2.0 * eb) +
                             std::max(0, R - 1) * (24.0 + 3.0 * eb) + std::max(0, R - 1) * eb +
                             std::max(0, R - 2) * (32.0 - eb));
      }
    }
    return 0.0;
  }
};

constexpr int kHistBuckets = 20;

struct RunSummary {
  int max_iters = 0, max_rounds = 0, not_conv = 0, breakdowns = 0, stagnated = 0;
  int64_t total_iters = 0;
  int64_t total_skips = 0;   // COCG steps that left d alone
  double max_rel_res = 0.0;
  // error bound of the result (relative, W-norm): sum over the solves of
  // wsum * (achieved |r3|) / |f|_W; explicit shifts: the largest relative
  // residual
  double err_bound = 0.0;
  int retried = 0;
  int hist[kHistBuckets] = {};
};

static RunSummary summarize(const Engine& en, int inst) {
  RunSummary r;
  for (size_t j = 0; j < en.stats.size(); ++j) {
    if (inst >= 0 && en.solve_inst[j] != inst) continue;
    const SolveStat& s = en.stats[j];
    r.max_iters = std::max(r.max_iters, s.it_total);
    r.max_rounds = std::max(r.max_rounds, s.rounds);
    r.total_iters += s.it_total;
    r.total_skips += s.skips;
    if (s.status == kFailBreakdown) r.breakdowns++;
    else if (s.status != kDone) r.not_conv++;
    r.stagnated += s.stagnated;
    if (j < en.retried.size() && en.retried[j]) r.retried++;
    const double rel = s.bn2 > 0 ? std::sqrt(s.rn2 / s.bn2) : 0.0;
    r.max_rel_res = std::max(r.max_rel_res, rel);
    const Plan& pl = *en.plans[en.solve_inst[j]];
    const SolveDesc& d = pl.solves[en.solve_index[j]];
    if (pl.shifts) {
      r.err_bound = std::max(r.err_bound, rel);
    } else if (d.ref2 > 0.0) {
      r.err_bound += d.wsum * std::sqrt(s.rn2 / d.ref2);
    }
    int b = 0;
    for (unsigned v = unsigned(std::max(s.it_total, 1)); v > 1 && b < kHistBuckets - 1; v >>= 1) ++b;
    r.hist[b]++;
  }
  return r;
}

static void fill_report(rexii_report* rep, const Plan& pl, const Engine* en, int inst, double secs) {
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
  if (en) {
    const RunSummary r = summarize(*en, inst);
    rep->max_iters = r.max_iters;
    rep->max_refine = r.max_rounds;
    rep->not_converged = r.not_conv + r.breakdowns;
    rep->total_iters = r.total_iters;
    rep->max_rel_residual = r.max_rel_res;
    rep->stagnated = r.stagnated;
    rep->err_bound = r.err_bound;
    rep->retried = r.retried;
    rep->seconds_solve = en->solve_seconds;
    rep->hist_buckets = kHistBuckets;
    for (int k = 0; k < kHistBuckets; ++k) rep->iter_hist[k] = r.hist[k];
    const double eb = double(inner_elem_bytes(pl.precision));
    // COCG: a pass reads x, r, p and writes them back (6 complex values per
    // point; 4 in a step that leaves d alone); BiCGStab: an iteration moves
    // 13 complex values and reads the depth three times
    // preconditioned BiCGStab (method 2, FP64): the vector kernels move 26
    // complex values and read the depth twice per point and iteration, the
    // four transforms read and write their vector once each (8 more)
    const double per_pt = en->z.method == 2   ? 34.0 * 16.0 + 2.0 * 8.0
                          : en->z.method == 1 ? 13.0 * eb + 3.0 * (eb == 8.0 ? 4.0 : 8.0)
                                              : 6.0 * eb;
    rep->alg_bytes = double(pl.nx) * pl.ny *
                     (double(r.total_iters) * per_pt - (en->z.method == 0 ? double(r.total_skips) * 2.0 * eb : 0.0));
    rep->slots = en->z.B;
    rep->tile_rows = en->z.th;
    rep->kernel_launches = en->launches;
    rep->kernel_ms = en->kernel_ms;
    rep->kernel_bytes = en->pass_bytes;
    for (int k = 0; k < 6; ++k) rep->step_ms[k] = en->step_ms[k];
    rep->u1_bytes = en->u1_bytes;
  }
}

// explicit shifts: one solve per shift, no weights
static void shift_solves(const rexii_swe_op* op, double t, const std::vector<cd>& shifts, double tol, Plan& pl) {
  pl.paired = false;
  pl.solves.clear();
  const double g = op->g, H = op->H0, fc = op->f_cor;
  const double lmax = max_s2(op->nx) + max_s2(op->ny);
  for (size_t k = 0; k < shifts.size(); ++k) {
    const cd zk = shifts[k];
    const cd den = zk * zk + t * t * fc * fc;
    SolveDesc s;
    s.tol = tol;  // explicit shifts: every solve to the caller's tolerance
    s.m1 = -zk / den;
    s.m2 = -t * fc / den;
    if (pl.bicg) {
      s.zeta = den / (t * t * g);
      s.gamma = t * fc / zk;
      s.sc = s.zeta / zk;
      s.a1 = t * s.m1;
      s.a2 = t * s.m2;
      s.inv_sigma = 1.0;
      s.c0 = s.c1 = s.c2 = 0.0;
      s.cost = cheb_cost(s.zeta / pl.hmax, lmax, tol);
      s.rscale = 1.0 / std::abs(s.sc);
      s.pole = int(k);
      pl.solves.push_back(s);
      continue;
    }
    const cd sig = t * t * g * H * zk / den;
    s.zeta = den / (t * t * g * H);
    s.a1 = t * H * s.m1;
    s.a2 = t * H * s.m2;
    s.inv_sigma = 1.0 / sig;
    s.c0 = s.c1 = s.c2 = 0.0;
    s.cost = cheb_cost(s.zeta, lmax, tol);
    s.pole = int(k);
    pl.solves.push_back(s);
  }
  pl.pole_tol = tol;
  pl.shifts = true;
}

// ---------------------------------------------------------------------------
// jobs: the problems of one call, run through one slot engine
// ---------------------------------------------------------------------------
struct JobItem {
  const rexii_swe_op* op = nullptr;
  const double* f = nullptr;              // device right-hand state
  double t = 0.0;
  double* u = nullptr;                    // device output (nullptr: none)
  bool adjoint = false;                   // transposed-operator weights
  const std::vector<cd>* shifts = nullptr;// explicit shifts (resolvents)
  double2* xout = nullptr;                // resolvent output
  rexii_report* rep = nullptr;
  bool skip = false;                      // t == 0: u = f
  double hmax = 0.0;                      // max of the depth field (variable depth)
};

// max of a device depth field (and its validity), synchronous on `st`
static double device_hmax(const double* H, size_t n, hipStream_t st) {
  const int nb = prep_vh_blocks();
  const size_t need = 256 + nb * sizeof(double);
  char* buf = nullptr;
  char* own = nullptr;
  if (tl_ctx && need <= DevCtx::kScratch) {
    if (!tl_ctx->dscr) HIPCHK(hipMalloc(reinterpret_cast<void**>(&tl_ctx->dscr), DevCtx::kScratch));
    buf = tl_ctx->dscr;
  } else {
    HIPCHK(hipMalloc(reinterpret_cast<void**>(&own), need));
    buf = own;
  }
  struct FreeDev {
    char* p;
    ~FreeDev() {
      if (p) (void)hipFree(p);
    }
  } fd{own};
  int* dfl = reinterpret_cast<int*>(buf);
  double* part = reinterpret_cast<double*>(buf + 256);
  launch_fill_zero(reinterpret_cast<double*>(dfl), 1, st);
  launch_hmax(H, n, dfl, part, st);
  HIPCHK(hipGetLastError());
  std::vector<double> hp(nb);
  int fl = 0;
  read_to_host(hp.data(), part, nb * sizeof(double), st);
  read_to_host(&fl, dfl, sizeof(int), st);
  if (fl & 8) throw HipError{REXII_ERR_NONFINITE, "depth field has a non-finite or non-positive value"};
  double m = 0.0;
  for (double v : hp) m = std::max(m, v);
  return m;
}

// Sizing plans: unpaired with velocity, an upper bound of every variant.
static rexii_status sizing_plan(const JobItem& it, const rexii_opts& o, Problem& pb) {
  rexii_status st = build_plan(it.op, it.t, o, true, false, pb.pl, it.adjoint, it.hmax);
  if (st != REXII_OK) return st;
  if (it.shifts) shift_solves(it.op, it.t, *it.shifts, o.tol, pb.pl);
  return REXII_OK;
}

// Preconditioned solver (method 2): slot count and device bytes.
// damping of the preconditioner's shift (precond.hip); measured on
// resonant poles of the 2048^2 depth field at t rho = 5000 (iterations for
// n = 50 / 200 / 500 / 1000): 0.1: 7 / 33 / 190 / 382, 0.3: 8 / 48 / 134 /
// 82, 0.5: 8 / 68 / 168 / 72, 1.0: 11 / 115 / 277 / 107; undamped it
// diverges for n >= 500
constexpr double kPcDampHost = 0.3;
constexpr int kPcCheck = 1;           // iterations between host checks (most solves take 2-3)

static int pc_slots(size_t points, size_t nsolves, int requested) {
  const size_t per_slot = 8 * points * 16;
  const size_t budget = size_t(24) << 30;
  size_t B = requested > 0 ? size_t(requested) : size_t(32);
  B = std::min(B, std::max<size_t>(1, budget / per_slot));
  B = std::min(B, std::max<size_t>(1, nsolves));
  return int(std::max<size_t>(1, B));
}

static size_t pc_engine_bytes(int nx, int ny, int B, size_t fft_work) {
  const size_t n = size_t(nx) * ny;
  return 8 * al256(size_t(B) * n * 16) + al256(size_t(B) * pc_blocks() * 8 * sizeof(double)) +
         al256(size_t(B) * sizeof(PcSlot)) + al256(pc_blocks() * 8) + al256(fft_work) + 4096;
}

static rexii_status job_bytes(const std::vector<JobItem>& items, const rexii_opts& o, bool keep, size_t extra,
                              size_t* bytes) {
  std::vector<Problem> pbs(items.size());
  std::vector<Problem*> ptrs;
  size_t b = extra + al256(std::max<size_t>(1, items.size()) * sizeof(int)) + 4096;
  b += al256(std::max<size_t>(1, items.size()) * wnorm_blocks() * sizeof(double));
  for (size_t i = 0; i < items.size(); ++i) {
    if (items[i].skip) continue;
    rexii_status st = sizing_plan(items[i], o, pbs[i]);
    if (st != REXII_OK) return st;
    ptrs.push_back(&pbs[i]);
    b += problem_bytes(pbs[i]);
  }
  if (!ptrs.empty() && o.method == 2) {
    // the preconditioned solver: one problem at a time, the largest engine
    size_t eb = 0;
    for (Problem* p : ptrs) {
      const int B = pc_slots(p->n(), p->pl.solves.size(), o.pole_batch);
      size_t work = 0;
      const rexii_status fs = fft_plans_c2c(p->pl.nx, p->pl.ny, B, &work, nullptr, nullptr);
      if (fs != REXII_OK) return fs;
      eb = std::max(eb, pc_engine_bytes(p->pl.nx, p->pl.ny, B, work));
    }
    *bytes = b + eb;
    return REXII_OK;
  }
  if (!ptrs.empty()) {
    const EngineSize z = engine_size(ptrs, o.pole_batch, o.precision, o.tile_rows);
    if (keep) b += al256(size_t(z.S) * z.cap * 16);
    size_t eb = engine_bytes(z);
    // mixed precision: room for an FP64 re-run engine of at least one slot
    if (o.precision == REXII_PREC_MIXED) eb = std::max(eb, engine_bytes(engine_size(ptrs, 1, REXII_PREC_FP64, 0)));
    b += eb;
  }
  *bytes = b;
  return REXII_OK;
}

// Workspace of run_items for these problems: job_bytes at the options'
// slot count, or with pole_batch < 0 the largest job the autotuner may run
// (its biggest candidate slot count for every tile height it tries).
static int tuner_cap_slots(const std::vector<JobItem>& items, const rexii_opts& o);
static rexii_status items_bytes(const std::vector<JobItem>& items, const rexii_opts& o, size_t* bytes) {
  if (o.method == 2) {   // the preconditioned solver takes no autotuning
    rexii_opts o2 = o;
    o2.pole_batch = std::max(0, o.pole_batch);
    return job_bytes(items, o2, false, 0, bytes);
  }
  if (o.pole_batch >= 0) return job_bytes(items, o, false, 0, bytes);
  const bool bicg = o.method == 1;
  std::vector<int> ths = (bicg && o.tile_rows == 0) ? std::vector<int>{32, 16} : std::vector<int>{o.tile_rows};
  size_t best = 0;
  for (int th : ths) {
    rexii_opts ot = o;
    ot.tile_rows = bicg ? th : 0;
    ot.pole_batch = tuner_cap_slots(items, ot);
    size_t b = 0;
    const rexii_status st = job_bytes(items, ot, false, 0, &b);
    if (st != REXII_OK) return st;
    best = std::max(best, b);
  }
  *bytes = best;
  return REXII_OK;
}

struct Job {
  hipStream_t st;
  rexii_opts o;
  std::vector<JobItem> items;
  std::vector<Problem> pbs;
  std::vector<Problem*> ptrs;    // problems in the engine
  std::vector<int> engine_index; // item -> problem index in the engine (-1: skipped)
  Engine* en = nullptr;
  bool keep = false;
  bool force_unpaired = false;
  bool pair_all = false;         // pairing decided jointly (adjoint)
  ~Job() { delete en; }
};

// Mixed precision: the solves that ended as kRetry (their FP32 inner
// solves went non-finite, diverged, stalled or hit their cap) are solved
// again from scratch by an FP64 engine in the first engine's memory, and
// accumulate into the same fields; their statistics are merged (iterations
// of both attempts, the outcome of the second).
static void rerun_fp64(Job& jb, Arena& ar, size_t mark, double2* yout) {
  Engine& en = *jb.en;
  en.retried.assign(en.z.S, 0);
  std::vector<Problem> rp(jb.ptrs.size());
  std::vector<std::vector<int>> origin(jb.ptrs.size());  // first-engine queue position of each re-run solve
  int nre = 0;
  for (int j = 0; j < en.z.S; ++j) {
    if (en.stats[j].status != kRetry) continue;
    const int inst = en.solve_inst[j];
    if (origin[inst].empty()) {
      rp[inst] = *jb.ptrs[inst];
      rp[inst].pl.solves.clear();
      rp[inst].pl.precision = REXII_PREC_FP64;
      rp[inst].Hin = rp[inst].H;   // FP64 inner passes read the FP64 depth
    }
    SolveDesc d = jb.ptrs[inst]->pl.solves[en.solve_index[j]];
    d.yidx = j;
    rp[inst].pl.solves.push_back(d);
    origin[inst].push_back(j);
    en.retried[j] = 1;
    ++nre;
  }
  if (nre == 0) return;
  std::vector<Problem*> rptr;
  std::vector<int> rinst;
  for (size_t i = 0; i < rp.size(); ++i)
    if (!origin[i].empty()) {
      rptr.push_back(&rp[i]);
      rinst.push_back(int(i));
    }
  ar.reset(mark);
  EngineSize z = engine_size(rptr, 0, REXII_PREC_FP64, 0);
  z.B = std::min(z.B, std::max(1, en.z.B));
  while (z.B > 1 && engine_bytes(z) > ar.remaining()) z.B = std::max(1, (z.B * 3) / 4);
  Engine er(jb.st);
  er.setup(ar, rptr, z, REXII_PREC_FP64, jb.o.max_iter, 0.0, en.profile, yout, en.z.cap);
  er.run<double>();
  for (int k = 0; k < er.z.S; ++k) {
    const int j = origin[rinst[er.solve_inst[k]]][er.solve_index[k]];
    SolveStat& a = en.stats[j];
    const SolveStat& b = er.stats[k];
    a.it_total += b.it_total;
    a.rounds += b.rounds;
    a.status = b.status;
    a.rn2 = b.rn2;
    a.bn2 = b.bn2;
    a.stagnated = b.stagnated;
  }
  en.pass_bytes += er.pass_bytes;
  en.u1_bytes += er.u1_bytes;
  en.kernel_ms += er.kernel_ms;
  en.launches += er.launches;
  for (int k = 0; k < Engine::kBcgEvents - 1; ++k) en.step_ms[k] += er.step_ms[k];
  en.solve_seconds += er.solve_seconds;
}

// ---------------------------------------------------------------------------
// FFT-preconditioned BiCGStab (opts.method = 2; precond.hip): the flux-form
// height equation of every pole, right-preconditioned by the exact inverse
// of the mean-depth operator with a damped shift, all FP64.  B slots run
// together; the host checks the slots after every iteration, takes the true
// residual of those whose recurrence met the stop test (or hit the cap, or
// broke down), finishes them (accumulating Re(c_j x) in queue order of
// finishing) or restarts them from that residual, and refills free slots
// from the queue (most expensive first).
// ---------------------------------------------------------------------------
static void run_pc(Job& jb, Arena& ar) {
  hipStream_t st = jb.st;
  Engine* en = new Engine(st);
  jb.en = en;
  en->z.method = 2;
  en->z.th = 0;
  en->precision = REXII_PREC_FP64;
  size_t total = 0;
  for (Problem* p : jb.ptrs) total += p->pl.solves.size();
  en->z.S = int(total);
  en->stats.assign(total, SolveStat{});
  en->solve_inst.assign(total, 0);
  en->solve_index.assign(total, 0);
  en->retried.assign(total, 0);
  en->plans.clear();
  for (Problem* p : jb.ptrs) en->plans.push_back(&p->pl);
  en->inst_points.clear();
  for (Problem* p : jb.ptrs) en->inst_points.push_back(p->n());
  const auto w0 = std::chrono::steady_clock::now();
  double every = 0.0;   // $REXII_PROGRESS: seconds between progress lines
  if (const char* pv = std::getenv("REXII_PROGRESS")) every = std::atof(pv);
  auto last = w0;
  int finished = 0;
  int qbase = 0;   // queue positions of the problems' solves follow each other
  for (size_t ip = 0; ip < jb.ptrs.size(); ++ip) {
    Problem& pb = *jb.ptrs[ip];
    const Plan& pl = pb.pl;
    const int nx = pl.nx, ny = pl.ny;
    const size_t n = pb.n();
    const int S = int(pl.solves.size());
    const int B = pc_slots(n, size_t(S), jb.o.pole_batch);
    en->z.B = std::max(en->z.B, B);
    size_t work = 0;
    void *fwd = nullptr, *inv = nullptr;
    const rexii_status fs = fft_plans_c2c(nx, ny, B, &work, &fwd, &inv);
    if (fs != REXII_OK) throw HipError{fs, g_err};
    const size_t mark = ar.mark();
    PcVec w;
    w.B = B;
    double2** vecs[8] = {&w.x, &w.r, &w.rh, &w.p, &w.v, &w.ph, &w.sh, &w.t};
    for (double2** v : vecs) *v = ar.take<double2>(size_t(B) * n);
    w.part = ar.take<double>(size_t(B) * pc_blocks() * 8);
    w.slots = ar.take<PcSlot>(B);
    double* hpart = ar.take<double>(pc_blocks());
    void* wk = work ? static_cast<void*>(ar.take<char>(work)) : nullptr;
    // axis symbols and the mean depth
    const std::shared_ptr<const SymTable> symt = symbol_table(nx, ny, 0);
    launch_pc_sum(pb.H, n, hpart, st);
    std::vector<double> hp(pc_blocks());
    read_to_host(hp.data(), hpart, hp.size() * sizeof(double), st);
    double hsum = 0.0;
    for (double v : hp) hsum += v;
    PcProb pr;
    pr.nx = nx;
    pr.ny = ny;
    pr.cx = 0.25 * double(nx) * nx;
    pr.cy = 0.25 * double(ny) * ny;
    pr.cxy = 0.25 * double(nx) * ny;
    pr.hbar = hsum / double(n);
    pr.H = pb.H;
    pr.eta0 = pb.f;
    pr.D0 = pl.has_vel ? pb.DZ : nullptr;
    pr.Z0 = pl.has_vel ? pb.DZ + n : nullptr;
    pr.sx = symt->dev.get(symt->s);
    // queue: most expensive first
    std::vector<int> order(S);
    for (int k = 0; k < S; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pl.solves[a].cost > pl.solves[b].cost; });
    std::vector<PcSlot> hs(B);
    std::vector<int> slot_solve(B, -1), slot_q(B, -1);
    std::vector<double> prev_true(B, 0.0);
    std::memset(static_cast<void*>(hs.data()), 0, sizeof(PcSlot) * B);
    const int cap = (jb.o.max_iter > 0) ? jb.o.max_iter : 5000;
    int next = 0;
    auto assign = [&](int b) {
      const int k = order[next];
      const SolveDesc& d = pl.solves[k];
      PcSlot& q = hs[b];
      std::memset(static_cast<void*>(&q), 0, sizeof(q));
      q.zeta = to_d2(d.zeta);
      q.gamma = to_d2(d.gamma);
      q.sc = to_d2(d.sc);
      q.a1 = to_d2(d.a1);
      q.a2 = to_d2(d.a2);
      const double damp = kPcDampHost * std::fabs(d.zeta.real()) * (d.zeta.imag() >= 0.0 ? 1.0 : -1.0);
      q.sigma = make_double2(d.zeta.real(), d.zeta.imag() + damp);
      q.rho = q.alpha = q.omega = make_double2(1.0, 0.0);
      q.beta = make_double2(0.0, 0.0);
      q.tol2 = d.tol * d.tol;
      q.ref2 = d.ref2 > 0.0 ? d.ref2 : 0.0;
      q.state = kPcStart;
      q.max_it = cap;
      slot_solve[b] = k;
      slot_q[b] = qbase + next;
      prev_true[b] = 0.0;
      en->solve_inst[qbase + next] = int(ip);
      en->solve_index[qbase + next] = k;
      ++next;
    };
    int live = 0;
    for (int b = 0; b < B && next < S; ++b) {
      assign(b);
      ++live;
    }
    HIPCHK(hipMemcpyAsync(w.slots, hs.data(), sizeof(PcSlot) * B, hipMemcpyHostToDevice, st));
    int64_t iters = 0;
    while (live > 0) {
      for (int c = 0; c < kPcCheck; ++c) {
        launch_pc_dir(w, pr, st);
        launch_pc_scalars(w, 0, st);
        rexii_status e1 = fft_execute(fwd, w.ph, w.ph, wk, work, st);
        if (e1 != REXII_OK) throw HipError{e1, g_err};
        launch_pc_scale(w.ph, w, pr, st);
        e1 = fft_execute(inv, w.ph, w.ph, wk, work, st);
        if (e1 != REXII_OK) throw HipError{e1, g_err};
        launch_pc_matvec(w.ph, w.v, 0, w, pr, st);
        launch_pc_scalars(w, 1, st);
        launch_pc_s(w, pr, st);
        e1 = fft_execute(fwd, w.sh, w.sh, wk, work, st);
        if (e1 != REXII_OK) throw HipError{e1, g_err};
        launch_pc_scale(w.sh, w, pr, st);
        e1 = fft_execute(inv, w.sh, w.sh, wk, work, st);
        if (e1 != REXII_OK) throw HipError{e1, g_err};
        launch_pc_matvec(w.sh, w.t, 1, w, pr, st);
        launch_pc_scalars(w, 2, st);
        launch_pc_xr(w, pr, st);
        launch_pc_scalars(w, 3, st);
        ++iters;
      }
      HIPCHK(hipGetLastError());
      read_to_host(hs.data(), w.slots, sizeof(PcSlot) * B, st);
      if (every > 0.0) {
        const auto now = std::chrono::steady_clock::now();
        if (std::chrono::duration<double>(now - last).count() >= every) {
          last = now;
          std::fprintf(stderr, "rexii: %d of %d solves finished, %d slots working, %.0f s\n", finished, en->z.S,
                       live, std::chrono::duration<double>(now - w0).count());
          std::fflush(stderr);
        }
      }
      bool any_check = false;
      for (int b = 0; b < B; ++b)
        if (hs[b].state == kPcConv || hs[b].state == kPcCap || hs[b].state == kPcBreak) any_check = true;
      if (!any_check) continue;
      launch_pc_resid(w, pr, st);
      HIPCHK(hipGetLastError());
      read_to_host(hs.data(), w.slots, sizeof(PcSlot) * B, st);
      bool changed = false;
      for (int b = 0; b < B; ++b) {
        PcSlot& q = hs[b];
        if (q.state != kPcConv && q.state != kPcCap && q.state != kPcBreak) continue;
        const SolveDesc& d = pl.solves[slot_solve[b]];
        SolveStat& ss = en->stats[slot_q[b]];
        ss.it_total = q.it;
        ss.rounds += 1;
        ss.rn2 = q.rn2;
        ss.bn2 = q.bn2;
        const bool ok = q.rn2 <= q.stop2;
        const bool stalled = prev_true[b] > 0.0 && q.rn2 > 0.25 * prev_true[b];
        int fin = -1;
        if (ok) {
          fin = kDone;
        } else if (q.state == kPcCap) {
          fin = kFailMaxIter;
        } else if (stalled) {
          fin = kDone;
          ss.stagnated = 1;
        } else if (q.state == kPcBreak && ss.rounds > 8) {
          fin = kFailBreakdown;
        }
        if (fin < 0) {
          // restart from the true residual (r, rh, p set by the residual kernel)
          prev_true[b] = q.rn2;
          q.state = kPcIter;
          changed = true;
          continue;
        }
        ss.status = fin;
        launch_pc_accum(w, b, to_d2(d.c0), to_d2(d.c1), to_d2(d.c2), pb.A, pr, st);
        q.state = kPcIdle;
        slot_solve[b] = -1;
        --live;
        ++finished;
        changed = true;
        if (next < S) {
          assign(b);
          ++live;
        }
      }
      if (changed) HIPCHK(hipMemcpyAsync(w.slots, hs.data(), sizeof(PcSlot) * B, hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    en->launches += iters;
    qbase += S;
    ar.reset(mark);
  }
  en->solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
}

// Prepares every problem (input checks, div/curl, plans) and runs the engine
// (only max_chunks chunks if > 0; returns their time in ms).
static double run_job(Job& jb, Arena& ar, int max_chunks = 0) {
  const size_t ni = jb.items.size();
  jb.pbs.resize(ni);
  jb.engine_index.assign(ni, -1);
  // pinned host copy of the input flags: the set's staging buffer (past
  // the part that read_to_host uses, which is at most one W-norm vector)
  // or an allocation of this call
  const size_t nflag = std::max<size_t>(1, ni);
  const size_t flag_off = al256(nflag * wnorm_blocks() * sizeof(double));
  int* flags = nullptr;
  int* own_flags = nullptr;
  if (void* pin = ctx_pinned(flag_off + nflag * sizeof(int))) {
    flags = reinterpret_cast<int*>(static_cast<char*>(pin) + flag_off);
  } else {
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&own_flags), nflag * sizeof(int), hipHostMallocDefault));
    flags = own_flags;
  }
  struct FreeHost {
    int* p;
    ~FreeHost() {
      if (p) (void)hipHostFree(p);
    }
  } fh{own_flags};
  int* dflags = ar.take<int>(std::max<size_t>(1, ni));
  launch_fill_zero(reinterpret_cast<double*>(dflags), (std::max<size_t>(1, ni) + 1) / 2, jb.st);
  // ||f||_W^2 of every problem (block partials, summed on the host)
  const int nwb = wnorm_blocks();
  double* dwn = ar.take<double>(std::max<size_t>(1, ni) * nwb);
  bool any_depth_field = false;
  for (const JobItem& it : jb.items) any_depth_field = any_depth_field || (!it.skip && it.op->H_field);
  // one engine runs one method: a depth field anywhere puts every problem
  // of the call on the flux-form path
  if (any_depth_field && jb.o.method == 0) jb.o.method = 1;
  for (size_t i = 0; i < ni; ++i) {
    JobItem& it = jb.items[i];
    if (it.skip) continue;
    Problem& pb = jb.pbs[i];
    const size_t n = size_t(it.op->nx) * it.op->ny;
    pb.f = it.f;
    pb.DZ = ar.take<double>(2 * n);
    pb.A = ar.take<double>(3 * n);
    double* hp = ar.take<double>(8 + prep_vh_blocks());
    double* hconst = ar.take<double>(n);
    float* hf32 = ar.take<float>(n);
    launch_fill_zero(pb.A, 3 * n, jb.st);
    if (it.op->H_field) {
      pb.H = it.op->H_field;
      launch_prep_vh(it.f, it.op->H_field, it.op->nx, it.op->ny, pb.DZ, pb.DZ + n, dflags + i, hp, jb.st);
    } else {
      if (jb.o.method >= 1) {
        launch_fill_value(hconst, n, it.op->H0, jb.st);
        pb.H = hconst;
      }
      launch_prep(it.f, it.op->nx, it.op->ny, pb.DZ, pb.DZ + n, dflags + i, jb.st);
      if (jb.o.method >= 1) {
        // flux form: D_H = H0 div, Z_H = H0 curl
        launch_scale1(pb.DZ, 2 * n, it.op->H0, jb.st);
      }
    }
    pb.Hin = pb.H;
    if (pb.H && jb.o.precision == REXII_PREC_MIXED) {
      // the inner iterations read the depth in FP32
      launch_to_f32(pb.H, hf32, n, jb.st);
      pb.Hin = hf32;
    }
    launch_wnorm2(it.f, it.op->H_field, it.op->H0, it.op->g, n, dwn + i * nwb, jb.st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(flags, dflags, ni * sizeof(int), hipMemcpyDeviceToHost, jb.st));
  std::vector<double> wn(ni * nwb, 0.0);
  read_to_host(wn.data(), dwn, ni * nwb * sizeof(double), jb.st);  // drains the stream
  for (size_t i = 0; i < ni; ++i) {
    double a = 0.0;
    for (int b = 0; b < nwb; ++b) a += wn[i * nwb + b];
    jb.pbs[i].fw2 = a;
  }
  bool all_div_free = true;
  for (size_t i = 0; i < ni; ++i) {
    if (jb.items[i].skip) continue;
    if (flags[i] & 1) throw HipError{REXII_ERR_NONFINITE, "non-finite value in an input state"};
    if (flags[i] & 8) throw HipError{REXII_ERR_NONFINITE, "depth field has a non-finite or non-positive value"};
    if (flags[i] & 4) all_div_free = false;
  }
  for (size_t i = 0; i < ni; ++i) {
    JobItem& it = jb.items[i];
    if (it.skip) continue;
    const bool has_vel = (flags[i] & 2) != 0;
    bool div_free = (flags[i] & 4) == 0;
    if (jb.pair_all) div_free = all_div_free;
    if (jb.force_unpaired || it.shifts) div_free = false;
    Plan& pl = jb.pbs[i].pl;
    rexii_status st = build_plan(it.op, it.t, jb.o, has_vel, div_free, pl, it.adjoint, it.hmax);
    if (st != REXII_OK) throw HipError{st, g_err};
    if (it.shifts) shift_solves(it.op, it.t, *it.shifts, jb.o.tol, pl);
    // pole sums: each solve stops when its share of the error bound,
    // wsum sqrt(g) |r3| / |f|_W with r3 = rscale (b - K x), is within
    // wsum eps_s, i.e. |b - K x|^2 <= eps_s^2 |f|_W^2 / (g rscale^2)
    if (!pl.shifts)
      for (SolveDesc& d : pl.solves) d.ref2 = jb.pbs[i].fw2 / (it.op->g * d.rscale * d.rscale);
    jb.engine_index[i] = int(jb.ptrs.size());
    jb.ptrs.push_back(&jb.pbs[i]);
  }
  if (jb.ptrs.empty()) return 0.0;
  if (jb.o.method == 2) {
    run_pc(jb, ar);
    return 0.0;
  }
  const EngineSize z = engine_size(jb.ptrs, jb.o.pole_batch, jb.o.precision, jb.o.tile_rows);
  double2* yout = jb.keep ? ar.take<double2>(size_t(z.S) * z.cap) : nullptr;
  const size_t mark = ar.mark();   // the engine's memory starts here
  jb.en = new Engine(jb.st);
  jb.en->setup(ar, jb.ptrs, z, jb.o.precision, jb.o.max_iter,
               (jb.o.precision == REXII_PREC_MIXED) ? jb.o.inner_tol : 0.0,
               jb.o.profile != 0 && max_chunks == 0, yout, z.cap);
  if (jb.o.precision != REXII_PREC_MIXED) return jb.en->run<double>(max_chunks);
  const double ms = jb.en->run<float>(max_chunks);
  if (max_chunks == 0) rerun_fp64(jb, ar, mark, yout);
  return ms;
}

// ---------------------------------------------------------------------------
// autotuner: slots per engine (opts.pole_batch < 0)
// ---------------------------------------------------------------------------
// For each candidate slot count the real problems run for a few HIP-graph
// chunks (all slots busy: the queue is longer than the slot count); the
// rate of (slot x point x pass) per second decides.  Results are cached in a
// text file keyed by grid, precision, method and CU count:
// $REXII_TUNE_CACHE, else $HOME/.cache/rexii_tune.txt, else /tmp/rexii_tune.txt.
static std::string tune_cache_path() {
  if (const char* p = std::getenv("REXII_TUNE_CACHE")) return p;
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/rexii_tune.txt";
  return "/tmp/rexii_tune.txt";
}

static std::string tune_key(const std::vector<JobItem>& items, const rexii_opts& o, int cus) {
  size_t maxp = 0;
  int nx = 0, ny = 0;
  bool depth = false;
  for (const JobItem& it : items) {
    if (it.skip) continue;
    const size_t n = size_t(it.op->nx) * it.op->ny;
    if (n > maxp) {
      maxp = n;
      nx = it.op->nx;
      ny = it.op->ny;
    }
    depth = depth || it.op->H_field != nullptr;
  }
  const int method = (depth || o.method == 1) ? 1 : 0;
  char buf[160];
  std::snprintf(buf, sizeof(buf), "nx=%d ny=%d prec=%d method=%d rows=%d cus=%d", nx, ny, o.precision, method,
                o.tile_rows, cus);
  return buf;
}

// Cached choice for key: slot count and tile rows (0 if none).
static int tune_lookup(const std::string& key, int* th) {
  FILE* fp = std::fopen(tune_cache_path().c_str(), "r");
  if (!fp) return 0;
  char line[256];
  int best = 0;
  while (std::fgets(line, sizeof(line), fp)) {
    std::string l(line);
    const size_t bar = l.find(" | B=");
    if (bar != std::string::npos && l.substr(0, bar) == key) {
      best = std::atoi(l.c_str() + bar + 5);
      const size_t tp = l.find(" T=", bar);
      *th = (tp != std::string::npos) ? std::atoi(l.c_str() + tp + 3) : 0;
    }
  }
  std::fclose(fp);
  return best;
}
static void tune_store(const std::string& key, int B, int th, double rate) {
  const std::string path = tune_cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    const std::string dir = path.substr(0, slash);
    (void)std::system(("mkdir -p '" + dir + "' 2>/dev/null").c_str());
  }
  FILE* fp = std::fopen(path.c_str(), "a");
  if (!fp) return;
  std::fprintf(fp, "%s | B=%d T=%d rate=%.4e\n", key.c_str(), B, th, rate);
  std::fclose(fp);
}

// Slot count and (BiCGStab path, when o.tile_rows == 0) tile rows: every
// candidate runs four graph chunks of the real problems; the best rate of
// grid points advanced per second wins and is cached.  Returns the slot
// count (0 on failure) and the tile rows in *th.
// Largest slot count the autotuner tries: twice the default count (at
// least 128), capped by kMaxSlots.
static int tuner_cap_slots(const std::vector<JobItem>& items, const rexii_opts& o) {
  int hb = 0;
  std::vector<Problem> pbs(items.size());
  std::vector<Problem*> ptrs;
  for (size_t i = 0; i < items.size(); ++i) {
    if (items[i].skip || sizing_plan(items[i], o, pbs[i]) != REXII_OK) continue;
    ptrs.push_back(&pbs[i]);
  }
  if (!ptrs.empty()) hb = engine_size(ptrs, 0, o.precision, o.tile_rows).B;
  return std::min(kMaxSlots, std::max(128, 2 * hb));
}

static int autotune_slots(const std::vector<JobItem>& items, const rexii_opts& o, hipStream_t st, int* th,
                          void* ws = nullptr, size_t ws_bytes = 0) {
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const std::string key = tune_key(items, o, cus);
  *th = 0;
  const int cached = tune_lookup(key, th);
  if (cached > 0) return cached;
  size_t nsolves = 0, maxp = 0;
  bool depth = false;
  {
    std::vector<JobItem> its = items;
    for (JobItem& it : its) {
      if (it.skip) continue;
      Problem pb;
      if (sizing_plan(it, o, pb) != REXII_OK) return 0;
      nsolves += pb.pl.solves.size();
      maxp = std::max(maxp, pb.n());
      depth = depth || it.op->H_field != nullptr;
    }
  }
  const bool bicg = depth || o.method == 1;
  std::vector<int> ths;
  if (bicg && o.tile_rows == 0)
    ths = {32, 16};
  else
    ths = {bicg ? o.tile_rows : 0};  // 0: the engine's default
  const int cands[] = {8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  int best = 0, best_th = 0;
  double best_rate = 0.0;
  for (int t : ths) {
    rexii_opts ot = o;
    ot.tile_rows = bicg ? t : 0;
    const int cap_b = tuner_cap_slots(items, ot);
    for (int B : cands) {
      if (B > cap_b || B > kMaxSlots) break;
      if (size_t(B) * 2 > nsolves && B != cands[0]) break;  // keep the queue longer than the slots
      Job jb;
      jb.st = st;
      jb.o = ot;
      jb.o.pole_batch = B;
      jb.o.profile = 0;
      jb.items = items;
      for (JobItem& it : jb.items) {
        it.u = nullptr;
        it.rep = nullptr;
      }
      size_t need = 0;
      if (job_bytes(jb.items, jb.o, false, 0, &need) != REXII_OK) break;
      // the caller's workspace when there is one (a candidate that does not
      // fit ends the search), else memory of this candidate's own
      Arena ar(ws, ws_bytes);
      if (ws) {
        if (need > ws_bytes) break;
      } else {
        try {
          ar.reserve_own(need + 4096);
        } catch (const HipError&) {
          break;  // out of memory: larger counts will not fit either
        }
      }
      const int chunks = 4;
      const double ms = run_job(jb, ar, chunks);
      if (!(ms > 0.0)) continue;
      const int chunk = jb.en ? jb.en->chunk : 16;
      const double rate = double(B) * double(maxp) * chunk * (chunks - 1) / (ms * 1e-3);
      if (rate > best_rate) {
        best_rate = rate;
        best = B;
        best_th = jb.en ? jb.en->z.th : t;
      }
    }
  }
  if (best > 0) tune_store(key, best, best_th, best_rate);
  *th = best_th;
  return best;
}

// Reports and status of every item after the run.
static rexii_status finish_job(Job& jb, double secs) {
  int bad_breakdown = 0, bad_conv = 0;
  double worst = 0.0;   // largest error bound over the items, relative to tol
  for (size_t i = 0; i < jb.items.size(); ++i) {
    JobItem& it = jb.items[i];
    if (it.skip) {
      if (it.rep) {
        std::memset(it.rep, 0, sizeof(*it.rep));
        it.rep->t = 0.0;
      }
      continue;
    }
    const int ei = jb.engine_index[i];
    fill_report(it.rep, jb.pbs[i].pl, jb.en, ei, secs);
    const RunSummary sm = summarize(*jb.en, ei);
    bad_breakdown += sm.breakdowns;
    bad_conv += sm.not_conv;
    worst = std::max(worst, sm.err_bound / jb.o.tol);
  }
  if (bad_breakdown > 0) return set_error(REXII_ERR_BREAKDOWN, "Krylov breakdown in a shifted solve");
  if (bad_conv > 0) return set_error(REXII_ERR_NOT_CONVERGED, "a shifted solve reached its iteration cap");
  // the contract: the achieved error bound (Theorem 1 with the solves'
  // residuals) is within tol; 1e-9 relative slack for the rounding of the sum
  if (worst > 1.0 + 1e-9) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "error bound %.3e x tol: a solve stopped above its tolerance (FP64 residual floor)",
                  worst);
    return set_error(REXII_ERR_NOT_CONVERGED, msg);
  }
  return clear_error();
}

static rexii_status check_op_and_t(const rexii_swe_op* op, double t, bool allow_zero, bool allow_depth_field = true) {
  rexii_status v = validate_op(op);
  if (v != REXII_OK) return v;
  if (!std::isfinite(t) || t < 0.0 || (!allow_zero && t == 0.0))
    return set_error(REXII_ERR_INVALID_ARG, allow_zero ? "t must be finite and >= 0" : "t must be > 0");
  if (op->H_field && !allow_depth_field)
    return set_error(REXII_ERR_INVALID_ARG, "variable depth is not supported by this entry point");
  return REXII_OK;
}

static bool overlaps(const double* a, size_t na, const double* b, size_t nb) { return a < b + nb && b < a + na; }

// Runs `body(stream)` on a private stream ordered after the caller's stream
// (graph capture needs a capturable stream; the caller's may be the null
// stream).  The call returns only when the work is complete, so later work
// on the caller's stream sees the results.
template <typename F>
static rexii_status on_private_stream(hipStream_t caller, F&& body) {
  DevCtx* c = device_ctx();
  std::unique_lock<std::mutex> held;
  if (c) held = std::unique_lock<std::mutex>(c->mu, std::try_to_lock);
  const bool shared = c && held.owns_lock();
  hipStream_t own = nullptr;
  hipEvent_t ev = nullptr;
  if (shared) {
    if (!c->st && hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) {
      c->st = nullptr;
      return set_error(REXII_ERR_HIP, "hipStreamCreateWithFlags failed");
    }
    if (!c->ev && hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess) {
      c->ev = nullptr;
      return set_error(REXII_ERR_HIP, "hipEventCreateWithFlags failed");
    }
    own = c->st;
    ev = c->ev;
  } else {
    if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess)
      return set_error(REXII_ERR_HIP, "hipStreamCreateWithFlags failed");
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
  }
  struct Hold {
    DevCtx* prev;
    Hold(DevCtx* c) : prev(tl_ctx) { tl_ctx = c; }
    ~Hold() { tl_ctx = prev; }
  } hold(shared ? c : nullptr);
  rexii_status st;
  if (!ev || hipEventRecord(ev, caller) != hipSuccess || hipStreamWaitEvent(own, ev, 0) != hipSuccess) {
    st = set_error(REXII_ERR_HIP, "could not order the private stream after the caller's stream");
  } else {
    try {
      st = body(own);
    } catch (const HipError& he) {
      st = set_error(he.st, he.msg);
    } catch (const std::bad_alloc&) {
      st = set_error(REXII_ERR_OOM, "host allocation failed");
    }
  }
  const std::string msg = g_err;
  if (hipStreamSynchronize(own) != hipSuccess && st == REXII_OK) st = set_error(REXII_ERR_HIP, "stream sync failed");
  if (!shared) {
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(own);
  }
  g_err = msg;
  return st;
}

// Common path of apply / batched / shifted_solve.
static rexii_status run_items(std::vector<JobItem> items, const rexii_opts* opts_in, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
  const auto t0 = std::chrono::steady_clock::now();
  return on_private_stream(stream, [&](hipStream_t st) -> rexii_status {
    Job jb;
    jb.st = st;
    jb.o = resolve_opts(opts_in);
    jb.items = items;
    for (JobItem& it : jb.items) {
      if (it.t == 0.0 && !it.shifts) {
        it.skip = true;
        launch_copy(it.f, it.u, 3 * size_t(it.op->nx) * it.op->ny, st);
      }
    }
    jb.keep = false;
    for (const JobItem& it : jb.items) jb.keep = jb.keep || (it.shifts != nullptr);
    bool any_depth_field = false;
    for (JobItem& it : jb.items) {
      if (it.skip || !it.op->H_field) continue;
      it.hmax = device_hmax(it.op->H_field, size_t(it.op->nx) * it.op->ny, st);
      any_depth_field = true;
    }
    if (jb.o.method == 2) {
      // the preconditioned solver: FP64, its own slot count, no kept solutions
      if (jb.keep) return set_error(REXII_ERR_INVALID_ARG, "method 2 does not return resolvents (explicit shifts)");
      jb.o.precision = REXII_PREC_FP64;
      if (jb.o.pole_batch < 0) jb.o.pole_batch = 0;
    }
    rexii_opts osz = jb.o;
    if (any_depth_field && osz.method == 0) osz.method = 1;
    if (jb.o.pole_batch < 0) {
      int th = 0;
      const int B = autotune_slots(jb.items, osz, st, &th, ws, ws_bytes);
      jb.o.pole_batch = (B > 0) ? B : 0;
      if (jb.o.tile_rows == 0 && (th == 16 || th == 32) && osz.method == 1) jb.o.tile_rows = th;
      osz.pole_batch = jb.o.pole_batch;
      osz.tile_rows = jb.o.tile_rows;
    }
    size_t need = 0;
    rexii_status s0 = job_bytes(jb.items, osz, jb.keep, 0, &need);
    if (s0 != REXII_OK) return s0;
    Arena ar(ws, ws_bytes);
    if (!ws) {
      ar.reserve_own(need + 4096);
    } else if (ws_bytes < need) {
      return set_error(REXII_ERR_WORKSPACE, "workspace smaller than rexii_workspace_size()");
    } else if (reinterpret_cast<uintptr_t>(ws) & 255) {
      return set_error(REXII_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    run_job(jb, ar);
    for (size_t i = 0; i < jb.items.size(); ++i) {
      const JobItem& it = jb.items[i];
      if (it.skip) continue;
      const Problem& pb = jb.pbs[i];
      const size_t n = size_t(it.op->nx) * it.op->ny;
      if (it.shifts) {
        for (int j = 0; j < jb.en->z.S; ++j) {
          if (jb.en->solve_inst[j] != jb.engine_index[i]) continue;
          const SolveDesc& d = pb.pl.solves[jb.en->solve_index[j]];
          launch_expand(jb.en->e.yout + size_t(j) * jb.en->z.cap, it.f, it.op->nx, it.op->ny, to_d2(d.inv_sigma),
                        to_d2(d.m1), to_d2(d.m2), it.t * it.op->g, pb.pl.has_vel ? 1 : 0,
                        it.xout + size_t(d.pole) * 3 * n, st);
        }
      } else if (it.u) {
        launch_reconstruct(it.f, pb.A, it.op->nx, it.op->ny, pb.pl.S1, pb.pl.S2, it.t * it.op->g,
                           pb.pl.has_vel ? 1 : 0, it.u, st);
      }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return finish_job(jb, secs);
  });
}

// Adjoint: dJdf = r(tA)^T gbar = W Re sum_k w'_k (tA - z_k)^{-1} W^{-1} gbar,
// dJdH = -t g Re sum_k w_k <conj(eta-part of (tA - z_{pi(k)})^{-1} W^{-1} gbar),
//                            div of the velocity of (tA - z_k)^{-1} f>,
// pi swapping the two poles of a term.
static rexii_status run_adjoint(const rexii_swe_op* op, const double* f, const double* gbar, double* dJdf,
                                double* dJdH, double t, const rexii_opts* opts_in, void* ws, size_t ws_bytes,
                                hipStream_t stream, rexii_report* rep) {
  const auto t0 = std::chrono::steady_clock::now();
  return on_private_stream(stream, [&](hipStream_t st) -> rexii_status {
    const size_t n = size_t(op->nx) * op->ny;
    Job jb;
    jb.st = st;
    jb.o = resolve_opts(opts_in);
    jb.o.method = 0;  // the dJ/dH dots use the constant-depth Helmholtz form
    jb.pair_all = true;
    const bool want_H = (dJdH != nullptr);
    jb.keep = want_H;
    JobItem G;
    G.op = op;
    G.t = t;
    G.adjoint = true;
    G.u = dJdf;
    G.rep = rep;
    jb.items.push_back(G);
    if (want_H) {
      JobItem F;
      F.op = op;
      F.f = f;
      F.t = t;
      jb.items.push_back(F);
    }
    size_t need = 0;
    size_t dots_bytes = 0;
    {
      // per-pole dot buffers of dJ/dH (one per pole in the unpaired case)
      Problem pz;
      rexii_status sp = build_plan(op, t, jb.o, true, false, pz.pl);
      if (sp != REXII_OK) return sp;
      const size_t nd = pz.pl.solves.size();
      dots_bytes = al256(nd * sizeof(AdjDot)) + al256(nd * size_t(adj_dot_blocks(n)) * 16) + al256(nd * 16);
    }
    rexii_status s0 = job_bytes(jb.items, jb.o, jb.keep, al256(3 * n * 8) + dots_bytes + 4096, &need);
    if (s0 != REXII_OK) return s0;
    Arena ar(ws, ws_bytes);
    if (!ws) {
      ar.reserve_own(need + 4096);
    } else if (ws_bytes < need) {
      return set_error(REXII_ERR_WORKSPACE, "workspace smaller than rexii_workspace_size()");
    } else if (reinterpret_cast<uintptr_t>(ws) & 255) {
      return set_error(REXII_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    // b' = W^{-1} gbar, W = diag(g, H, H)
    double* bprime = ar.take<double>(3 * n);
    launch_scale3(gbar, bprime, n, 1.0 / op->g, 1.0 / op->H0, 1.0 / op->H0, st);
    jb.items[0].f = bprime;
    run_job(jb, ar);
    const Problem& pg = jb.pbs[0];
    if (dJdf) {
      launch_reconstruct(bprime, pg.A, op->nx, op->ny, pg.pl.S1, pg.pl.S2, t * op->g, pg.pl.has_vel ? 1 : 0, dJdf,
                         st);
      launch_scale3(dJdf, dJdf, n, op->g, op->H0, op->H0, st);
    }
    if (want_H) {
      const Problem& pf = jb.pbs[1];
      const Engine& en = *jb.en;
      // queue positions of every (instance, solve) pair
      std::vector<int> qpos_g(pg.pl.solves.size(), -1), qpos_f(pf.pl.solves.size(), -1);
      for (int j = 0; j < en.z.S; ++j) {
        if (en.solve_inst[j] == 0) qpos_g[en.solve_index[j]] = j;
        else qpos_f[en.solve_index[j]] = j;
      }
      // adjoint solve by pole index
      std::vector<int> g_by_pole(pg.pl.P, -1);
      for (size_t k = 0; k < pg.pl.solves.size(); ++k) g_by_pole[pg.pl.solves[k].pole] = int(k);
      std::vector<AdjDot> dots;
      std::vector<cd> coef;
      const bool paired = pf.pl.paired;
      for (size_t k = 0; k < pf.pl.solves.size(); ++k) {
        const SolveDesc& d = pf.pl.solves[k];
        const int pole = d.pole;
        const int partner = paired ? pole : (pole ^ 1);
        const int gk = g_by_pole[partner];
        if (gk < 0) throw HipError{REXII_ERR_INVALID_ARG, "adjoint: partner solve missing"};
        const SolveDesc& dg = pg.pl.solves[gk];
        AdjDot a;
        a.m1 = to_d2(d.m1);
        a.m2 = to_d2(d.m2);
        a.a1 = to_d2(d.a1);
        a.a2 = to_d2(d.a2);
        a.zeta = to_d2(d.zeta);
        a.isig = to_d2(d.inv_sigma);
        a.ysc = to_d2(paired ? dg.inv_sigma : std::conj(dg.inv_sigma));
        a.conj = paired ? 0 : 1;
        a.jf = qpos_f[k];
        a.ja = qpos_g[gk];
        dots.push_back(a);
        coef.push_back(paired ? (std::conj(pf.pl.w_fwd[pole + 1]) - pf.pl.w_fwd[pole]) : pf.pl.w_fwd[pole]);
      }
      const int nd = int(dots.size());
      AdjDot* ddots = ar.take<AdjDot>(nd);
      const int nblk = adj_dot_blocks(n);
      double2* part = ar.take<double2>(size_t(nd) * nblk);
      double2* out = ar.take<double2>(nd);
      HIPCHK(hipMemcpyAsync(ddots, dots.data(), nd * sizeof(AdjDot), hipMemcpyHostToDevice, st));
      launch_adj_dots(ddots, nd, en.e.yout, en.z.cap, f, pf.DZ, pf.pl.has_vel ? pf.DZ + n : nullptr, op->nx, op->ny,
                      t * op->g, pf.pl.has_vel ? 1 : 0, part, nblk, out, st);
      std::vector<double2> hout(nd);
      read_to_host(hout.data(), out, nd * sizeof(double2), st);
      double acc = 0.0;
      for (int k = 0; k < nd; ++k) acc += (coef[k] * cd(hout[k].x, hout[k].y)).real();
      *dJdH = -t * op->g * acc;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return finish_job(jb, secs);
  });
}

// ---------------------------------------------------------------------------
// Fourier-space path (constant depth): FFT, per-mode filter by the REXII sum
// in closed form, inverse FFT (kernels_fft.hip).
// ---------------------------------------------------------------------------
// Poles and weights of the reduced sum (Sec. 2.2), then, per pole, the
// real parts of the interpolation coefficients of r(x) = w / (x - z) on
// {0, +-i theta} as functions of theta^2 (see kernels_fft.hip); poles with
// the same z^2 up to the sign of Im z^2 share a denominator and one entry.
// The table depends on (M, h, scheme) only (t enters through theta), so it
// is formed once per such triple and kept (8 most recent triples; entries in
// use are never freed), with device copies the calls read in place.
struct TermTable {
  int P = 0, nterm = 0;
  double kappa = 0.0, c0 = 0.0;
  std::vector<double> tab;   // nterm x (a, b^2, A1, B1, A2, B2)
  DevCopies dev;
};

static std::shared_ptr<const TermTable> term_table(int M, double h, int scheme) {
  static std::mutex mu;
  using Entry = std::pair<std::tuple<int, double, int>, std::shared_ptr<const TermTable>>;
  static std::deque<Entry>& cache = *new std::deque<Entry>();
  const auto key = std::make_tuple(M, h, scheme);
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto it = cache.begin(); it != cache.end(); ++it)
      if (it->first == key) {
        auto hit = *it;
        cache.erase(it);
        cache.push_front(hit);
        return hit.second;
      }
  }
  std::vector<cplx> z, w;
  if (scheme == REXII_SCHEME_REXI)
    rexi_poles_weights(M, h, z, w);
  else
    poles_weights(M, h, z, w);
  auto tt = std::make_shared<TermTable>();
  tt->P = int(z.size());
  tt->kappa = kappa_sum(w, h);
  std::vector<double>& tab = tt->tab;
  tab.reserve(size_t(tt->P) * 6);
  for (int k = 0; k < tt->P; ++k) {
    const cd zk(z[k].re, z[k].im), wk(w[k].re, w[k].im);
    const cd q = -wk * std::conj(zk) / std::norm(zk);  // r(0) = -w / z of this pole
    tt->c0 += q.real();
    const double a = zk.real() * zk.real() - zk.imag() * zk.imag();
    const double b = 2.0 * zk.real() * zk.imag();
    const double e[6] = {a, b * b, -wk.real(), -wk.imag() * b, q.real(), q.imag() * b};
    const size_t m = tab.size();
    if (m >= 6 && tab[m - 6] == e[0] && tab[m - 5] == e[1]) {
      for (int j = 2; j < 6; ++j) tab[m - 6 + j] += e[j];
    } else {
      tab.insert(tab.end(), e, e + 6);
    }
  }
  tt->nterm = int(tab.size() / 6);
  std::shared_ptr<const TermTable> out = tt;
  std::lock_guard<std::mutex> lk(mu);
  for (auto it = cache.begin(); it != cache.end(); ++it)
    if (it->first == key) {   // made meanwhile by another thread
      cache.erase(it);
      break;
    }
  cache.push_front({key, out});
  while (cache.size() > 8) cache.pop_back();
  return out;
}

struct FourierPlan {
  int M = 0, N = 0, P = 0, m0 = 0, nterm = 0;
  double rho = 0.0, kappa = 0.0, c0 = 0.0;
  std::shared_ptr<const TermTable> tab;
};

// Spectral radius of the constant-depth symbol: centred differences, or
// Fourier differentiation (largest |k| is (n-1)/2: the Nyquist mode has a
// zero odd derivative).
static double rho_fourier(const rexii_swe_op* op, int deriv) {
  if (deriv == 0) return rho_const(op->nx, op->ny, op->g, op->H0, op->f_cor);
  const double sx = 2.0 * M_PI * double((op->nx - 1) / 2), sy = 2.0 * M_PI * double((op->ny - 1) / 2);
  return std::sqrt(op->f_cor * op->f_cor + op->g * op->H0 * (sx * sx + sy * sy));
}

static rexii_status fourier_plan(const rexii_swe_op* op, double t, const rexii_opts& o, int deriv,
                                 FourierPlan& fp) {
  if (!(o.h > 0.0 && o.h < M_PI)) return set_error(REXII_ERR_INVALID_ARG, "h must be in (0, pi)");
  if (o.scheme != REXII_SCHEME_REXII && o.scheme != REXII_SCHEME_REXI)
    return set_error(REXII_ERR_INVALID_ARG, "unknown scheme");
  if (!(o.tol > 0.0 && o.tol < 1.0)) return set_error(REXII_ERR_INVALID_ARG, "tol must be in (0, 1)");
  fp.rho = (o.rho > 0.0) ? o.rho : rho_fourier(op, deriv);
  fp.m0 = (o.m0 >= 0) ? o.m0 : m0_from_tol(o.tol);
  const double Md = std::ceil(t * fp.rho / o.h) + fp.m0;
  if (Md > 2.0e6) return set_error(REXII_ERR_INVALID_ARG, "t*rho/h too large for this library");
  fp.M = m_rule(t, fp.rho, o.h, fp.m0);
  fp.N = fp.M + terms_L();
  fp.tab = term_table(fp.M, o.h, o.scheme);
  fp.P = fp.tab->P;
  fp.kappa = fp.tab->kappa;
  fp.c0 = fp.tab->c0;
  fp.nterm = fp.tab->nterm;
  return REXII_OK;
}

// distinct canonical wavenumbers of the half spectrum's x (k = 0..nx/2) and
// y (k = 0..ny-1) indices
static void fourier_canon(int nx, int ny, int deriv, int* cnx, int* cny) {
  *cnx = canon_count(nx, nx / 2, deriv);
  *cny = canon_count(ny, ny - 1, deriv);
}

static size_t fourier_bytes(int nx, int ny, int deriv, int nterm, size_t fft_work) {
  const size_t nm = size_t(nx / 2 + 1) * ny;
  int cnx = 0, cny = 0;
  fourier_canon(nx, ny, deriv, &cnx, &cny);
  const int ne = mode_entries(cnx, cny, nx == ny ? 1 : 0);
  int nw = 1, ns = 1;
  mode_coef_shape(ne, nterm, &nw, &ns);
  const size_t part = (ns > 1) ? al256(size_t(ns) * ne * 16) : 0;
  // spectra, coefficients, split sums, finiteness words, and (copied in by
  // the no-allocation entry point) the term and symbol tables
  return al256(3 * nm * 16) + al256(size_t(ne) * 16) + part + al256(kCopyCheckMaxBlocks * sizeof(int)) +
         al256(size_t(nterm) * 48) + al256((size_t(nx / 2 + 1) + ny) * 8) + al256(fft_work);
}

// noalloc: device scratch from the library's static array, FFT plans only
// if they exist, no events and no pinned host memory (the entry point for
// callers that cannot allocate).
static rexii_status run_fourier(const rexii_swe_op* op, const double* f, double* u, double t, int deriv,
                                const rexii_opts* opts_in, void* ws, size_t ws_bytes, hipStream_t stream,
                                rexii_report* rep, bool noalloc = false) {
  const auto t0 = std::chrono::steady_clock::now();
  // Runs on the caller's stream (nothing here is captured into a graph) and
  // returns when the result is complete on it.
  hipStream_t st = stream;
  try {
    const int nx = op->nx, ny = op->ny;
    const size_t n3 = 3 * size_t(nx) * ny, nm = size_t(nx / 2 + 1) * ny;
    if (rep) std::memset(rep, 0, sizeof(*rep));
    if (t == 0.0) {
      launch_copy(f, u, n3, st);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(st));
      return clear_error();
    }
    rexii_opts o = resolve_opts(opts_in);
    if (noalloc) o.profile = 0;
    FourierPlan fp;
    rexii_status s = fourier_plan(op, t, o, deriv, fp);
    if (s != REXII_OK) return s;
    if (noalloc) {
      const size_t fixed = fourier_bytes(nx, ny, deriv, fp.nterm, 0);
      if (fixed > REXII_STATIC_SCRATCH_BYTES)
        return set_error(REXII_ERR_WORKSPACE, "problem needs more than the " +
                                                  std::to_string(REXII_STATIC_SCRATCH_BYTES >> 20) +
                                                  " MiB of static scratch (" + std::to_string(fixed) +
                                                  " bytes before the FFT work buffer)");
    }
    size_t work = 0;
    void *fwd = nullptr, *inv = nullptr;
    s = fft_plans(nx, ny, &work, &fwd, &inv, !noalloc);
    if (s != REXII_OK) return s;
    const size_t need = fourier_bytes(nx, ny, deriv, fp.nterm, work);
    int cnx = 0, cny = 0;
    fourier_canon(nx, ny, deriv, &cnx, &cny);
    if (noalloc) {
      if (need > REXII_STATIC_SCRATCH_BYTES)
        return set_error(REXII_ERR_WORKSPACE, "problem needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                                  std::to_string(REXII_STATIC_SCRATCH_BYTES));
      s = static_scratch(&ws);
      if (s != REXII_OK) return s;
      ws_bytes = REXII_STATIC_SCRATCH_BYTES;
    }
    Arena ar(ws, ws_bytes);
    if (!ws) {
      ar.reserve_own(need + 4096);
    } else if (ws_bytes < need) {
      return set_error(REXII_ERR_WORKSPACE, "workspace smaller than rexii_fourier_workspace_size()");
    } else if (reinterpret_cast<uintptr_t>(ws) & 255) {
      return set_error(REXII_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    const int sq = (nx == ny) ? 1 : 0;   // square grid: unordered frequency pairs
    const int ne = mode_entries(cnx, cny, sq);
    int nw = 1, ns = 1;
    mode_coef_shape(ne, fp.nterm, &nw, &ns);
    const bool sum_in_apply = mode_sum_in_apply(ne, ns);
    const std::vector<double>& htab = fp.tab->tab;
    const std::shared_ptr<const SymTable> sym = symbol_table(nx, ny, deriv);
    const int ncheck = copy_check_blocks(n3);
    double2* F = ar.take<double2>(3 * nm);
    double2* coef = ar.take<double2>(size_t(ne));
    double2* part = (ns > 1) ? ar.take<double2>(size_t(ns) * ne) : nullptr;
    int* flags = ar.take<int>(kCopyCheckMaxBlocks);
    void* wk = work ? static_cast<void*>(ar.take<char>(work)) : nullptr;
    // the term and symbol tables: the library's device copies, or (the
    // no-allocation entry point) copies from pageable host memory into its
    // scratch
    const double* tab = nullptr;
    const double* sxt = nullptr;
    if (noalloc) {
      double* dtab = ar.take<double>(htab.size());
      double* dsym = ar.take<double>(sym->s.size());
      HIPCHK(hipMemcpyAsync(dtab, htab.data(), htab.size() * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dsym, sym->s.data(), sym->s.size() * sizeof(double), hipMemcpyHostToDevice, st));
      tab = dtab;
      sxt = dsym;
    } else {
      tab = fp.tab->dev.get(htab);
      sxt = sym->dev.get(sym->s);
    }
    const double* syt = sxt + (nx / 2 + 1);
    const bool prof = (o.profile != 0);
    const double scale = 1.0 / (double(nx) * ny);
    auto pole_sums = [&](hipStream_t q) {
      launch_mode_coef(coef, part, cnx, cny, sq, sxt, syt, t, op->g, op->H0, op->f_cor, scale, tab, fp.nterm, nw, ns,
                       q);
    };
    auto apply_modes = [&](hipStream_t q) {
      launch_mode_apply(F, sum_in_apply ? part : coef, sum_in_apply ? ns : 1, ne, scale, cnx, sq, nx, ny, deriv, sxt,
                        syt, t, op->g, op->H0, op->f_cor, scale * fp.c0, q);
    };
    // the whole sequence on stream q (eager, or captured into a graph)
    auto enqueue = [&](hipStream_t q) -> rexii_status {
      launch_copy_check(f, u, n3, flags, q);  // the forward transform may overwrite its input
      rexii_status e1 = fft_execute(fwd, u, F, wk, work, q);
      if (e1 != REXII_OK) return e1;
      pole_sums(q);
      apply_modes(q);
      return fft_execute(inv, F, u, wk, work, q);
    };
    // profiling events: created once per host thread and kept
    static thread_local hipEvent_t ev[6] = {};
    if (prof) {
      if (!ev[0])
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
      // one stage after the other, timed
      HIPCHK(hipEventRecord(ev[0], st));
      launch_copy_check(f, u, n3, flags, st);  // the forward transform may overwrite its input
      HIPCHK(hipEventRecord(ev[1], st));
      s = fft_execute(fwd, u, F, wk, work, st);
      if (s != REXII_OK) return s;
      HIPCHK(hipEventRecord(ev[2], st));
      pole_sums(st);
      HIPCHK(hipEventRecord(ev[3], st));
      apply_modes(st);
      HIPCHK(hipEventRecord(ev[4], st));
      s = fft_execute(inv, F, u, wk, work, st);
      if (s != REXII_OK) return s;
      HIPCHK(hipEventRecord(ev[5], st));
    } else {
      s = enqueue(st);
      if (s != REXII_OK) return s;
    }
    HIPCHK(hipGetLastError());
    std::vector<int> hflags;
    const int* fl = nullptr;
    if (noalloc) {
      // no pinned memory: the stream is drained, then the words are copied
      hflags.resize(ncheck);
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipMemcpy(hflags.data(), flags, ncheck * sizeof(int), hipMemcpyDeviceToHost));
      fl = hflags.data();
    } else {
      // the words are read into pinned host memory (kept per host thread for
      // the life of the process), ordered on the stream
      static thread_local int* hflag = nullptr;
      if (!hflag)
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hflag), kCopyCheckMaxBlocks * sizeof(int), hipHostMallocDefault));
      HIPCHK(hipMemcpyAsync(hflag, flags, ncheck * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      fl = hflag;
    }
    int bad = 0;
    for (int b = 0; b < ncheck; ++b) bad |= fl[b];
    if (rep) {
      rep->P = fp.P;
      rep->M = fp.M;
      rep->N = fp.N;
      rep->m0 = fp.m0;
      rep->solves = fp.nterm;
      rep->h = o.h;
      rep->t = t;
      rep->rho = fp.rho;
      rep->kappa_sum = fp.kappa;
      rep->slots = nw;
      rep->tile_rows = ns;    // term splits of the sum kernel
      rep->total_iters = ne;  // distinct frequencies the pole sums were formed at
      // copy 16, forward FFT 8 + 16 nm/n, apply 2 x 48 nm/n, inverse 16 nm/n + 8 bytes per point and field
      rep->alg_bytes = double(n3) * 32.0 + 3.0 * double(nm) * (16.0 + 96.0 + 16.0);
      rep->kernel_bytes = 96.0 * double(nm);
      if (prof) {
        float ms[5] = {};
        for (int k = 0; k < 5; ++k) HIPCHK(hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]));
        for (int k = 0; k < 5; ++k) rep->step_ms[k] = ms[k];
        rep->kernel_launches = 1;
        rep->kernel_ms = ms[2];
      }
      rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (bad) return set_error(REXII_ERR_NONFINITE, "non-finite value in f");
    return clear_error();
  } catch (const HipError& he) {
    return set_error(he.st, he.msg);
  } catch (const std::bad_alloc&) {
    return set_error(REXII_ERR_OOM, "host allocation failed");
  }
}

// ---------------------------------------------------------------------------
// Shared-Krylov (multi-shift) path: one W-skew Lanczos process per state
// serves every pole (kernels_lz.hip); the small problems on T_m run here.
// ---------------------------------------------------------------------------
constexpr int kMultishiftMaxM = 50000;   // default cap on the Krylov dimension

struct SmallResult {
  int P = 0, M = 0, N = 0;
  double rho = 0.0, kappa = 0.0, tail = 0.0;
};

// y = beta0 Re sum_k w_k (t T - z_k I)^{-1} e_1 for the m x m real skew
// tridiagonal T with T[j+1][j] = b[j] = -T[j][j+1] (b[1..m-1]).  The poles
// come from the M rule for rho(T) (Gershgorin bound, capped by a bound on
// rho(A)).  A conjugate pair
// z_2 = -conj(z_1) needs one solve: with D = diag((-1)^(j-1)), D T D = -T, so
// (tT - z_2)^{-1} e_1 = -D conj((tT - z_1)^{-1} e_1).  Each solve is Gaussian
// elimination without pivoting, stable here because the Hermitian part of
// tT - z is -Re(z) I, definite.
static SmallResult small_problem(const double* b, int m, double t, double h, int m0, double beta0,
                                 double rho_cap, std::vector<double>& y) {
  SmallResult res;
  double rho = 0.0;
  for (int j = 1; j <= m; ++j) {
    const double lo = (j >= 2) ? b[j - 1] : 0.0, hi = (j <= m - 1) ? b[j] : 0.0;
    rho = std::max(rho, lo + hi);
  }
  // the eigenvalues of T = V^T W A V lie in the W-numerical range of A,
  // the segment i [-rho(A), rho(A)]: a bound on rho(A) caps Gershgorin's
  rho = std::min(rho, rho_cap);
  res.rho = rho;
  res.M = m_rule(t, std::max(rho, 1e-300), h, m0);
  res.N = res.M + terms_L();
  std::vector<cplx> z, w;
  poles_weights(res.M, h, z, w);
  res.P = int(z.size());
  res.kappa = kappa_sum(w, h);
  const int npair = res.P / 2;
  unsigned nth = std::thread::hardware_concurrency();
  nth = std::max(1u, std::min(16u, nth));
  nth = std::min<unsigned>(nth, std::max(1, npair));
  std::vector<std::vector<double>> part(nth, std::vector<double>(m, 0.0));
  auto work = [&](unsigned id) {
    std::vector<cd> cp(m), rp(m);
    std::vector<double>& yp = part[id];
    for (int q = int(id); q < npair; q += int(nth)) {
      const cd z1(z[2 * q].re, z[2 * q].im);
      const cd w1(w[2 * q].re, w[2 * q].im), w2(w[2 * q + 1].re, w[2 * q + 1].im);
      // forward elimination of (tT - z1) x = e_1: diagonal -z1, sub t b_j, super -t b_j
      cd den = -z1;
      cd inv = 1.0 / den;
      cp[0] = (m > 1) ? cd(-t * b[1]) * inv : cd(0.0);
      rp[0] = inv;
      for (int j = 1; j < m; ++j) {
        const double sub = t * b[j];
        den = -z1 - sub * cp[j - 1];
        inv = 1.0 / den;
        cp[j] = (j + 1 < m) ? cd(-t * b[j + 1]) * inv : cd(0.0);
        rp[j] = -sub * rp[j - 1] * inv;
      }
      cd x = rp[m - 1];
      for (int j = m - 1; j >= 0; --j) {
        if (j < m - 1) x = rp[j] - cp[j] * x;
        const double sgn = (j % 2 == 0) ? -1.0 : 1.0;  // -(-1)^j for 0-based j
        yp[j] += (w1 * x).real() + sgn * (w2 * std::conj(x)).real();
      }
    }
  };
  std::vector<std::thread> th;
  for (unsigned k = 1; k < nth; ++k) th.emplace_back(work, k);
  work(0);
  for (auto& x : th) x.join();
  y.assign(m, 0.0);
  for (unsigned k = 0; k < nth; ++k)
    for (int j = 0; j < m; ++j) y[j] += part[k][j];
  double tot = 0.0, tail = 0.0;
  for (int j = 0; j < m; ++j) {
    y[j] *= beta0;
    tot += y[j] * y[j];
    if (j >= m - 8) tail += y[j] * y[j];
  }
  res.tail = (tot > 0.0) ? std::sqrt(tail / tot) : 0.0;
  return res;
}

static rexii_status run_multishift(const rexii_swe_op* op, int nrhs, const double* f, double* u, double t,
                                   const rexii_opts* opts_in, void* ws, size_t ws_bytes, hipStream_t st,
                                   rexii_report* rep) {
  const auto t0 = std::chrono::steady_clock::now();
  try {
    const int nx = op->nx, ny = op->ny;
    const size_t n = size_t(nx) * ny, n3 = 3 * n;
    if (rep) std::memset(rep, 0, sizeof(*rep));
    if (t == 0.0) {
      launch_copy(f, u, n3 * nrhs, st);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(st));
      return clear_error();
    }
    const rexii_opts o = resolve_opts(opts_in);
    if (!(o.h > 0.0 && o.h < M_PI)) return set_error(REXII_ERR_INVALID_ARG, "h must be in (0, pi)");
    if (!(o.tol > 0.0 && o.tol < 1.0)) return set_error(REXII_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (o.scheme != REXII_SCHEME_REXII)
      return set_error(REXII_ERR_INVALID_ARG, "the REXI scheme is available on the Fourier path only");
    const int m0 = (o.m0 >= 0) ? o.m0 : m0_from_tol(o.tol);
    const int mmax = std::max(8, o.max_iter > 0 ? o.max_iter : kMultishiftMaxM);
    const int ldb = mmax + 2, ldy = mmax;
    const int nb = lz_blocks(nx, ny);
    const size_t need = 2 * al256(size_t(nrhs) * n3 * 8) + al256(size_t(nrhs) * nb * 8) +
                        al256(size_t(nrhs) * ldb * 8) + al256(size_t(nrhs) * ldy * 8) + al256(256);
    Arena ar(ws, ws_bytes);
    if (!ws) {
      ar.reserve_own(need + 4096);
    } else if (ws_bytes < need) {
      return set_error(REXII_ERR_WORKSPACE, "workspace smaller than rexii_multishift_workspace_size()");
    } else if (reinterpret_cast<uintptr_t>(ws) & 255) {
      return set_error(REXII_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    double* X = ar.take<double>(size_t(nrhs) * n3);
    double* Y = ar.take<double>(size_t(nrhs) * n3);
    double* part = ar.take<double>(size_t(nrhs) * nb);
    double* beta = ar.take<double>(size_t(nrhs) * ldb);
    double* ydev = ar.take<double>(size_t(nrhs) * ldy);
    double* flagd = ar.take<double>(32);
    int* flag = reinterpret_cast<int*>(flagd);
    const double* Hf = op->H_field;
    const double H0 = op->H0, g = op->g, fc = op->f_cor;
    hipEvent_t ev[2] = {};  // around the whole call (pass 2 is timed per state)
    const bool prof = (o.profile != 0);
    if (prof)
      for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    struct EvGuard {
      hipEvent_t* e;
      ~EvGuard() {
        for (int k = 0; k < 2; ++k)
          if (e[k]) (void)hipEventDestroy(e[k]);
      }
    } guard{ev};

    // pass 1: the Lanczos coefficients, in chunks; after each chunk the host
    // checks for breakdown and, once m reaches t rho(T), for convergence
    launch_fill_zero(flagd, 32, st);
    if (prof) HIPCHK(hipEventRecord(ev[0], st));
    launch_lz_start(f, X, Hf, H0, g, nx, ny, nrhs, part, flag, beta, ldb, st);
    std::vector<double> hb(size_t(nrhs) * ldb, 0.0);
    // device-to-host reads go to pinned host memory, ordered on the stream
    // and waited for through an event
    struct Pinned {
      void* p = nullptr;
      ~Pinned() {
        if (p) (void)hipHostFree(p);
      }
    } pin;
    HIPCHK(hipHostMalloc(&pin.p, size_t(nrhs) * ldb * 8 + 256, hipHostMallocDefault));
    double* hbp = static_cast<double*>(pin.p);
    int* hflag = reinterpret_cast<int*>(hbp + size_t(nrhs) * ldb);
    hipEvent_t rd = nullptr;
    HIPCHK(hipEventCreateWithFlags(&rd, hipEventDisableTiming));
    struct EvFree {
      hipEvent_t e;
      ~EvFree() { (void)hipEventDestroy(e); }
    } rdfree{rd};
    auto wait_reads = [&]() {
      HIPCHK(hipEventRecord(rd, st));
      HIPCHK(hipEventSynchronize(rd));
    };
    HIPCHK(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hbp, beta, size_t(nrhs) * ldb * 8, hipMemcpyDeviceToHost, st));
    wait_reads();
    const int bad = *hflag;
    std::copy(hbp, hbp + size_t(nrhs) * ldb, hb.begin());
    if (bad) return set_error(REXII_ERR_NONFINITE, "non-finite value in f");
    // scale of A for the breakdown test (beta_j -> 0: an invariant subspace)
    const double hscale = Hf ? device_hmax(Hf, n, st) : H0;
    const double rho_ref = std::sqrt(g * hscale) * std::sqrt(double(nx) * nx + double(ny) * ny) + std::fabs(fc);
    std::vector<int> mr(nrhs, 0);     // Krylov dimension per state (0: not fixed yet)
    for (int r = 0; r < nrhs; ++r)
      if (!(hb[size_t(r) * ldb] > 0.0)) mr[r] = -1;  // zero state: u = 0
    std::vector<std::vector<double>> ys(nrhs);
    std::vector<SmallResult> sr(nrhs);
    // pass 2 of a state is enqueued as soon as its small problem is solved,
    // so the GPU runs it while the host solves the next state's; the stream
    // orders it before any later pass-1 chunk (pass 1 never touches u, and a
    // state's own coefficients up to its m are never rewritten)
    std::vector<char> fin(nrhs, 0);
    std::vector<hipEvent_t> ev2(prof ? 2 * nrhs : 0, nullptr);
    struct Ev2Guard {
      std::vector<hipEvent_t>& e;
      ~Ev2Guard() {
        for (auto x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } guard2{ev2};
    for (auto& e : ev2) HIPCHK(hipEventCreate(&e));
    launch_fill_zero(u, size_t(nrhs) * n3, st);
    auto pass2 = [&](int r, int mm) {
      double* Xr = X + size_t(r) * n3;
      double* Yr = Y + size_t(r) * n3;
      double* br = beta + size_t(r) * ldb;
      double* yr = ydev + size_t(r) * ldy;
      HIPCHK(hipMemcpyAsync(yr, ys[r].data(), size_t(mm) * 8, hipMemcpyHostToDevice, st));
      if (prof) HIPCHK(hipEventRecord(ev2[2 * r], st));
      launch_lz_start(f + size_t(r) * n3, Xr, Hf, H0, g, nx, ny, 1, part, flag, br, ldb, st);
      for (int j = 1; j <= mm; ++j) {
        const double* cur = (j % 2 == 1) ? Xr : Yr;
        double* prv = (j % 2 == 1) ? Yr : Xr;
        launch_lz_step(cur, prv, Hf, H0, g, fc, nx, ny, 1, j, br, ldb, nullptr, yr, ldy, u + size_t(r) * n3,
                       j == mm ? 1 : 0, st);
      }
      if (prof) HIPCHK(hipEventRecord(ev2[2 * r + 1], st));
      HIPCHK(hipGetLastError());
    };
    const int chunk = 32;
    int m = 0, launched = 0, next_check = 0;
    bool done = false, hit_max = false;
    double host_s = 0.0;
    auto enqueue = [&](int upto) {
      for (int j = launched + 1; j <= upto; ++j) {
        const double* cur = (j % 2 == 1) ? X : Y;
        double* prv = (j % 2 == 1) ? Y : X;
        launch_lz_step(cur, prv, Hf, H0, g, fc, nx, ny, nrhs, j, beta, ldb, part, nullptr, 0, nullptr, 0, st);
      }
      launched = std::max(launched, upto);
    };
    while (!done) {
      enqueue(std::min(mmax, m + chunk));
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpy2DAsync(hbp + m + 1, size_t(ldb) * 8, beta + m + 1, size_t(ldb) * 8,
                              size_t(launched - m) * 8, nrhs, hipMemcpyDeviceToHost, st));
      wait_reads();
      for (int r = 0; r < nrhs; ++r)
        std::copy(hbp + size_t(r) * ldb + m + 1, hbp + size_t(r) * ldb + launched + 1, hb.begin() + size_t(r) * ldb + m + 1);
      m = launched;
      // breakdown: an invariant subspace of dimension j (exact result)
      double rho_all = 0.0;
      for (int r = 0; r < nrhs; ++r) {
        if (mr[r] != 0) continue;
        const double* b = hb.data() + size_t(r) * ldb;
        for (int j = 1; j <= m; ++j) {
          if (!(b[j] > 1e-13 * rho_ref) || !std::isfinite(b[j])) {
            mr[r] = j;
            break;
          }
          if (j >= 2) rho_all = std::max(rho_all, b[j - 1] + b[j]);
        }
      }
      rho_all = std::min(rho_all, rho_ref);
      const bool all_fixed = std::all_of(mr.begin(), mr.end(), [](int v) { return v != 0; });
      hit_max = (m >= mmax);
      if (!(all_fixed || hit_max || (m >= next_check && m >= 0.75 * t * rho_all))) continue;
      // the next chunk runs on the GPU while the host solves the small problems
      if (!all_fixed && !hit_max) enqueue(std::min(mmax, m + chunk));
      const auto h0 = std::chrono::steady_clock::now();
      // states share the operator and converge at similar m: stop at the
      // first one that has not converged yet
      bool conv = true;
      for (int r = 0; r < nrhs; ++r) {
        if (fin[r]) continue;
        if (mr[r] < 0) {  // zero state: u stays 0
          fin[r] = 1;
          continue;
        }
        const int mm = (mr[r] > 0) ? mr[r] : m;
        sr[r] = small_problem(hb.data() + size_t(r) * ldb, mm, t, o.h, m0, hb[size_t(r) * ldb], rho_ref, ys[r]);
        if (!(mr[r] > 0 || hit_max || sr[r].tail <= 0.1 * o.tol)) {
          conv = false;
          break;
        }
        mr[r] = mm;
        pass2(r, mm);
        fin[r] = 1;
      }
      host_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
      next_check = int(m * 1.1) + chunk;
      done = conv || hit_max;
    }
    int mfin = 0;
    int64_t m2 = 0;  // pass-2 steps over all states
    for (int r = 0; r < nrhs; ++r) {
      mfin = std::max(mfin, mr[r]);
      if (mr[r] > 0) m2 += mr[r];
    }
    if (prof) HIPCHK(hipEventRecord(ev[1], st));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    if (rep) {
      int P = 0, M = 0, N = 0;
      double rho = 0.0, kap = 0.0, tail = 0.0;
      int64_t tot = 0;
      for (int r = 0; r < nrhs; ++r) {
        if (mr[r] <= 0) continue;
        if (sr[r].P > P) {
          P = sr[r].P;
          M = sr[r].M;
          N = sr[r].N;
        }
        rho = std::max(rho, sr[r].rho);
        kap = std::max(kap, sr[r].kappa);
        tail = std::max(tail, sr[r].tail);
        tot += mr[r];
      }
      rep->P = P;
      rep->M = M;
      rep->N = N;
      rep->m0 = m0;
      rep->solves = mfin;
      rep->max_iters = mfin;
      rep->total_iters = tot;
      rep->not_converged = hit_max ? 1 : 0;
      rep->h = o.h;
      rep->t = t;
      rep->rho = rho;
      rep->kappa_sum = kap;
      rep->max_rel_residual = tail;
      rep->pole_tol = o.tol;
      // per step and state: pass 1 reads buf_j, buf_{j-1} (and the depth),
      // writes buf_{j+1}; pass 2 also reads and writes u
      const double per1 = (Hf ? 80.0 : 72.0), per2 = per1 + 48.0;
      rep->alg_bytes = (double(launched) * nrhs * per1 + double(m2) * per2) * double(n);
      rep->kernel_launches = 2 * int64_t(launched) + m2;
      if (prof) {
        float a = 0.f, b2 = 0.f;
        HIPCHK(hipEventElapsedTime(&a, ev[0], ev[1]));
        for (int r = 0; r < nrhs; ++r) {
          if (mr[r] <= 0) continue;
          float x = 0.f;
          HIPCHK(hipEventElapsedTime(&x, ev2[2 * r], ev2[2 * r + 1]));
          b2 += x;
        }
        rep->step_ms[0] = a - b2;     // pass 1 (GPU stream time less pass 2, host waits included)
        rep->step_ms[1] = host_s * 1e3;
        rep->step_ms[2] = b2;         // pass 2, summed over states
        rep->kernel_ms = b2;
        rep->kernel_bytes = double(m2) * double(n) * per2;
      }
      rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (hit_max) return set_error(REXII_ERR_NOT_CONVERGED, "Krylov dimension reached max_iter");
    return clear_error();
  } catch (const HipError& he) {
    return set_error(he.st, he.msg);
  } catch (const std::bad_alloc&) {
    return set_error(REXII_ERR_OOM, "host allocation failed");
  }
}

static size_t multishift_bytes(int nx, int ny, int nrhs, int max_iter) {
  const size_t n3 = 3 * size_t(nx) * ny;
  const int mmax = std::max(8, max_iter > 0 ? max_iter : kMultishiftMaxM);
  return 2 * al256(size_t(nrhs) * n3 * 8) + al256(size_t(nrhs) * lz_blocks(nx, ny) * 8) +
         al256(size_t(nrhs) * (mmax + 2) * 8) + al256(size_t(nrhs) * mmax * 8) + al256(256);
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
  o->max_iter = 0;
  o->m0 = -1;
  o->rho = 0.0;
  o->pole_batch = 0;
  o->pair_conjugate = 1;
  o->inner_tol = 1e-4;
}

rexii_status rexii_fourier_workspace_size(const rexii_swe_op* op, const rexii_opts* opts, double t, int32_t derivative,
                                          size_t* bytes) {
  rexii_status v = check_op_and_t(op, t, true, false);
  if (v != REXII_OK) return v;
  if (!bytes) return set_error(REXII_ERR_INVALID_ARG, "bytes is NULL");
  if (derivative != REXII_DERIV_CENTRED && derivative != REXII_DERIV_SPECTRAL)
    return set_error(REXII_ERR_INVALID_ARG, "unknown derivative");
  if (t == 0.0) {
    *bytes = 0;
    return clear_error();
  }
  FourierPlan fp;
  try {
    v = fourier_plan(op, t, resolve_opts(opts), derivative, fp);
  } catch (const HipError& he) {
    return set_error(he.st, he.msg);
  }
  if (v != REXII_OK) return v;
  size_t work = 0;
  v = fft_plans(op->nx, op->ny, &work, nullptr, nullptr);
  if (v != REXII_OK) return v;
  *bytes = fourier_bytes(op->nx, op->ny, derivative, fp.nterm, work);
  return clear_error();
}

rexii_status rexii_apply_fourier(const rexii_swe_op* op, const double* f, double* u, double t, int32_t derivative,
                                 const rexii_opts* opts, void* workspace, size_t ws_bytes, hipStream_t stream,
                                 rexii_report* rep) {
  rexii_status v = check_op_and_t(op, t, true, false);
  if (v != REXII_OK) return v;
  if (!f || !u) return set_error(REXII_ERR_INVALID_ARG, "NULL state pointer");
  if (derivative != REXII_DERIV_CENTRED && derivative != REXII_DERIV_SPECTRAL)
    return set_error(REXII_ERR_INVALID_ARG, "unknown derivative");
  const size_t n3 = 3 * size_t(op->nx) * op->ny;
  if (overlaps(f, n3, u, n3)) return set_error(REXII_ERR_INVALID_ARG, "u overlaps f");
  return run_fourier(op, f, u, t, derivative, opts, workspace, ws_bytes, stream, rep);
}

rexii_status rexii_apply_fourier_noalloc(const rexii_swe_op* op, const double* f, double* u, double t,
                                         int32_t derivative, const rexii_opts* opts, hipStream_t stream,
                                         rexii_report* rep) {
  rexii_status v = check_op_and_t(op, t, true, false);
  if (v != REXII_OK) return v;
  if (!f || !u) return set_error(REXII_ERR_INVALID_ARG, "NULL state pointer");
  if (derivative != REXII_DERIV_CENTRED && derivative != REXII_DERIV_SPECTRAL)
    return set_error(REXII_ERR_INVALID_ARG, "unknown derivative");
  const size_t n3 = 3 * size_t(op->nx) * op->ny;
  if (overlaps(f, n3, u, n3)) return set_error(REXII_ERR_INVALID_ARG, "u overlaps f");
  return run_fourier(op, f, u, t, derivative, opts, nullptr, 0, stream, rep, true);
}

rexii_status rexii_multishift_workspace_size(const rexii_swe_op* op, int32_t nrhs, const rexii_opts* opts,
                                             size_t* bytes) {
  rexii_status v = validate_op(op);
  if (v != REXII_OK) return v;
  if (!bytes || nrhs <= 0) return set_error(REXII_ERR_INVALID_ARG, "need bytes and nrhs > 0");
  *bytes = multishift_bytes(op->nx, op->ny, nrhs, resolve_opts(opts).max_iter);
  return clear_error();
}

rexii_status rexii_apply_multishift(const rexii_swe_op* op, int32_t nrhs, const double* f, double* u, double t,
                                    const rexii_opts* opts, void* workspace, size_t ws_bytes, hipStream_t stream,
                                    rexii_report* rep) {
  rexii_status v = check_op_and_t(op, t, true);
  if (v != REXII_OK) return v;
  if (nrhs <= 0 || nrhs > 65535) return set_error(REXII_ERR_INVALID_ARG, "nrhs must be in [1, 65535]");
  if (!f || !u) return set_error(REXII_ERR_INVALID_ARG, "NULL state pointer");
  const size_t nall = 3 * size_t(op->nx) * op->ny * size_t(nrhs);
  if (overlaps(f, nall, u, nall)) return set_error(REXII_ERR_INVALID_ARG, "u overlaps f");
  return run_multishift(op, nrhs, f, u, t, opts, workspace, ws_bytes, stream, rep);
}

const char* rexii_last_error(void) { return g_err.c_str(); }

rexii_status rexii_rho(const rexii_swe_op* op, hipStream_t stream, double* rho) {
  rexii_status st = validate_op(op);
  if (st != REXII_OK) return st;
  if (!rho) return set_error(REXII_ERR_INVALID_ARG, "rho is NULL");
  if (op->H_field) {
    try {
      const double hm = device_hmax(op->H_field, size_t(op->nx) * op->ny, stream);
      *rho = rho_bound_var(op->nx, op->ny, op->g, hm, op->f_cor);
    } catch (const HipError& he) {
      return set_error(he.st, he.msg);
    }
    return clear_error();
  }
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
  if (op->H_field) {
    // flux-form path: one problem, needs max H (read on the null stream)
    JobItem it;
    it.op = op;
    it.t = t;
    try {
      it.hmax = device_hmax(op->H_field, size_t(op->nx) * op->ny, nullptr);
    } catch (const HipError& he) {
      return set_error(he.st, he.msg);
    }
    if (o.method == 0) o.method = 1;
    size_t b = 0;
    try {
      st = items_bytes({it}, o, &b);
    } catch (const HipError& he) {
      return set_error(he.st, he.msg);
    }
    if (st != REXII_OK) return st;
    *bytes = b + 4096;
    return clear_error();
  }
  // the adjoint with dJ/dH is the largest user of one operator: two
  // problems, every solution kept, plus W^{-1} gbar and the dot buffers
  const size_t n = size_t(op->nx) * op->ny;
  JobItem G, F;
  G.op = F.op = op;
  G.t = F.t = t;
  G.adjoint = true;
  size_t b = 0;
  st = job_bytes({G, F}, o, true, al256(3 * n * 8) + 4096, &b);
  if (st != REXII_OK) return st;
  Problem pb;
  st = build_plan(op, t, o, true, false, pb.pl);
  if (st != REXII_OK) return st;
  const size_t nd = pb.pl.solves.size();
  b += al256(nd * sizeof(AdjDot)) + al256(nd * size_t(adj_dot_blocks(n)) * 16) + al256(nd * 16) + 4096;
  if (o.pole_batch < 0) {
    // rexii_apply with the autotuner may run more slots than the adjoint
    JobItem A;
    A.op = op;
    A.t = t;
    size_t ba = 0;
    st = items_bytes({A}, o, &ba);
    if (st != REXII_OK) return st;
    b = std::max(b, ba + 4096);
  }
  *bytes = b;
  return clear_error();
}

rexii_status rexii_batched_workspace_size(int32_t count, const rexii_swe_op* ops, const double* t,
                                          const rexii_opts* opts, size_t* bytes) {
  if (count <= 0 || !ops || !t || !bytes) return set_error(REXII_ERR_INVALID_ARG, "need count > 0, ops, t and bytes");
  std::vector<JobItem> items(count);
  rexii_opts o = resolve_opts(opts);
  bool any = false;
  try {
    for (int i = 0; i < count; ++i) {
      rexii_status v = check_op_and_t(&ops[i], t[i], true);
      if (v != REXII_OK) return v;
      items[i].op = &ops[i];
      items[i].t = t[i];
      if (t[i] == 0.0) {
        items[i].skip = true;
        continue;
      }
      any = true;
      if (ops[i].H_field) {
        items[i].hmax = device_hmax(ops[i].H_field, size_t(ops[i].nx) * ops[i].ny, nullptr);
        if (o.method == 0) o.method = 1;
      }
    }
    if (!any) {
      *bytes = 0;
      return clear_error();
    }
    size_t b = 0;
    rexii_status st = items_bytes(items, o, &b);
    if (st != REXII_OK) return st;
    *bytes = b + 4096;
  } catch (const HipError& he) {
    return set_error(he.st, he.msg);
  }
  return clear_error();
}

rexii_status rexii_apply(const rexii_swe_op* op, const double* f, double* u, double t, const rexii_opts* opts,
                         void* workspace, size_t ws_bytes, hipStream_t stream, rexii_report* rep) {
  rexii_status v = check_op_and_t(op, t, true);
  if (v != REXII_OK) return v;
  if (!f || !u) return set_error(REXII_ERR_INVALID_ARG, "NULL state pointer");
  const size_t n3 = 3 * size_t(op->nx) * op->ny;
  if (overlaps(f, n3, u, n3)) return set_error(REXII_ERR_INVALID_ARG, "u overlaps f");
  JobItem it;
  it.op = op;
  it.f = f;
  it.u = u;
  it.t = t;
  it.rep = rep;
  return run_items({it}, opts, workspace, ws_bytes, stream);
}

rexii_status rexii_shifted_solve(const rexii_swe_op* op, const double* f, double t, int32_t npoles, const double* z,
                                 double* x, const rexii_opts* opts, void* workspace, size_t ws_bytes,
                                 hipStream_t stream, rexii_report* rep) {
  rexii_status v = check_op_and_t(op, t, false);
  if (v != REXII_OK) return v;
  if (npoles <= 0 || !z || !x || !f) return set_error(REXII_ERR_INVALID_ARG, "need f, npoles > 0, z and x");
  std::vector<cd> sh(npoles);
  for (int k = 0; k < npoles; ++k) {
    sh[k] = cd(z[2 * k], z[2 * k + 1]);
    if (!(sh[k].real() != 0.0) || !std::isfinite(sh[k].real()) || !std::isfinite(sh[k].imag()))
      return set_error(REXII_ERR_INVALID_ARG, "shifts need a finite, non-zero real part");
  }
  JobItem it;
  it.op = op;
  it.f = f;
  it.t = t;
  it.shifts = &sh;
  it.xout = reinterpret_cast<double2*>(x);
  it.rep = rep;
  return run_items({it}, opts, workspace, ws_bytes, stream);
}

rexii_status rexii_apply_adjoint(const rexii_swe_op* op, const double* f, const double* gbar, double* dJdf,
                                 double* dJdH, double t, const rexii_opts* opts, void* workspace, size_t ws_bytes,
                                 hipStream_t stream, rexii_report* rep) {
  rexii_status v = check_op_and_t(op, t, false, false);
  if (v != REXII_OK) return v;
  if (!gbar) return set_error(REXII_ERR_INVALID_ARG, "gbar is NULL");
  if (!dJdf && !dJdH) return set_error(REXII_ERR_INVALID_ARG, "nothing to compute (dJdf and dJdH are NULL)");
  if (dJdH && !f) return set_error(REXII_ERR_INVALID_ARG, "dJdH needs f");
  const size_t n3 = 3 * size_t(op->nx) * op->ny;
  if (dJdf && (overlaps(dJdf, n3, gbar, n3) || (f && overlaps(dJdf, n3, f, n3))))
    return set_error(REXII_ERR_INVALID_ARG, "dJdf overlaps an input");
  return run_adjoint(op, f, gbar, dJdf, dJdH, t, opts, workspace, ws_bytes, stream, rep);
}

rexii_status rexii_apply_batched(int32_t count, const rexii_swe_op* ops, const double* const* f, double* const* u,
                                 const double* t, const rexii_opts* opts, void* workspace, size_t ws_bytes,
                                 hipStream_t stream, rexii_report* reps) {
  if (count <= 0 || !ops || !f || !u || !t) return set_error(REXII_ERR_INVALID_ARG, "need count > 0 and arrays");
  std::vector<JobItem> items(count);
  for (int i = 0; i < count; ++i) {
    rexii_status v = check_op_and_t(&ops[i], t[i], true);
    if (v != REXII_OK) return v;
    if (!f[i] || !u[i]) return set_error(REXII_ERR_INVALID_ARG, "NULL state pointer in batch");
    const size_t n3 = 3 * size_t(ops[i].nx) * ops[i].ny;
    if (overlaps(f[i], n3, u[i], n3)) return set_error(REXII_ERR_INVALID_ARG, "u overlaps f in batch");
    items[i].op = &ops[i];
    items[i].f = f[i];
    items[i].u = u[i];
    items[i].t = t[i];
    items[i].rep = reps ? &reps[i] : nullptr;
  }
  return run_items(items, opts, workspace, ws_bytes, stream);
}

}  // extern "C"
