// The paper's matrix experiments (Sec. 3.2) on the GPU: REXII
// (eq. modifiedRexiMatrixReducedSum), the original REXI
// (eq. originalREXImatrix) and REXIE (eq. REXIE) applied to a circulant
// matrix, (A f)_j = sum_d c_d f_{(j + d) mod n}, e.g. the periodic
// finite-difference matrices A_1 (advection) and A_2 (free Schroedinger).
//
// The DFT diagonalises every circulant matrix: on the mode e^{2 pi i j k / n}
// A acts as lambda(k) = sum_d c_d e^{2 pi i d k / n}, so each resolvent
// (tA - z)^{-1} is a division per mode and a scheme's pole sum is a function
// g(k) = sum_p w_p / (t lambda(k) - z_p).  The schemes take real parts of
// vectors in physical space; for real data f (DFT F with F(-k) = conj F(k))
// the DFT of Re(ifft(g F)) is m(k) F(k) with m(k) = (g(k) + conj g(-k)) / 2,
// so every scheme is: F = fft(f), U = m F, u = ifft(U).  REXIE has two pole
// sums (weights beta^Re and beta^Im) and m = m_re + i m_im; its shift nu
// (A - nu I = i B) is folded into lambda, and e^{t nu} into m.
//
// Kernels: k_circ_load (f real -> complex u, finiteness flag), rocFFT 1D
// complex transforms in place (batch of nrhs vectors), k_circ_sums (g per
// mode; 64 modes per block, term slices over the block's waves, slices
// added in wave order), k_circ_apply (u <- m u / n), and for REXII and REXI
// k_circ_real (the real part).  All FP64.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "rexii_internal.h"

namespace rexii {

namespace {

constexpr int kCircWaves = 16;     // most waves (term slices) per block
constexpr int kMaxStencil = 64;

struct CircStencil {
  int nst;
  int off[kMaxStencil];       // offsets d mod n, in [0, n)
  double re[kMaxStencil], im[kMaxStencil];
};

// Term table entry: pole z and the weights of the (one or two) sums.
struct CircTerm {
  double zr, zi, w1r, w1i, w2r, w2i;
};

// 1/x to full FP64 precision: hardware reciprocal estimate and two
// Newton-Raphson steps r <- r + r (1 - x r).
__device__ __forceinline__ double circ_recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// t (lambda(k) - i nu) for mode k.
__device__ inline void mode_symbol(const CircStencil& s, int k, int n, double t, double nu, double& xr, double& xi) {
  double lr = 0.0, li = 0.0;
  for (int q = 0; q < s.nst; ++q) {
    const long long dk = (static_cast<long long>(s.off[q]) * k) % n;
    double sn, cs;
    sincospi(2.0 * double(dk) / double(n), &sn, &cs);
    lr += s.re[q] * cs - s.im[q] * sn;
    li += s.re[q] * sn + s.im[q] * cs;
  }
  xr = t * lr;
  xi = t * (li - nu);
}

// g[k] (and g2[k] for two weight sets) = sum_p w_p / (x_k - z_p).  Block: 64
// modes (one per lane) x nw waves; wave w takes one slice of the terms (the
// term index is wave-uniform, so the table arrives through scalar loads).
// Two terms share one reciprocal: 1/d1 = d2 / (d1 d2) with d = |x - z|^2,
// which lies in [(h mu)^2, (|x| + h(N + |mu|))^2], so the product stays in
// range for any h above 1e-3 and |x| below 1e70.
template <bool TWO>
__global__ __launch_bounds__(64 * kCircWaves) void k_circ_sums(double2* __restrict__ g, double2* __restrict__ g2,
                                                               int n, CircStencil s, double t, double nu,
                                                               const CircTerm* __restrict__ tab, int nterm) {
  extern __shared__ double red[];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nw = int(blockDim.x >> 6);
  const int k = int(blockIdx.x) * 64 + lane;
  const bool live = k < n;
  double xr = 0.0, xi = 0.0;
  mode_symbol(s, live ? k : 0, n, t, nu, xr, xi);
  const int per = (nterm + nw - 1) / nw;
  const int lo = min(nterm, w * per), hi = min(nterm, lo + per);
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
  // w / (x - z) with 1 / (x - z) = conj(x - z) * inv, inv = 1 / |x - z|^2
  auto acc = [&](const CircTerm& q, double dr, double di, double inv) {
    const double er = dr * inv, ei = -di * inv;
    ar = fma(q.w1r, er, fma(-q.w1i, ei, ar));
    ai = fma(q.w1r, ei, fma(q.w1i, er, ai));
    if (TWO) {
      br = fma(q.w2r, er, fma(-q.w2i, ei, br));
      bi = fma(q.w2r, ei, fma(q.w2i, er, bi));
    }
  };
  int j = lo;
  for (; j + 1 < hi; j += 2) {
    const CircTerm q1 = tab[j], q2 = tab[j + 1];
    const double dr1 = xr - q1.zr, di1 = xi - q1.zi, dr2 = xr - q2.zr, di2 = xi - q2.zi;
    const double d1 = fma(dr1, dr1, di1 * di1), d2 = fma(dr2, dr2, di2 * di2);
    const double r = circ_recip(d1 * d2);
    acc(q1, dr1, di1, r * d2);
    acc(q2, dr2, di2, r * d1);
  }
  if (j < hi) {
    const CircTerm q = tab[j];
    const double dr = xr - q.zr, di = xi - q.zi;
    acc(q, dr, di, circ_recip(fma(dr, dr, di * di)));
  }
  if (nw > 1) {
    if (w > 0) {
      double* r = red + (w - 1) * 256;
      r[lane] = ar;
      r[64 + lane] = ai;
      r[128 + lane] = br;
      r[192 + lane] = bi;
    }
    __syncthreads();
    if (w != 0) return;
    for (int v = 1; v < nw; ++v) {
      const double* r = red + (v - 1) * 256;
      ar += r[lane];
      ai += r[64 + lane];
      br += r[128 + lane];
      bi += r[192 + lane];
    }
  }
  if (!live) return;
  g[k] = make_double2(ar, ai);
  if (TWO) g2[k] = make_double2(br, bi);
}

// u[r][k] <- m(k) u[r][k] / n with m(k) = (g(k) + conj g(-k)) / 2 (one sum),
// or m_re + i m_im (two sums), times the scalar e^{t nu} = (er, ei).
__global__ __launch_bounds__(256) void k_circ_apply(double2* __restrict__ u, const double2* __restrict__ g,
                                                    const double2* __restrict__ g2, int n, int nrhs, double er,
                                                    double ei) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= size_t(n) * nrhs) return;
  const int k = int(i % size_t(n));
  const int km = (k == 0) ? 0 : n - k;
  const double2 a = g[k], b = g[km];
  double mr = 0.5 * (a.x + b.x), mi = 0.5 * (a.y - b.y);
  if (g2) {
    const double2 c = g2[k], d = g2[km];
    // m_re + i m_im with m_im = ((c + conj d) / 2)
    const double pr = 0.5 * (c.x + d.x), pi = 0.5 * (c.y - d.y);
    mr -= pi;
    mi += pr;
  }
  const double inv = 1.0 / double(n);
  const double sr = (er * mr - ei * mi) * inv, si = (er * mi + ei * mr) * inv;
  const double2 v = u[i];
  u[i] = make_double2(sr * v.x - si * v.y, sr * v.y + si * v.x);
}

// u = (f, 0); flag[0] = 1 if a value of f is not finite.
__global__ void k_circ_load(const double* __restrict__ f, double2* __restrict__ u, size_t n, int* flag) {
  bool bad = false;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const double v = f[i];
    u[i] = make_double2(v, 0.0);
    bad = bad || !isfinite(v);
  }
  if (bad) atomicOr(flag, 1);
}

// REXII and REXI keep the real part of the vector (the inverse transform of
// the Hermitian spectrum leaves a rounding-level imaginary part).
__global__ void k_circ_real(double2* __restrict__ u, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    u[i].y = 0.0;
}

__global__ void k_circ_clear(int* flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

// ---------------------------------------------------------------------------
// rocFFT plans: batch of nrhs 1D complex transforms of length n, in place,
// FP64, cached per (device, n, nrhs) for the life of the process.
// ---------------------------------------------------------------------------
struct CircFft {
  rocfft_plan fwd = nullptr, inv = nullptr;
  size_t work = 0;
};
std::mutex g_circ_mu;
std::map<std::tuple<int, int, int>, CircFft> g_circ;

std::string rf_msg(const char* what, rocfft_status s) {
  return std::string(what) + " failed (rocfft status " + std::to_string(int(s)) + ")";
}

rexii_status circ_plans(int n, int nrhs, CircFft* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(REXII_ERR_HIP, "hipGetDevice failed");
  const rexii_status su = rocfft_ensure_setup();
  if (su != REXII_OK) return su;
  std::lock_guard<std::mutex> lk(g_circ_mu);
  const auto key = std::make_tuple(dev, n, nrhs);
  auto it = g_circ.find(key);
  if (it == g_circ.end()) {
    CircFft p;
    const size_t len[1] = {size_t(n)};
    rocfft_status s = rocfft_plan_create(&p.fwd, rocfft_placement_inplace, rocfft_transform_type_complex_forward,
                                         rocfft_precision_double, 1, len, size_t(nrhs), nullptr);
    if (s != rocfft_status_success) return set_error(REXII_ERR_HIP, rf_msg("rocfft_plan_create (forward)", s));
    s = rocfft_plan_create(&p.inv, rocfft_placement_inplace, rocfft_transform_type_complex_inverse,
                           rocfft_precision_double, 1, len, size_t(nrhs), nullptr);
    if (s != rocfft_status_success) {
      rocfft_plan_destroy(p.fwd);
      return set_error(REXII_ERR_HIP, rf_msg("rocfft_plan_create (inverse)", s));
    }
    size_t w1 = 0, w2 = 0;
    rocfft_plan_get_work_buffer_size(p.fwd, &w1);
    rocfft_plan_get_work_buffer_size(p.inv, &w2);
    p.work = std::max(w1, w2);
    it = g_circ.emplace(key, p).first;
  }
  *out = it->second;
  return REXII_OK;
}

inline size_t al256c(size_t b) { return (b + 255) & ~size_t(255); }

// Checked description of one call.
struct CircPlan {
  int n = 0, nrhs = 0, scheme = 0, M = 0, N = 0, P = 0, m0 = 0;
  double t = 0, nu = 0, h = 0.5, tol = 1e-10, rho = 0, kappa = 0;
  CircStencil st{};
  std::vector<CircTerm> terms;
};

rexii_status circ_plan(int32_t n, int32_t nstencil, const int32_t* offsets, const double* coefs, int32_t nrhs,
                       double t, double nu, int32_t scheme, int32_t M, const rexii_opts* opts, CircPlan& cp) {
  if (n < 2 || nrhs < 1 || size_t(n) * size_t(nrhs) > (size_t(1) << 31))
    return set_error(REXII_ERR_INVALID_ARG, "circulant: need n >= 2, nrhs >= 1 and n * nrhs <= 2^31");
  if (nstencil < 1 || nstencil > kMaxStencil || !offsets || !coefs)
    return set_error(REXII_ERR_INVALID_ARG, "circulant: need 1..64 stencil entries (offsets and coefs)");
  if (scheme < REXII_CIRC_REXII || scheme > REXII_CIRC_REXIE)
    return set_error(REXII_ERR_INVALID_ARG, "circulant: unknown scheme");
  if (!(t >= 0.0) || !std::isfinite(t) || !std::isfinite(nu))
    return set_error(REXII_ERR_INVALID_ARG, "circulant: need a finite t >= 0 and a finite nu");
  if (scheme != REXII_CIRC_REXIE && nu != 0.0)
    return set_error(REXII_ERR_INVALID_ARG, "circulant: the shift nu is a REXIE option");
  rexii_opts o;
  rexii_default_opts(&o);
  if (opts) o = *opts;
  cp.h = (o.h > 0.0) ? o.h : 0.5;
  cp.tol = (o.tol > 0.0) ? o.tol : 1e-10;
  if (!(cp.h < M_PI)) return set_error(REXII_ERR_INVALID_ARG, "circulant: need 0 < h < pi");
  cp.n = n;
  cp.nrhs = nrhs;
  cp.scheme = scheme;
  cp.t = t;
  cp.nu = nu;
  // the matrix as a sum per offset class (d mod n)
  std::map<int, std::pair<double, double>> cls;
  cp.st.nst = nstencil;
  for (int q = 0; q < nstencil; ++q) {
    const double re = coefs[2 * q], im = coefs[2 * q + 1];
    if (!std::isfinite(re) || !std::isfinite(im)) return set_error(REXII_ERR_INVALID_ARG, "circulant: coefficient not finite");
    const int d = int(((long long)offsets[q] % n + n) % n);
    cp.st.off[q] = d;
    cp.st.re[q] = re;
    cp.st.im[q] = im;
    cls[d].first += re;
    cls[d].second += im;
  }
  // the schemes' premises: REXII and REXI need A real with imaginary
  // spectrum (a real circulant matrix: skew-symmetric); REXIE needs
  // A - nu I = i B with B real symmetric (real eigenvectors)
  double cmax = 0.0;
  for (const auto& kv : cls) cmax = std::max(cmax, std::hypot(kv.second.first, kv.second.second));
  const double slack = 1e-13 * std::max(cmax, 1e-300);
  for (const auto& kv : cls) {
    const int d = kv.first, dm = (n - d) % n;
    const auto& a = kv.second;
    const auto itm = cls.find(dm);
    const std::pair<double, double> b = (itm == cls.end()) ? std::make_pair(0.0, 0.0) : itm->second;
    if (scheme == REXII_CIRC_REXIE) {
      if (std::fabs(a.first) > slack || std::fabs(a.second - b.second) > slack)
        return set_error(REXII_ERR_INVALID_ARG,
                         "circulant REXIE: A - nu I must be i times a real symmetric circulant matrix");
    } else {
      if (std::fabs(a.second) > slack || std::fabs(a.first + b.first) > slack)
        return set_error(REXII_ERR_INVALID_ARG,
                         "circulant REXII/REXI: A must be a real skew-symmetric circulant matrix");
    }
  }
  // rho = max_k |lambda(k) - i nu| (exact), unless given; O(n) sines, so
  // kept per (n, matrix, nu) for repeated calls (16 most recent)
  if (o.rho > 0.0) {
    cp.rho = o.rho;
  } else {
    using Key = std::tuple<int, double, std::vector<std::pair<int, std::pair<double, double>>>>;
    static std::mutex mu;
    static std::deque<std::pair<Key, double>> known;
    Key key{n, nu, std::vector<std::pair<int, std::pair<double, double>>>(cls.begin(), cls.end())};
    bool hit = false;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (const auto& e : known)
        if (e.first == key) {
          cp.rho = e.second;
          hit = true;
          break;
        }
    }
    if (!hit) {
      double r = 0.0;
      for (int k = 0; k < n; ++k) {
        double lr = 0.0, li = 0.0;
        for (const auto& kv : cls) {
          const double ph = 2.0 * M_PI * double((static_cast<long long>(kv.first) * k) % n) / double(n);
          const double cs = std::cos(ph), sn = std::sin(ph);
          lr += kv.second.first * cs - kv.second.second * sn;
          li += kv.second.first * sn + kv.second.second * cs;
        }
        r = std::max(r, std::hypot(lr, li - nu));
      }
      cp.rho = r;
      std::lock_guard<std::mutex> lk(mu);
      known.push_front({key, r});
      while (known.size() > 16) known.pop_back();
    }
  }
  cp.m0 = (o.m0 >= 0) ? o.m0 : m0_from_tol(cp.tol);
  if (M > 0) {
    cp.M = M;
  } else {
    const double Md = std::ceil(t * std::max(cp.rho, 1e-300) / cp.h) + cp.m0;
    if (Md > 5.0e7) return set_error(REXII_ERR_INVALID_ARG, "circulant: t*rho/h too large");
    cp.M = m_rule(t, std::max(cp.rho, 1e-300), cp.h, cp.m0);
  }
  if (cp.M > 50000000) return set_error(REXII_ERR_INVALID_ARG, "circulant: M too large");
  cp.N = cp.M + terms_L();
  // the term table depends on (scheme, M, h) only: kept for repeated calls
  // (8 most recent)
  using Key = std::tuple<int, int, double>;
  static std::mutex mu;
  static std::deque<std::pair<Key, std::pair<std::vector<CircTerm>, double>>> known;
  const Key key{scheme, cp.M, cp.h};
  {
    std::lock_guard<std::mutex> lk(mu);
    for (const auto& e : known)
      if (e.first == key) {
        cp.terms = e.second.first;
        cp.kappa = e.second.second;
        cp.P = int(cp.terms.size());
        return REXII_OK;
      }
  }
  std::vector<cplx> z, w1, w2;
  if (scheme == REXII_CIRC_REXII) {
    poles_weights(cp.M, cp.h, z, w1);
    cp.kappa = kappa_sum(w1, cp.h);
  } else if (scheme == REXII_CIRC_REXI) {
    rexi_poles_weights(cp.M, cp.h, z, w1);
    cp.kappa = kappa_sum(w1, cp.h);
  } else {
    rexie_terms(cp.M, cp.h, z, w1, w2);
    cp.kappa = kappa_sum(w1, cp.h) + kappa_sum(w2, cp.h);
  }
  cp.P = int(z.size());
  cp.terms.resize(z.size());
  for (size_t p = 0; p < z.size(); ++p) {
    CircTerm& q = cp.terms[p];
    q.zr = z[p].re;
    q.zi = z[p].im;
    q.w1r = w1[p].re;
    q.w1i = w1[p].im;
    q.w2r = w2.empty() ? 0.0 : w2[p].re;
    q.w2i = w2.empty() ? 0.0 : w2[p].im;
  }
  std::lock_guard<std::mutex> lk(mu);
  known.push_front({key, {cp.terms, cp.kappa}});
  while (known.size() > 8) known.pop_back();
  return REXII_OK;
}

size_t circ_bytes(const CircPlan& cp, size_t fft_work) {
  return al256c(size_t(cp.n) * 16) * 2 + al256c(cp.terms.size() * sizeof(CircTerm)) + 256 + al256c(fft_work) + 1024;
}

int circ_waves(int n, int nterm) {
  const int blocks = (n + 63) / 64;
  const int cap = (blocks < 1024) ? kCircWaves : 8;
  int nw = 1;
  while (nw < cap && nterm >= 64 * nw) nw *= 2;
  return nw;
}

void fill_circ_report(rexii_report* rep, const CircPlan& cp, double secs) {
  if (!rep) return;
  std::memset(rep, 0, sizeof(*rep));
  rep->P = cp.P;
  rep->M = cp.M;
  rep->N = cp.N;
  rep->m0 = cp.m0;
  rep->solves = cp.P;
  rep->h = cp.h;
  rep->t = cp.t;
  rep->rho = cp.rho;
  rep->kappa_sum = cp.kappa;
  rep->seconds = secs;
  rep->seconds_solve = secs;
  rep->total_iters = int64_t(cp.n);   // modes the pole sums were formed at
  rep->hist_buckets = 20;
  // f read and u written as complex, twice over by the transforms' own
  // passes aside: algorithmic bytes of the load and apply kernels
  rep->alg_bytes = double(cp.n) * cp.nrhs * (8.0 + 16.0 + 32.0) + double(cp.n) * 16.0 * (cp.scheme == 2 ? 2 : 1);
}

}  // namespace

}  // namespace rexii

extern "C" {

rexii_status rexii_circulant_workspace_size(int32_t n, int32_t nstencil, const int32_t* offsets, const double* coefs,
                                            int32_t nrhs, double t, double nu, int32_t scheme, int32_t M,
                                            const rexii_opts* opts, size_t* bytes) {
  using namespace rexii;
  if (!bytes) return set_error(REXII_ERR_INVALID_ARG, "bytes is NULL");
  CircPlan cp;
  rexii_status st = circ_plan(n, nstencil, offsets, coefs, nrhs, t, nu, scheme, M, opts, cp);
  if (st != REXII_OK) return st;
  CircFft fp;
  st = circ_plans(n, nrhs, &fp);
  if (st != REXII_OK) return st;
  *bytes = circ_bytes(cp, fp.work);
  return clear_error();
}

rexii_status rexii_apply_circulant(int32_t n, int32_t nstencil, const int32_t* offsets, const double* coefs,
                                   int32_t nrhs, const double* f, double* u, double t, double nu, int32_t scheme,
                                   int32_t M, const rexii_opts* opts, void* workspace, size_t ws_bytes,
                                   hipStream_t stream, rexii_report* rep) {
  using namespace rexii;
  const auto t0 = std::chrono::steady_clock::now();
  if (!f || !u) return set_error(REXII_ERR_INVALID_ARG, "circulant: NULL vector pointer");
  CircPlan cp;
  rexii_status st = circ_plan(n, nstencil, offsets, coefs, nrhs, t, nu, scheme, M, opts, cp);
  if (st != REXII_OK) return st;
  const size_t nall = size_t(n) * nrhs;
  {
    const char* fb = reinterpret_cast<const char*>(f);
    const char* ub = reinterpret_cast<const char*>(u);
    if (fb < ub + nall * 16 && ub < fb + nall * 8) return set_error(REXII_ERR_INVALID_ARG, "circulant: u overlaps f");
  }
  CircFft fp;
  st = circ_plans(n, nrhs, &fp);
  if (st != REXII_OK) return st;
  const size_t need = circ_bytes(cp, fp.work);
  char* base = static_cast<char*>(workspace);
  bool own = false;
  if (!workspace) {
    if (hipMalloc(reinterpret_cast<void**>(&base), need) != hipSuccess)
      return set_error(REXII_ERR_OOM, "circulant: device allocation failed");
    own = true;
  } else if (ws_bytes < need) {
    return set_error(REXII_ERR_WORKSPACE, "workspace smaller than rexii_circulant_workspace_size()");
  } else if (reinterpret_cast<uintptr_t>(workspace) & 255) {
    return set_error(REXII_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  }
  struct Free {
    char* p;
    bool own;
    ~Free() {
      if (own && p) (void)hipFree(p);
    }
  } fr{base, own};
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += al256c(b);
    return p;
  };
  double2* g = reinterpret_cast<double2*>(take(size_t(n) * 16));
  double2* g2 = reinterpret_cast<double2*>(take(size_t(n) * 16));
  CircTerm* dtab = reinterpret_cast<CircTerm*>(take(cp.terms.size() * sizeof(CircTerm)));
  int* flag = reinterpret_cast<int*>(take(256));
  void* work = fp.work ? take(fp.work) : nullptr;
  double2* ud = reinterpret_cast<double2*>(u);
  auto hipfail = [&](const char* what) { return set_error(REXII_ERR_HIP, std::string("circulant: ") + what + " failed"); };
  const bool prof = opts && opts->profile != 0;
  static thread_local hipEvent_t ev[6] = {};   // profiling events, created once per host thread
  if (prof && !ev[0])
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) return hipfail("hipEventCreate");
  auto mark = [&](int k) { return !prof || hipEventRecord(ev[k], stream) == hipSuccess; };
  hipLaunchKernelGGL(k_circ_clear, dim3(1), dim3(64), 0, stream, flag);
  if (!mark(0)) return hipfail("hipEventRecord");
  {
    size_t b = (nall + 255) / 256;
    b = std::min<size_t>(std::max<size_t>(b, 1), 4096);
    hipLaunchKernelGGL(k_circ_load, dim3(unsigned(b)), dim3(256), 0, stream, f, ud, nall, flag);
  }
  if (hipGetLastError() != hipSuccess) return hipfail("load kernel");
  if (t == 0.0) {
    int hflag = 0;
    if (hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return hipfail("flag read");
    fill_circ_report(rep, cp, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    if (hflag) return set_error(REXII_ERR_NONFINITE, "circulant: non-finite value in f");
    return clear_error();
  }
  if (hipMemcpyAsync(dtab, cp.terms.data(), cp.terms.size() * sizeof(CircTerm), hipMemcpyHostToDevice, stream) !=
      hipSuccess)
    return hipfail("term table upload");
  if (!mark(1)) return hipfail("hipEventRecord");
  st = fft_execute(fp.fwd, ud, ud, work, fp.work, stream);
  if (st != REXII_OK) return st;
  if (!mark(2)) return hipfail("hipEventRecord");
  const int nw = circ_waves(n, cp.P);
  const bool two = (scheme == REXII_CIRC_REXIE);
  if (two)
    hipLaunchKernelGGL(k_circ_sums<true>, dim3(unsigned((n + 63) / 64)), dim3(64 * nw),
                       size_t(nw - 1) * 256 * sizeof(double), stream, g, g2, n, cp.st, t, nu, dtab, cp.P);
  else
    hipLaunchKernelGGL(k_circ_sums<false>, dim3(unsigned((n + 63) / 64)), dim3(64 * nw),
                       size_t(nw - 1) * 256 * sizeof(double), stream, g, nullptr, n, cp.st, t, nu, dtab, cp.P);
  if (hipGetLastError() != hipSuccess) return hipfail("pole-sum kernel");
  if (!mark(3)) return hipfail("hipEventRecord");
  // REXIE: exp(tA) = e^{t nu} exp(t(A - nu I)), nu = i nu_im
  const double er = two ? std::cos(t * nu) : 1.0, ei = two ? std::sin(t * nu) : 0.0;
  hipLaunchKernelGGL(k_circ_apply, dim3(unsigned((nall + 255) / 256)), dim3(256), 0, stream, ud, g,
                     two ? g2 : nullptr, n, nrhs, er, ei);
  if (hipGetLastError() != hipSuccess) return hipfail("apply kernel");
  if (!mark(4)) return hipfail("hipEventRecord");
  st = fft_execute(fp.inv, ud, ud, work, fp.work, stream);
  if (st != REXII_OK) return st;
  if (!mark(5)) return hipfail("hipEventRecord");
  if (!two) {
    size_t b = (nall + 255) / 256;
    b = std::min<size_t>(std::max<size_t>(b, 1), 4096);
    hipLaunchKernelGGL(k_circ_real, dim3(unsigned(b)), dim3(256), 0, stream, ud, nall);
    if (hipGetLastError() != hipSuccess) return hipfail("real-part kernel");
  }
  int hflag = 0;
  if (hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return hipfail("stream synchronisation");
  fill_circ_report(rep, cp, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  if (rep) {
    rep->slots = nw;
    if (prof) {
      // load, forward FFT, pole sums, apply, inverse FFT (ms)
      for (int k = 0; k < 5; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) return hipfail("hipEventElapsedTime");
        rep->step_ms[k] = ms;
      }
      rep->kernel_ms = rep->step_ms[2];
      rep->kernel_launches = 1;
    }
  }
  if (hflag) return set_error(REXII_ERR_NONFINITE, "circulant: non-finite value in f");
  return clear_error();
}

}  // extern "C"
