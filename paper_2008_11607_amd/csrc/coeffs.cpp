// Host-side FP64 REXII coefficients: poles and weights of the reduced
// partial-fraction sum, the accuracy rule and the spectral radius bound.
//
// Paper: Caliari, Einkemmer, Moriggl, Ostermann, arXiv 2008.11607.
//   * b_m = e^{-imh} e^{h^2}                                   (Sec. 2.1, eq. bm)
//   * c_{1,n} = h sum_{k=L1(n)}^{L2(n)} Re(a_k) b_{n-k},
//     c_{2,n} = h sum_{k=L1(n)}^{L2(n)} Im(a_k) b_{n-k}          (eq. modifiedRexi)
//   * C_{1,n} = c_{1,n} h mu + c_{2,n} h n,  C_{2,n} = i c_{2,n}  (Sec. 2.2)
//   * reduced sum over n = 0..N with Gamma_0 = 1, Gamma_n = 2   (eq. modifiedRexiMatrixReducedSum)
//   * M = ceil(t rho / h) + m0                                  (eq. matrixAccuracyBound)
//   * m0 from psi_h(z) <= tol for |z| >= c h                     (Appendix B)
//   * mu and a_0..a_24                                          (Appendix A, Table coef_al)
//
// Term n, a rational function of X = tA, is
//   Gamma_n (C_{1,n} - C_{2,n} X) (alpha_{-n} - X)^{-1} (alpha_n + X)^{-1};
// its poles alpha_{-n} and -alpha_n differ by 2 h mu, so it splits into
//   w1 / (X - z1) + w2 / (X - z2),  z1 = h(mu - i n),  z2 = -h(mu + i n),
//   w1 = -Gamma_n (C1 - C2 z1) / (2 h mu),  w2 = Gamma_n (C1 - C2 z2) / (2 h mu).
// C1 - C2 z is formed directly: c_{2,n} can be ~1e-9, so the form with
// C1/C2 would lose accuracy.
#include "rexii_internal.h"

#include <cmath>
#include <algorithm>
#include <complex>
#include <map>
#include <mutex>
#include <vector>

namespace rexii {

namespace {

constexpr int kL = 24;
constexpr double kMu = -5.133333333333333;

// Appendix A: (Re a_l, Im a_l) for l = 0..24.  The sign column of the
// printed table applies to the real part only; a_{-l} = conj(a_l).
constexpr double kA[kL + 1][2] = {
    {-6.520430828919864e+01, 0.0},
    {4.261818064131437e+01, 2.761406741120911e+01},
    {-9.801650304425239e+00, -2.189295463610722e+01},
    {-1.054225194693395e+00, 6.791786454153551e+00},
    {7.950505668209775e-01, -8.904997258367445e-01},
    {-1.218558380859130e-01, 3.321241563407446e-02},
    {7.365401806949337e-03, 2.212802103193251e-03},
    {-2.801087265991056e-04, -5.566945197754387e-04},
    {1.254835436432561e-04, -2.467200513365371e-04},
    {2.295472292491263e-04, -8.494118951459107e-05},
    {1.858484460459430e-04, 9.242889460185034e-05},
    {4.068056518449676e-05, 1.653479957565515e-04},
    {-8.341508001647741e-05, 1.045331460447588e-04},
    {-9.970528169841103e-05, -5.856228484297677e-06},
    {-3.499639858693093e-05, -6.129059473910835e-05},
    {2.295021920298455e-05, -4.099832469456381e-05},
    {2.931048772724314e-05, 1.708815129697846e-07},
    {7.502088478301169e-06, 1.525082051744077e-05},
    {-5.815291167450100e-06, 6.919604247338349e-06},
    {-4.069948458364005e-06, -1.440010113050771e-06},
    {7.932524475429588e-08, -1.794169428574330e-06},
    {6.120984882186265e-07, -1.131894636585849e-07},
    {5.531365159161319e-08, 1.585749903175946e-07},
    {-2.867805871375946e-08, 1.239499740327838e-08},
    {-1.143081277095316e-09, -2.763239274253499e-09},
};

inline double a_re(int l) { return kA[l < 0 ? -l : l][0]; }
inline double a_im(int l) { return l >= 0 ? kA[l][1] : -kA[-l][1]; }

}  // namespace

double mu() { return kMu; }
int terms_L() { return kL; }

int m0_from_tol(double tol) {
  const double c = 2.0 * std::sqrt(-std::log(std::sqrt(4.0 * M_PI) * tol));
  return static_cast<int>(std::ceil(c - 1.0));
}

int m_rule(double t, double rho, double h, int m0) {
  return static_cast<int>(std::ceil(t * rho / h)) + m0;
}

void poles_weights(int M, double h, std::vector<cplx>& z, std::vector<cplx>& w) {
  using std::complex;
  const int N = M + kL;
  z.resize(2 * (N + 1));
  w.resize(2 * (N + 1));
  const double eh2 = std::exp(h * h);
  // Where the window is the full k = -L..L, b_{n-k} = e^{h^2} e^{-inh} e^{ikh}
  // makes the k-sum a fixed factor: c_{j,n} = h e^{h^2} e^{-inh} S_j.
  complex<double> S1(0.0, 0.0), S2(0.0, 0.0);
  for (int k = -kL; k <= kL; ++k) {
    const complex<double> e = std::polar(1.0, static_cast<double>(k) * h);
    S1 += a_re(k) * e;
    S2 += a_im(k) * e;
  }
  for (int n = 0; n <= N; ++n) {
    // c_{1,n}, c_{2,n}: k from L1(n) = max(-L, n-M) to L2(n) = min(L, n+M)
    complex<double> c1(0.0, 0.0), c2(0.0, 0.0);
    const int k1 = std::max(-kL, n - M), k2 = std::min(kL, n + M);
    if (k1 == -kL && k2 == kL) {
      const complex<double> e = std::polar(eh2, -static_cast<double>(n) * h);
      c1 = e * S1;
      c2 = e * S2;
    } else {
      for (int k = k1; k <= k2; ++k) {
        const double m = static_cast<double>(n - k);
        const complex<double> bm = std::polar(eh2, -m * h);  // e^{h^2} e^{-imh}
        c1 += a_re(k) * bm;
        c2 += a_im(k) * bm;
      }
    }
    c1 *= h;
    c2 *= h;
    const complex<double> C1 = c1 * (h * kMu) + c2 * (h * n);
    const complex<double> C2 = complex<double>(0.0, 1.0) * c2;
    const double gam = (n == 0) ? 1.0 : 2.0;
    const complex<double> z1(h * kMu, -h * n);    // alpha_{-n}
    const complex<double> z2(-h * kMu, -h * n);   // -alpha_n
    const complex<double> w1 = -gam * (C1 - C2 * z1) / (2.0 * h * kMu);
    const complex<double> w2 = gam * (C1 - C2 * z2) / (2.0 * h * kMu);
    z[2 * n] = {z1.real(), z1.imag()};
    z[2 * n + 1] = {z2.real(), z2.imag()};
    w[2 * n] = {w1.real(), w1.imag()};
    w[2 * n + 1] = {w2.real(), w2.imag()};
  }
}

// The original REXI matrix scheme (eq. originalREXImatrix):
//   REXI(tA) = sum_{n=-N}^{N} Re(beta^Re_n (tA + alpha_n I)^{-1}),
//   alpha_n = h (mu + i n),  beta^Re_n = h sum_k a_k Re(b_{n-k})  (eq. originalRexi),
// as Re sum w (tA - z)^{-1} with z = -alpha_n, w = beta^Re_n (a_k complex),
// ordered n = 0, 1, -1, 2, -2, ... (2N + 1 poles; z_{-n} = conj(z_n)).
void rexi_poles_weights(int M, double h, std::vector<cplx>& z, std::vector<cplx>& w) {
  using std::complex;
  const int N = M + kL;
  z.resize(2 * N + 1);
  w.resize(2 * N + 1);
  const double eh2 = std::exp(h * h);
  // full window: Re b_{n-k} = e^{h^2} (cos(nh) cos(kh) + sin(nh) sin(kh))
  complex<double> Sc(0.0, 0.0), Ss(0.0, 0.0);
  for (int k = -kL; k <= kL; ++k) {
    const complex<double> ak(a_re(k), a_im(k));
    Sc += ak * std::cos(k * h);
    Ss += ak * std::sin(k * h);
  }
  auto beta_re = [&](int n) {
    const int k1 = std::max(-kL, n - M), k2 = std::min(kL, n + M);
    complex<double> s(0.0, 0.0);
    if (k1 == -kL && k2 == kL) {
      s = eh2 * (std::cos(n * h) * Sc + std::sin(n * h) * Ss);
    } else {
      for (int k = k1; k <= k2; ++k) s += complex<double>(a_re(k), a_im(k)) * (eh2 * std::cos((n - k) * h));
    }
    return h * s;
  };
  for (int q = 0; q < 2 * N + 1; ++q) {
    const int n = (q + 1) / 2 * ((q % 2 == 1) ? 1 : -1);  // 0, 1, -1, 2, -2, ...
    const complex<double> b = beta_re(n);
    z[q] = {-h * kMu, -h * n};
    w[q] = {b.real(), b.imag()};
  }
}

// REXIE (eq. REXIE, the remark after eq. originalREXImatrix): for A = iB, B
// real with real eigenvectors, and real f,
//   exp(tA) f ~ sum_{n=-N}^{N} Re(beta^Re_n (tA + alpha_n I)^{-1} f)
//                            + i Re(beta^Im_n (tA + alpha_n I)^{-1} f),
// beta^Im_n = h sum_k a_k Im(b_{n-k}) (eq. originalRexi).  Poles z = -alpha_n
// and the two weight sets, ordered like rexi_poles_weights.
void rexie_terms(int M, double h, std::vector<cplx>& z, std::vector<cplx>& wre, std::vector<cplx>& wim) {
  using std::complex;
  const int N = M + kL;
  z.resize(2 * N + 1);
  wre.resize(2 * N + 1);
  wim.resize(2 * N + 1);
  const double eh2 = std::exp(h * h);
  for (int q = 0; q < 2 * N + 1; ++q) {
    const int n = (q + 1) / 2 * ((q % 2 == 1) ? 1 : -1);  // 0, 1, -1, 2, -2, ...
    const int k1 = std::max(-kL, n - M), k2 = std::min(kL, n + M);
    complex<double> br(0.0, 0.0), bi(0.0, 0.0);
    for (int k = k1; k <= k2; ++k) {
      const complex<double> ak(a_re(k), a_im(k));
      const double m = static_cast<double>(n - k);
      // b_m = e^{h^2} e^{-imh}: Re b_m = e^{h^2} cos(mh), Im b_m = -e^{h^2} sin(mh)
      br += ak * (eh2 * std::cos(m * h));
      bi += ak * (-eh2 * std::sin(m * h));
    }
    z[q] = {-h * kMu, -h * n};
    wre[q] = {h * br.real(), h * br.imag()};
    wim[q] = {h * bi.real(), h * bi.imag()};
  }
}

double kappa_sum(const std::vector<cplx>& w, double h) {
  double s = 0.0;
  for (const cplx& c : w) s += std::hypot(c.re, c.im);
  return s / std::fabs(h * kMu);
}

double max_s2(int n) {
  // max over k of (n sin(2 pi k / n))^2; O(n), so kept per n
  static std::mutex mu;
  static std::map<int, double> known;
  {
    std::lock_guard<std::mutex> lk(mu);
    const auto it = known.find(n);
    if (it != known.end()) return it->second;
  }
  double m = 0.0;
  for (int k = 0; k < n; ++k) {
    const double s = n * std::sin(2.0 * M_PI * k / n);
    m = std::max(m, s * s);
  }
  std::lock_guard<std::mutex> lk(mu);
  known[n] = m;
  return m;
}

double rho_const(int nx, int ny, double g, double H, double fc) {
  return std::sqrt(fc * fc + g * H * (max_s2(nx) + max_s2(ny)));
}

double rho_bound_var(int nx, int ny, double g, double Hmax, double fc) {
  return std::sqrt(g * Hmax) * std::sqrt(double(nx) * nx + double(ny) * ny) + std::fabs(fc);
}

}  // namespace rexii

extern "C" rexii_status rexii_coeffs_rexi(double t, double rho, double h, double tol, int32_t m0, int32_t* P,
                                          double* beta, double* alpha) {
  using namespace rexii;
  if (!P) return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs_rexi: P is NULL");
  if (!(t > 0.0) || !(rho > 0.0) || !(h > 0.0) || !(h < M_PI) || !std::isfinite(t) || !std::isfinite(rho))
    return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs_rexi: need t > 0, rho > 0, 0 < h < pi");
  if (m0 < 0) {
    if (!(tol > 0.0 && tol < 1.0)) return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs_rexi: tol must be in (0, 1)");
    m0 = m0_from_tol(tol);
  }
  if (std::ceil(t * rho / h) + m0 > 5.0e7) return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs_rexi: t*rho/h too large");
  const int M = m_rule(t, rho, h, m0);
  const int Pn = 2 * (M + terms_L()) + 1;
  *P = Pn;
  if (!beta && !alpha) return clear_error();
  std::vector<cplx> z, w;
  rexi_poles_weights(M, h, z, w);
  for (int k = 0; k < Pn; ++k) {
    if (beta) {
      beta[2 * k] = z[k].re / t;
      beta[2 * k + 1] = z[k].im / t;
    }
    if (alpha) {
      alpha[2 * k] = w[k].re / t;
      alpha[2 * k + 1] = w[k].im / t;
    }
  }
  return clear_error();
}

extern "C" rexii_status rexii_coeffs(double t, double rho, double h, double tol, int32_t m0,
                                     int32_t* P, double* beta, double* alpha, double* kappa) {
  using namespace rexii;
  if (!P) return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs: P is NULL");
  if (!(t > 0.0) || !(rho > 0.0) || !(h > 0.0) || !(h < M_PI) || !std::isfinite(t) ||
      !std::isfinite(rho))
    return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs: need t > 0, rho > 0, 0 < h < pi");
  if (m0 < 0) {
    if (!(tol > 0.0 && tol < 1.0))
      return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs: tol must be in (0, 1)");
    m0 = m0_from_tol(tol);
  }
  const double Md = std::ceil(t * rho / h) + m0;
  if (Md > 5.0e7) return set_error(REXII_ERR_INVALID_ARG, "rexii_coeffs: t*rho/h too large");
  const int M = m_rule(t, rho, h, m0);
  const int Pn = 2 * (M + terms_L() + 1);
  *P = Pn;
  if (!beta && !alpha && !kappa) return clear_error();
  std::vector<cplx> z, w;
  poles_weights(M, h, z, w);
  for (int k = 0; k < Pn; ++k) {
    if (beta) {
      beta[2 * k] = z[k].re / t;
      beta[2 * k + 1] = z[k].im / t;
    }
    if (alpha) {
      alpha[2 * k] = w[k].re / t;
      alpha[2 * k + 1] = w[k].im / t;
    }
  }
  if (kappa) *kappa = kappa_sum(w, h);
  return clear_error();
}

// ---------------------------------------------------------------------------
// A refit of the Gaussian's rational approximation (Sec. 2.1, step 2): the
// symmetric form R(x) of eq. A(x,mu), linear in y = [a_0, Re a_1..Re a_L,
// Im a_1..Im a_L], fitted by least squares (eq. minl2approx) on K points
// taken from n_candidates equally spaced values of [0, x_max] one at a
// time, Leja fashion: x_1 = 0, then the candidate with the largest product
// of distances to the points so far (near-ties, within 1e-12 relative of
// the log-product, go to the smallest x).  Householder QR, then one refinement
// step with the residual in extended precision (the matrix is
// ill-conditioned, ~1e12 at L = 24).
// ---------------------------------------------------------------------------
namespace rexii {
namespace {

// row of eq. A(x,mu) for one x
void design_row(double x, double m, int L, double* row) {
  const double x2 = x * x, m2 = m * m;
  row[0] = m / (x2 + m2);
  for (int l = 1; l <= L; ++l) {
    const double l2 = double(l) * l;
    const double den = x2 * x2 + 2.0 * (m2 - l2) * x2 + (m2 + l2) * (m2 + l2);
    row[l] = 2.0 * m * (m2 + l2 + x2) / den;
    row[L + l] = 2.0 * l * (m2 + l2 - x2) / den;
  }
}

// Least squares min |G y - b| for G (m x n, row-major, m >= n) by Householder
// QR: column k below the diagonal and the diagonal hold the reflector v_k
// (H_k = I - beta_k v_k v_k^T), the rest of the upper triangle holds R, and
// diag(R) is kept in rdiag.  The factorisation serves several right-hand
// sides (qr_solve).
struct QR {
  int m, n;
  std::vector<double> a;      // factored matrix, row-major
  std::vector<double> beta;   // reflector scalars
  std::vector<double> rdiag;  // diagonal of R
};

bool qr_factor(QR& q) {
  const int m = q.m, n = q.n;
  q.beta.assign(n, 0.0);
  q.rdiag.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double norm = 0.0;
    for (int i = k; i < m; ++i) norm = std::hypot(norm, q.a[size_t(i) * n + k]);
    if (norm == 0.0) return false;
    const double akk = q.a[size_t(k) * n + k];
    const double alpha = (akk > 0.0) ? -norm : norm;
    // v = x - alpha e1, stored in column k below and on the diagonal
    const double v0 = akk - alpha;
    q.a[size_t(k) * n + k] = v0;
    double vnorm2 = v0 * v0;
    for (int i = k + 1; i < m; ++i) vnorm2 += q.a[size_t(i) * n + k] * q.a[size_t(i) * n + k];
    q.beta[k] = 2.0 / vnorm2;
    for (int j = k + 1; j < n; ++j) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += q.a[size_t(i) * n + k] * q.a[size_t(i) * n + j];
      s *= q.beta[k];
      for (int i = k; i < m; ++i) q.a[size_t(i) * n + j] -= s * q.a[size_t(i) * n + k];
    }
    q.rdiag[k] = alpha;
  }
  return true;
}

std::vector<double> qr_solve(const QR& q, std::vector<double> b) {
  const int m = q.m, n = q.n;
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int i = k; i < m; ++i) s += q.a[size_t(i) * n + k] * b[i];
    s *= q.beta[k];
    for (int i = k; i < m; ++i) b[i] -= s * q.a[size_t(i) * n + k];
  }
  std::vector<double> y(n, 0.0);
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= q.a[size_t(k) * n + j] * y[j];
    y[k] = s / q.rdiag[k];
  }
  return y;
}

inline double psi_unit(double x) { return std::exp(-x * x / 4.0) / std::sqrt(4.0 * M_PI); }

}  // namespace
}  // namespace rexii

extern "C" rexii_status rexii_fit_gaussian(int32_t L, double mu, double x_max, int32_t K, int32_t n_candidates,
                                           double* a, double* points, double* max_err) {
  using namespace rexii;
  if (!a) return set_error(REXII_ERR_INVALID_ARG, "rexii_fit_gaussian: a is NULL");
  if (L < 1 || L > 64 || !(mu != 0.0) || !std::isfinite(mu) || !(x_max > 0.0) || !std::isfinite(x_max))
    return set_error(REXII_ERR_INVALID_ARG, "rexii_fit_gaussian: need 1 <= L <= 64, mu != 0, x_max > 0");
  const int ncol = 2 * L + 1;
  if (K < ncol || n_candidates < K || n_candidates > 20000000)
    return set_error(REXII_ERR_INVALID_ARG, "rexii_fit_gaussian: need 2L+1 <= K <= n_candidates <= 2e7");
  try {
    // Leja points on the candidate grid
    std::vector<double> cand(n_candidates), logp(n_candidates, 0.0);
    for (int i = 0; i < n_candidates; ++i) cand[i] = x_max * double(i) / double(n_candidates - 1);
    std::vector<double> pts;
    pts.reserve(K);
    pts.push_back(cand[0]);
    for (int k = 1; k < K; ++k) {
      const double last = pts.back();
      double bv = -INFINITY;
      for (int i = 0; i < n_candidates; ++i) {
        logp[i] += std::log(std::fabs(cand[i] - last));   // -inf at chosen points
        bv = std::max(bv, logp[i]);
      }
      if (!std::isfinite(bv)) return set_error(REXII_ERR_INVALID_ARG, "rexii_fit_gaussian: too few distinct candidates");
      // mirror-image candidates tie exactly: values within 1e-12 (relative)
      // of the largest count as ties, which go to the smallest x
      const double cut = bv - 1e-12 * std::max(1.0, std::fabs(bv));
      int best = 0;
      while (logp[best] < cut) ++best;
      pts.push_back(cand[best]);
    }
    QR q;
    q.m = K;
    q.n = ncol;
    q.a.resize(size_t(K) * ncol);
    std::vector<double> G(size_t(K) * ncol), b(K);
    for (int k = 0; k < K; ++k) {
      design_row(pts[k], mu, L, &G[size_t(k) * ncol]);
      b[k] = psi_unit(pts[k]);
    }
    q.a = G;
    if (!qr_factor(q)) return set_error(REXII_ERR_INVALID_ARG, "rexii_fit_gaussian: rank-deficient system");
    std::vector<double> y = qr_solve(q, b);
    // one refinement step: r = b - G y in extended precision
    std::vector<double> r(K);
    for (int k = 0; k < K; ++k) {
      long double s = b[k];
      for (int j = 0; j < ncol; ++j) s -= (long double)G[size_t(k) * ncol + j] * (long double)y[j];
      r[k] = double(s);
    }
    const std::vector<double> dy = qr_solve(q, r);
    for (int j = 0; j < ncol; ++j) y[j] += dy[j];
    a[0] = y[0];
    a[1] = 0.0;
    for (int l = 1; l <= L; ++l) {
      a[2 * l] = y[l];
      a[2 * l + 1] = y[L + l];
    }
    if (points)
      for (int k = 0; k < K; ++k) points[k] = pts[k];
    if (max_err) {
      // largest |psi_1 - R| over the candidate grid (both are even)
      std::vector<double> row(ncol);
      double e = 0.0;
      for (int i = 0; i < n_candidates; ++i) {
        design_row(cand[i], mu, L, row.data());
        double s = 0.0;
        for (int j = 0; j < ncol; ++j) s += row[j] * y[j];
        e = std::max(e, std::fabs(s - psi_unit(cand[i])));
      }
      *max_err = e;
    }
  } catch (const std::bad_alloc&) {
    return set_error(REXII_ERR_OOM, "rexii_fit_gaussian: host allocation failed");
  }
  return clear_error();
}
