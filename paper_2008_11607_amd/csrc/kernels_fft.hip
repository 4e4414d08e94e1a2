// Fourier-space REXII for a constant depth (the paper solves its test
// problem this way, per Fourier mode, Sec. 4).
//
// After a 2D FFT of (eta, u, v), mode k carries the 3 x 3 symbol
//   A(k) = [[0, -i H s_x, -i H s_y], [-i g s_x, 0, f_c], [-i g s_y, -f_c, 0]],
// with s = n sin(2 pi k / n) for centred differences, or s = 2 pi k (signed
// k, the odd derivative of the Nyquist mode taken as 0) for Fourier
// differentiation.  Its eigenvalues are 0 and +-i omega,
// omega^2 = f_c^2 + g H (s_x^2 + s_y^2), so for X = t A(k) and theta = t omega
// any function r of X is the quadratic that interpolates r on {0, +-i theta}
// (Theorem 1 of the paper, matrix functions through the eigenvalues):
//   r(X) = c0 I + c1 X + c2 X^2.
// For one pole, r(x) = w / (x - z), the Newton divided differences on the
// nodes (0, i theta, -i theta) are w/(-z), w/(z (i theta - z)) and
// -w/(z (z^2 + theta^2)), which give
//   c1 = -w / (z^2 + theta^2),  c2 = (-w / z) / (z^2 + theta^2).
// The result must be real (eq. modifiedRexiMatrixReducedSum takes the real
// part); since A(-k) = conj(A(k)) and F(-k) = conj(F(k)) for a real state,
// the real part in physical space is, per mode, the same quadratic with
// Re c0, Re c1, Re c2.  So the half spectrum of a real-to-complex FFT is
// filtered with real coefficients and a complex-to-real FFT returns u.
//
// Per term of the sum the filter needs Re(c1) and Re(c2) at theta^2:
// with z^2 = a + i b and s = a + theta^2,
//   Re(-w e) = -(w_r s + w_i b) / (s^2 + b^2),  e = 1/(z^2 + theta^2),
// and the two poles of one term of the reduced sum have equal a and b^2
// (z_2 = -conj(z_1)), so they share the denominator s^2 + b^2 and are
// merged into one table entry (a, b^2, A1, B1, A2, B2):
//   Re c1 += (A1 s + B1) / (s^2 + b^2),  Re c2 += (A2 s + B2) / (s^2 + b^2).
// theta^2 depends on the mode only through s_x^2 and s_y^2, which repeat
// along each axis, so the sums are formed once per distinct pair
// (k_mode_coef) and a second kernel applies the quadratic to every mode
// (k_mode_apply).  On square grids the pair is unordered (s_x and s_y are
// the same function), which halves the table again.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "kernels.h"
#include "kernels_fft.h"
#include "rexii_internal.h"

namespace rexii {

constexpr int kModeWaves = 16;  // most waves (term slices) per block
constexpr int kTermDoubles = 6;

// 1/x to full FP64 precision: hardware reciprocal estimate and two
// Newton-Raphson steps r <- r + r (1 - x r) (each squares the relative error).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// s * s + b with b read from a scalar register (one VOP3 instruction; the
// compiler otherwise copies b into vector registers for a VOP2 fmac).
__device__ __forceinline__ double sq_plus(double s, double b) {
  double d;
  asm("v_fma_f64 %0, %1, %1, %2" : "=v"(d) : "v"(s), "s"(b));
  return d;
}

// s for wavenumber index k of an axis of n points (see file comment); the
// kernels read it from a table the host fills once per grid.
double axis_symbol(int k, int n, int deriv) {
  if (deriv == 0) return double(n) * std::sin(2.0 * M_PI * double(k) / double(n));
  const int ks = (2 * k == n) ? 0 : (2 * k < n ? k : k - n);
  return 2.0 * M_PI * double(ks);
}

// Re c1 and Re c2 at theta^2 = th2 over the terms [w per, (w + 1) per) of
// the table (per = ceil(nterm / nw)); the table index is wave-uniform, so
// the entries arrive through scalar loads.
__device__ __forceinline__ void term_sums(const double* __restrict__ tab, int nterm, int w, int nw, double th2,
                                          double& c1, double& c2) {
  const int per = (nterm + nw - 1) / nw;
  const int lo = min(nterm, w * per), hi = min(nterm, lo + per);
  // (A s + B) / d is accumulated as (s/d) A + (1/d) B: one scalar (table)
  // operand per FMA, and four independent chains.  Four terms share one
  // reciprocal: 1/d1 = (d2 d3 d4) / (d1 d2 d3 d4).  d >= b^2 = (2 h^2 mu n)^2
  // for n >= 1 and d >= a^2 = (h mu)^4 for n = 0, and d < 4 (theta^2 + (h N)^2)^2,
  // so the product stays in range for any h above 1e-3 and theta below 1e18.
  double c1a = 0.0, c1b = 0.0, c2a = 0.0, c2b = 0.0;
  auto one = [&](const double* q, double i1) {
    const double e1 = i1 * (q[0] + th2);
    c1a = fma(e1, q[2], c1a);
    c1b = fma(i1, q[3], c1b);
    c2a = fma(e1, q[4], c2a);
    c2b = fma(i1, q[5], c2b);
  };
  auto den = [&](const double* q) { return sq_plus(q[0] + th2, q[1]); };
  auto pair = [&](const double* q) {
    const double d1 = den(q), d2 = den(q + kTermDoubles);
    const double r = recip(d1 * d2);
    one(q, r * d2);
    one(q + kTermDoubles, r * d1);
  };
  auto quad = [&](const double* q) {
    const double d1 = den(q), d2 = den(q + kTermDoubles);
    const double d3 = den(q + 2 * kTermDoubles), d4 = den(q + 3 * kTermDoubles);
    const double p12 = d1 * d2, p34 = d3 * d4;
    const double r = recip(p12 * p34);
    const double r12 = r * p34, r34 = r * p12;
    one(q, r12 * d2);
    one(q + kTermDoubles, r12 * d1);
    one(q + 2 * kTermDoubles, r34 * d4);
    one(q + 3 * kTermDoubles, r34 * d3);
  };
  int j = lo;
  for (; j + 7 < hi; j += 8) {  // unrolled by hand: the loads of two quads issue together
    const double* q = tab + size_t(j) * kTermDoubles;
    quad(q);
    quad(q + 4 * kTermDoubles);
  }
  for (; j + 1 < hi; j += 2) pair(tab + size_t(j) * kTermDoubles);
  if (j < hi) {
    const double* q = tab + size_t(j) * kTermDoubles;
    one(q, recip(den(q)));
  }
  c1 = c1a + c1b;
  c2 = c2a + c2b;
}

// Canonical wavenumber of k on an axis of n points: the smallest index
// with the same s^2 (centred differences: sin^2(2 pi k / n) has period n/2
// and is symmetric about n/4 for even n, symmetric about n/2 for odd n;
// Fourier differentiation: s^2 depends on |signed k|, the Nyquist mode's
// derivative is 0).  theta, and with it the coefficients of r(t A(k)),
// depends on the mode only through these two numbers.
__host__ __device__ inline int canon_index(int k, int n, int deriv) {
  if (deriv == 0 && n % 2 == 0) {
    const int h = n / 2, kc = k % h;
    return kc < h - kc ? kc : h - kc;
  }
  if (deriv != 0 && 2 * k == n) return 0;
  return k < n - k ? k : n - k;
}

int canon_count(int n, int kmax, int deriv) {
  int c = 0;
  for (int k = 0; k <= kmax; ++k) {
    const int v = canon_index(k, n, deriv);
    c = v > c ? v : c;
  }
  return c + 1;
}

// The pole sums per distinct frequency: coef[cy * cnx + cx] = scale (Re c1,
// Re c2) at theta^2 = t^2 (f_c^2 + g H (s_x^2 + s_y^2)) for the canonical
// wavenumbers (cx, cy).  tab: nterm entries of kTermDoubles.  Block: 64
// entries (one per lane) x nw waves; grid row s (blockIdx.y) takes split s of
// the terms, wave w of the block slice w of that split, and the slices are
// added in wave order through (nw - 1) x 1 KB of dynamic LDS.  With one
// split the block writes scale (c1, c2) to coef; with several it writes its
// unscaled sums to part[s][e] and k_mode_coef_sum adds the splits in order.
// Symmetric tables (square grids: s_x and s_y are the same function, so the
// pairs (a, b) and (b, a) share theta): entries e = b (b + 1) / 2 + a, a <= b.
__host__ __device__ inline int tri_index(int a, int b) { return a <= b ? b * (b + 1) / 2 + a : a * (a + 1) / 2 + b; }
__device__ inline void tri_coords(int e, int& a, int& b) {
  b = int((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
  if ((b + 1) * (b + 2) / 2 <= e) ++b;
  if (b * (b + 1) / 2 > e) --b;
  a = e - b * (b + 1) / 2;
}

__global__ __launch_bounds__(64 * kModeWaves) void k_mode_coef(double2* __restrict__ coef,
                                                               double2* __restrict__ part, int cnx, int cny, int sym,
                                                               const double* __restrict__ sxt,
                                                               const double* __restrict__ syt, double t, double g,
                                                               double H, double fc, double scale,
                                                               const double* __restrict__ tab, int nterm) {
  extern __shared__ double red[];
  const int ne = sym ? cnx * (cnx + 1) / 2 : cnx * cny;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nw = int(blockDim.x >> 6);
  const int ns = int(gridDim.y), sp = int(blockIdx.y);
  const int per_s = (nterm + ns - 1) / ns;
  const int lo_s = min(nterm, sp * per_s), cnt_s = min(nterm, lo_s + per_s) - lo_s;
  const int e = int(blockIdx.x) * 64 + lane;
  const bool live = e < ne;
  int cx = 0, cy = 0;
  if (live) {
    if (sym) {
      tri_coords(e, cx, cy);
    } else {
      cx = e % cnx;
      cy = e / cnx;
    }
  }
  const double sx = sxt[cx], sy = syt[cy];
  const double th2 = t * t * fma(g * H, fma(sx, sx, sy * sy), fc * fc);
  double c1, c2;
  term_sums(tab + size_t(lo_s) * kTermDoubles, cnt_s, w, nw, th2, c1, c2);
  if (nw > 1) {
    if (w > 0) {
      red[(w - 1) * 128 + lane] = c1;
      red[(w - 1) * 128 + 64 + lane] = c2;
    }
    __syncthreads();
    if (w != 0) return;
    for (int v = 1; v < nw; ++v) {
      c1 += red[(v - 1) * 128 + lane];
      c2 += red[(v - 1) * 128 + 64 + lane];
    }
  }
  if (!live) return;
  if (ns == 1)
    coef[e] = make_double2(scale * c1, scale * c2);
  else
    part[size_t(sp) * ne + e] = make_double2(c1, c2);
}

// coef[e] = scale sum_s part[s][e], splits added in index order.
__global__ __launch_bounds__(256) void k_mode_coef_sum(double2* __restrict__ coef, const double2* __restrict__ part,
                                                       int ne, int ns, double scale) {
  const int e = int(blockIdx.x) * 256 + threadIdx.x;
  if (e >= ne) return;
  double c1 = 0.0, c2 = 0.0;
  for (int s = 0; s < ns; ++s) {
    const double2 v = part[size_t(s) * ne + e];
    c1 += v.x;
    c2 += v.y;
  }
  coef[e] = make_double2(scale * c1, scale * c2);
}

// F: [3][ny][nxh] half spectra, filtered in place with the coefficients of
// the mode's canonical frequency: F <- scale c0 F + C1 X F + C2 X^2 F,
// X = t A(k) with the mode's own (signed) symbols.
__global__ __launch_bounds__(256) void k_mode_apply(double2* __restrict__ F, const double2* __restrict__ coef,
                                                    int ns, int ne, double scale, int cnx, int sym, int nx, int ny,
                                                    int deriv, const double* __restrict__ sxt,
                                                    const double* __restrict__ syt, double t, double g, double H,
                                                    double fc, double a0) {
  const int nxh = nx / 2 + 1;
  const int nm = nxh * ny;
  const int m = int(blockIdx.x) * 256 + threadIdx.x;
  if (m >= nm) return;
  const int kx = m % nxh, ky = m / nxh;
  const int ca = canon_index(kx, nx, deriv), cb = canon_index(ky, ny, deriv);
  const int e = sym ? tri_index(ca, cb) : cb * cnx + ca;
  double2 c;
  if (ns <= 1) {
    c = coef[e];
  } else {
    // the splits' unscaled sums, added in split order (as k_mode_coef_sum)
    double c1 = 0.0, c2 = 0.0;
    for (int q = 0; q < ns; ++q) {
      const double2 v = coef[size_t(q) * ne + e];
      c1 += v.x;
      c2 += v.y;
    }
    c = make_double2(scale * c1, scale * c2);
  }
  const double sx = sxt[kx], sy = syt[ky];
  double2 f[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) f[q] = F[size_t(q) * nm + m];
  // X v with X = t A(k); -i a (x + i y) = (a y, -a x)
  const double hx = t * H * sx, hy = t * H * sy, gx = t * g * sx, gy = t * g * sy, tf = t * fc;
  auto apply = [&](const double2 (&v)[3], double2 (&o)[3]) {
    o[0] = make_double2(hx * v[1].y + hy * v[2].y, -(hx * v[1].x + hy * v[2].x));
    o[1] = make_double2(gx * v[0].y + tf * v[2].x, -gx * v[0].x + tf * v[2].y);
    o[2] = make_double2(gy * v[0].y - tf * v[1].x, -gy * v[0].x - tf * v[1].y);
  };
  double2 x1[3], x2[3];
  apply(f, x1);
  apply(x1, x2);
#pragma unroll
  for (int q = 0; q < 3; ++q)
    F[size_t(q) * nm + m] = make_double2(a0 * f[q].x + c.x * x1[q].x + c.y * x2[q].x,
                                         a0 * f[q].y + c.x * x1[q].y + c.y * x2[q].y);
}

// u = f; flags[b] = 1 if block b met a value that is not finite, else 0
// (every block writes its word, so nothing has to be cleared first).
__global__ __launch_bounds__(256) void k_copy_check(const double* __restrict__ f, double* __restrict__ u, size_t n,
                                                    int* __restrict__ flags) {
  bool bad = false;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const double v = f[i];
    u[i] = v;
    bad = bad || !isfinite(v);
  }
  const int any = __syncthreads_or(bad ? 1 : 0);
  if (threadIdx.x == 0) flags[blockIdx.x] = any;
}

// Shape of k_mode_coef: waves per block (kCoefWaves, fewer when a wave would
// get under 64 terms) and term splits (grid rows): blocks up to about
// kCoefBlocks (32 per CU) while every wave keeps at least kMinTermsPerWave
// terms.  Measured (pole-sum stage, events; waves x splits) on square grids
// with the unordered table: 512^2 at t rho 1000 (132 entry blocks, 2034
// terms) 8 x 4: 16.8 us, 8 x 8: 16.1, 4 x 8: 16.0, 4 x 16: 21.0, 2 x 16:
// 21.1, 8 x 2: 19.6; 2048^2 at t rho 5000 (2060 entry blocks, 10034 terms)
// 8 x 4: 533 us, 8 x 2: 508, 8 x 1: 528, 4 x 4: 475, 4 x 8: 471, 2 x 8: 475.
constexpr int kCoefWaves = 4;
constexpr int kCoefBlocks = 8192;
constexpr int kMinTermsPerWave = 32;
// Split sums of at most this many bytes are added by k_mode_apply as it reads
// them (they stay in L2); larger ones by k_mode_coef_sum first.
constexpr size_t kSplitsInApplyBytes = size_t(2) << 20;

void mode_coef_shape(int entries, int nterm, int* nw_out, int* ns_out) {
  const int blocks = (entries + 63) / 64;
  int nw = 1;
  while (nw < kCoefWaves && nterm >= 128 * nw) nw *= 2;
  int ns = 1;
  while (ns < 64 && blocks * ns < kCoefBlocks && nterm >= 2 * ns * nw * kMinTermsPerWave) ns *= 2;
  *nw_out = nw;
  *ns_out = ns;
}

int mode_entries(int cnx, int cny, int sym) { return sym ? cnx * (cnx + 1) / 2 : cnx * cny; }

bool mode_sum_in_apply(int entries, int ns) { return ns > 1 && size_t(ns) * entries * 16 <= kSplitsInApplyBytes; }

void launch_mode_coef(double2* coef, double2* part, int cnx, int cny, int sym, const double* sxt, const double* syt,
                      double t, double g, double H, double fc, double scale, const double* tab, int nterm, int nw,
                      int ns, hipStream_t s) {
  const int ne = mode_entries(cnx, cny, sym);
  const size_t lds = size_t(nw - 1) * 128 * sizeof(double);
  hipLaunchKernelGGL(k_mode_coef, dim3(unsigned((ne + 63) / 64), unsigned(ns)), dim3(64 * nw), lds, s, coef, part,
                     cnx, cny, sym, sxt, syt, t, g, H, fc, scale, tab, nterm);
  if (ns > 1 && !mode_sum_in_apply(ne, ns))
    hipLaunchKernelGGL(k_mode_coef_sum, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, s, coef, part, ne, ns, scale);
}

void launch_mode_apply(double2* F, const double2* coef, int ns, int ne, double scale, int cnx, int sym, int nx,
                       int ny, int deriv, const double* sxt, const double* syt, double t, double g, double H,
                       double fc, double a0, hipStream_t s) {
  const long nm = long(nx / 2 + 1) * ny;
  hipLaunchKernelGGL(k_mode_apply, dim3(unsigned((nm + 255) / 256)), dim3(256), 0, s, F, coef, ns, ne, scale, cnx,
                     sym, nx, ny, deriv, sxt, syt, t, g, H, fc, a0);
}

int copy_check_blocks(size_t n) {
  const size_t b = (n + 255) / 256;
  return int(b < 1 ? 1 : (b > size_t(kCopyCheckMaxBlocks) ? size_t(kCopyCheckMaxBlocks) : b));
}

void launch_copy_check(const double* f, double* u, size_t n, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_check, dim3(unsigned(copy_check_blocks(n))), dim3(256), 0, s, f, u, n, flags);
}

// ---------------------------------------------------------------------------
// rocFFT plans: batch of 3 real 2D transforms, [3][ny][nx] real <->
// [3][ny][nx/2+1] complex, not in place, FP64.  Cached per (device, nx, ny)
// for the life of the process.
// ---------------------------------------------------------------------------
namespace {
struct FftPair {
  rocfft_plan fwd = nullptr, inv = nullptr;
  size_t work = 0;
};
std::mutex g_fft_mu;
std::map<std::tuple<int, int, int>, FftPair> g_fft;
bool g_fft_setup = false;

std::string fft_msg(const char* what, rocfft_status s) { return std::string(what) + " failed (rocfft status " + std::to_string(int(s)) + ")"; }
}  // namespace

rexii_status rocfft_ensure_setup() {
  std::lock_guard<std::mutex> lk(g_fft_mu);
  if (!g_fft_setup) {
    const rocfft_status s = rocfft_setup();
    if (s != rocfft_status_success) return set_error(REXII_ERR_HIP, fft_msg("rocfft_setup", s));
    g_fft_setup = true;
  }
  return REXII_OK;
}

rexii_status fft_plans(int nx, int ny, size_t* work_bytes, void** fwd, void** inv, bool create) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(REXII_ERR_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_fft_mu);
  if (!create) {
    const auto found = g_fft.find(std::make_tuple(dev, nx, ny));
    if (found == g_fft.end())
      return set_error(REXII_ERR_INVALID_ARG,
                       "no FFT plan for this grid on this device yet: call rexii_fourier_workspace_size "
                       "(or rexii_apply_fourier) for it first; creating a plan allocates device memory");
    if (work_bytes) *work_bytes = found->second.work;
    if (fwd) *fwd = found->second.fwd;
    if (inv) *inv = found->second.inv;
    return REXII_OK;
  }
  if (!g_fft_setup) {
    const rocfft_status s = rocfft_setup();
    if (s != rocfft_status_success) return set_error(REXII_ERR_HIP, fft_msg("rocfft_setup", s));
    g_fft_setup = true;
  }
  const auto key = std::make_tuple(dev, nx, ny);
  auto it = g_fft.find(key);
  if (it == g_fft.end()) {
    FftPair p;
    const size_t len[2] = {size_t(nx), size_t(ny)};  // fastest dimension first
    rocfft_status s = rocfft_plan_create(&p.fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                                         rocfft_precision_double, 2, len, 3, nullptr);
    if (s != rocfft_status_success) return set_error(REXII_ERR_HIP, fft_msg("rocfft_plan_create (forward)", s));
    s = rocfft_plan_create(&p.inv, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                           rocfft_precision_double, 2, len, 3, nullptr);
    if (s != rocfft_status_success) {
      rocfft_plan_destroy(p.fwd);
      return set_error(REXII_ERR_HIP, fft_msg("rocfft_plan_create (inverse)", s));
    }
    size_t w1 = 0, w2 = 0;
    rocfft_plan_get_work_buffer_size(p.fwd, &w1);
    rocfft_plan_get_work_buffer_size(p.inv, &w2);
    p.work = w1 > w2 ? w1 : w2;
    it = g_fft.emplace(key, p).first;
  }
  if (work_bytes) *work_bytes = it->second.work;
  if (fwd) *fwd = it->second.fwd;
  if (inv) *inv = it->second.inv;
  return REXII_OK;
}

// Batch of `batch` complex 2D transforms [batch][ny][nx], in place, FP64,
// forward and inverse (unnormalised); cached per (device, nx, ny, batch).
namespace {
std::map<std::tuple<int, int, int, int>, FftPair> g_fft_c2c;
}

rexii_status fft_plans_c2c(int nx, int ny, int batch, size_t* work_bytes, void** fwd, void** inv) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(REXII_ERR_HIP, "hipGetDevice failed");
  const rexii_status su = rocfft_ensure_setup();
  if (su != REXII_OK) return su;
  std::lock_guard<std::mutex> lk(g_fft_mu);
  const auto key = std::make_tuple(dev, nx, ny, batch);
  auto it = g_fft_c2c.find(key);
  if (it == g_fft_c2c.end()) {
    FftPair p;
    const size_t len[2] = {size_t(nx), size_t(ny)};
    rocfft_status s = rocfft_plan_create(&p.fwd, rocfft_placement_inplace, rocfft_transform_type_complex_forward,
                                         rocfft_precision_double, 2, len, size_t(batch), nullptr);
    if (s != rocfft_status_success) return set_error(REXII_ERR_HIP, fft_msg("rocfft_plan_create (c2c forward)", s));
    s = rocfft_plan_create(&p.inv, rocfft_placement_inplace, rocfft_transform_type_complex_inverse,
                           rocfft_precision_double, 2, len, size_t(batch), nullptr);
    if (s != rocfft_status_success) {
      rocfft_plan_destroy(p.fwd);
      return set_error(REXII_ERR_HIP, fft_msg("rocfft_plan_create (c2c inverse)", s));
    }
    size_t w1 = 0, w2 = 0;
    rocfft_plan_get_work_buffer_size(p.fwd, &w1);
    rocfft_plan_get_work_buffer_size(p.inv, &w2);
    p.work = w1 > w2 ? w1 : w2;
    it = g_fft_c2c.emplace(key, p).first;
  }
  if (work_bytes) *work_bytes = it->second.work;
  if (fwd) *fwd = it->second.fwd;
  if (inv) *inv = it->second.inv;
  return REXII_OK;
}

rexii_status fft_execute(void* plan, void* in, void* out, void* work, size_t work_bytes, hipStream_t s) {
  rocfft_execution_info info = nullptr;
  rocfft_status st = rocfft_execution_info_create(&info);
  if (st != rocfft_status_success) return set_error(REXII_ERR_HIP, fft_msg("rocfft_execution_info_create", st));
  st = rocfft_execution_info_set_stream(info, s);
  if (st == rocfft_status_success && work_bytes > 0) st = rocfft_execution_info_set_work_buffer(info, work, work_bytes);
  if (st == rocfft_status_success) {
    void* ib[1] = {in};
    void* ob[1] = {out};
    st = rocfft_execute(static_cast<rocfft_plan>(plan), ib, ob, info);
  }
  rocfft_execution_info_destroy(info);
  if (st != rocfft_status_success) return set_error(REXII_ERR_HIP, fft_msg("rocfft_execute", st));
  return REXII_OK;
}

// ---------------------------------------------------------------------------
// Static device scratch of rexii_apply_fourier_noalloc: one copy of this
// array per GPU, held until the process ends.  In host code its name is
// only a host-side stand-in; the device address comes from
// hipGetSymbolAddress (per device, with that device current) and only that
// address is handed to kernels and library calls.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[REXII_STATIC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch;  // device -> address of its copy of scratch
}  // namespace

rexii_status static_scratch(void** ptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(REXII_ERR_HIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return set_error(REXII_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    if (reinterpret_cast<uintptr_t>(p) & 255)
      return set_error(REXII_ERR_HIP, "static scratch is not 256-byte aligned");
    it = g_scratch.emplace(dev, p).first;
  }
  *ptr = it->second;
  return REXII_OK;
}

}  // namespace rexii
