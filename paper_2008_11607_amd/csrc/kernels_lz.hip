// Shared-Krylov (multi-shift) REXII: every shifted system of the pole sum
// is (tA - z_k I) x_k = f with the same right-hand side, and Krylov spaces
// are shift invariant, K_m(tA - z I, f) = K_m(A, f).  One Lanczos process
// therefore serves all poles:
//   A V_m = V_m T_m + beta_m v_{m+1} e_m^T,
//   r(tA) f ~ ||f||_W V_m Re sum_k w_k (t T_m - z_k I)^{-1} e_1.
// With W = diag(g, H, H) the operator (any depth field, flux form) satisfies
// W A = -(W A)^T, so A is skew-adjoint in <x, y>_W = x^T W y: the Lanczos
// recurrence has no diagonal term and is real,
//   w_j = A v_j + beta_{j-1} v_{j-1},  beta_j = ||w_j||_W,  v_{j+1} = w_j / beta_j,
// and T_m is real skew-tridiagonal (T[j+1][j] = beta_j = -T[j][j+1]).
//
// Two passes over the same recurrence avoid keeping the m basis vectors:
// pass 1 yields beta_1..beta_m (and the host solves the small problems),
// pass 2 repeats the identical steps and accumulates u += y_j v_j.  The
// reductions are in a fixed order, so pass 2 reproduces pass 1 bit for bit.
//
// Storage: the vectors are kept unnormalised, buf_j = beta_{j-1} v_j
// (buf_1 = f, beta_0 = ||f||_W), in two buffers that alternate; step j
// reads buf_j and buf_{j-1} and overwrites buf_{j-1} with w_j = buf_{j+1}.
#include <hip/hip_runtime.h>

#include "kernels_lz.h"

namespace rexii {

constexpr int kLzTX = 64;   // tile columns (one per lane)
constexpr int kLzRows = 8;  // rows per thread (a sliding window of three rows)
constexpr int kLzNT = 256;  // threads: 64 x 4
constexpr int kLzTY = kLzRows * (kLzNT / kLzTX);  // 32 rows per tile

__device__ __forceinline__ double block_sum_lz(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kLzNT / 64; ++k) s += sh[k];
  return s;  // valid in thread 0
}

// One Lanczos step for every state r (blockIdx.y) of the batch.
//   cur = buf_j, prev = buf_{j-1} (overwritten with w_j).
//   beta[r * ldb + j - 1] = beta_{j-1} (beta_0 = ||f||_W), beta[.. + j - 2].
//   j == 1: no prev term (prev is not read).
//   part[r * nblk + block] = this block's sum of g w_eta^2 + H (w_u^2 + w_v^2)
//     (skipped when part == nullptr).
//   y != nullptr (pass 2): u += (y[r * ldy + j - 1] / beta_{j-1}) buf_j.
//   last: pass 2's final step (w_m is not needed: prev is left alone).
__global__ __launch_bounds__(kLzNT) void k_lz_step(const double* __restrict__ cur, double* __restrict__ prev,
                                                   const double* __restrict__ H, double H0, double g, double fc,
                                                   int nx, int ny, int j, const double* __restrict__ beta, int ldb,
                                                   double* __restrict__ part, const double* __restrict__ y, int ldy,
                                                   double* __restrict__ u, int last) {
  __shared__ double sh[kLzNT / 64];
  const int r = blockIdx.y;
  const size_t n = size_t(nx) * ny;
  const double* c = cur + size_t(r) * 3 * n;
  double* pv = prev + size_t(r) * 3 * n;
  const double* br = beta + size_t(r) * ldb;
  const double sc = 1.0 / br[j - 1];                                  // v_j = sc * buf_j
  const double sp = (j >= 2) ? br[j - 1] / br[j - 2] : 0.0;          // beta_{j-1} v_{j-1} = sp * buf_{j-1}
  const double yv = y ? y[size_t(r) * ldy + j - 1] : 0.0;
  const double yc = (yv != 0.0) ? yv * sc : 0.0;  // a zero state has beta_0 = 0 and y = 0
  double* ur = u ? u + size_t(r) * 3 * n : nullptr;
  const int tiles_x = (nx + kLzTX - 1) / kLzTX;
  const int i = (blockIdx.x % tiles_x) * kLzTX + (threadIdx.x & 63);
  const int j0 = (blockIdx.x / tiles_x) * kLzTY + (threadIdx.x >> 6) * kLzRows;
  const double hx = 0.5 * nx, hy = 0.5 * ny;
  double acc = 0.0;
  if (i < nx && j0 < ny) {
    const int ie = (i + 1 == nx) ? 0 : i + 1, iw = (i == 0) ? nx - 1 : i - 1;
    const double* ce = c;
    const double* cu = c + n;
    const double* cv = c + 2 * n;
    // rows jj - 1, jj, jj + 1 of eta, v and the depth in registers: each
    // row is loaded once per thread and slides down the window
    auto row = [&](int jj) { return size_t(jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj)) * nx + i; };
    const size_t q0 = row(j0 - 1), q1 = row(j0);
    double eS = ce[q0], eC = ce[q1], vS = cv[q0], vC = cv[q1];
    double HS = H ? H[q0] : H0, HC = H ? H[q1] : H0;
    for (int k = 0; k < kLzRows; ++k) {
      const int jj = j0 + k;
      if (jj >= ny) break;
      const size_t p = size_t(jj) * nx + i, qn = row(jj + 1);
      const size_t pe = size_t(jj) * nx + ie, pw = size_t(jj) * nx + iw;
      const double eN = ce[qn], vN = cv[qn], HN = H ? H[qn] : H0;
      const double He = H ? H[pe] : H0, Hw = H ? H[pw] : H0;
      const double b0 = eC, b1 = cu[p], b2 = vC;
      // A buf_j (flux form, centred differences)
      const double ae = -(hx * (He * cu[pe] - Hw * cu[pw]) + hy * (HN * vN - HS * vS));
      const double au = -g * hx * (ce[pe] - ce[pw]) + fc * b2;
      const double av = -g * hy * (eN - eS) - fc * b1;
      if (ur && yc != 0.0) {  // y_j = 0 beyond a state's own Krylov dimension
        ur[p] += yc * b0;
        ur[n + p] += yc * b1;
        ur[2 * n + p] += yc * b2;
      }
      if (!last) {
        double w0 = sc * ae, w1 = sc * au, w2 = sc * av;
        if (j >= 2) {
          w0 += sp * pv[p];
          w1 += sp * pv[n + p];
          w2 += sp * pv[2 * n + p];
        }
        pv[p] = w0;
        pv[n + p] = w1;
        pv[2 * n + p] = w2;
        acc += g * w0 * w0 + HC * (w1 * w1 + w2 * w2);
      }
      eS = eC;
      eC = eN;
      vS = vC;
      vC = vN;
      HS = HC;
      HC = HN;
    }
  }
  if (!part) return;
  const double s = block_sum_lz(acc, sh);
  if (threadIdx.x == 0) part[size_t(r) * gridDim.x + blockIdx.x] = s;
}

// ||f||_W partial sums of each state (for beta_0), and buf_1 = f.
__global__ __launch_bounds__(kLzNT) void k_lz_start(const double* __restrict__ f, double* __restrict__ buf,
                                                    const double* __restrict__ H, double H0, double g, int nx,
                                                    int ny, double* __restrict__ part, int* __restrict__ flag) {
  __shared__ double sh[kLzNT / 64];
  const int r = blockIdx.y;
  const size_t n = size_t(nx) * ny;
  const double* fr = f + size_t(r) * 3 * n;
  double* br = buf + size_t(r) * 3 * n;
  const int tiles_x = (nx + kLzTX - 1) / kLzTX;
  const int i = (blockIdx.x % tiles_x) * kLzTX + (threadIdx.x & 63);
  const int j0 = (blockIdx.x / tiles_x) * kLzTY + (threadIdx.x >> 6) * kLzRows;
  double acc = 0.0;
  bool bad = false;
  if (i < nx) {
    for (int k = 0; k < kLzRows; ++k) {
      const int jj = j0 + k;
      if (jj >= ny) break;
      const size_t p = size_t(jj) * nx + i;
      const double a = fr[p], b = fr[n + p], c = fr[2 * n + p];
      br[p] = a;
      br[n + p] = b;
      br[2 * n + p] = c;
      const double Hp = H ? H[p] : H0;
      acc += g * a * a + Hp * (b * b + c * c);
      bad = bad || !isfinite(a) || !isfinite(b) || !isfinite(c);
    }
  }
  if (bad) atomicOr(flag, 1);
  const double s = block_sum_lz(acc, sh);
  if (threadIdx.x == 0) part[size_t(r) * gridDim.x + blockIdx.x] = s;
}

// beta[r * ldb + slot] = sqrt(sum of part[r][0..nblk)) in a fixed order
// (one block per state).
__global__ __launch_bounds__(kLzNT) void k_lz_norm(const double* __restrict__ part, int nblk,
                                                   double* __restrict__ beta, int ldb, int slot) {
  __shared__ double sh[kLzNT / 64];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kLzNT) s += part[size_t(r) * nblk + k];
  s = block_sum_lz(s, sh);
  if (threadIdx.x == 0) beta[size_t(r) * ldb + slot] = sqrt(s);
}

int lz_blocks(int nx, int ny) { return ((nx + kLzTX - 1) / kLzTX) * ((ny + kLzTY - 1) / kLzTY); }

void launch_lz_start(const double* f, double* buf, const double* H, double H0, double g, int nx, int ny, int nrhs,
                     double* part, int* flag, double* beta, int ldb, hipStream_t s) {
  const int nb = lz_blocks(nx, ny);
  hipLaunchKernelGGL(k_lz_start, dim3(nb, nrhs), dim3(kLzNT), 0, s, f, buf, H, H0, g, nx, ny, part, flag);
  hipLaunchKernelGGL(k_lz_norm, dim3(nrhs), dim3(kLzNT), 0, s, part, nb, beta, ldb, 0);
}

void launch_lz_step(const double* cur, double* prev, const double* H, double H0, double g, double fc, int nx, int ny,
                    int nrhs, int j, double* beta, int ldb, double* part, const double* y, int ldy, double* u,
                    int last, hipStream_t s) {
  const int nb = lz_blocks(nx, ny);
  hipLaunchKernelGGL(k_lz_step, dim3(nb, nrhs), dim3(kLzNT), 0, s, cur, prev, H, H0, g, fc, nx, ny, j, beta, ldb,
                     part, y, ldy, u, last);
  if (part) hipLaunchKernelGGL(k_lz_norm, dim3(nrhs), dim3(kLzNT), 0, s, part, nb, beta, ldb, j);
}

}  // namespace rexii
