// Preconditioned shifted solves for the flux-form (depth-field) operator.
//
// Each pole of the REXII sum needs (Sec. 4, the per-term systems, here as
// the height equation of the flux form)
//   K eta = (L_H + gamma C_H - zeta) eta = b,   b = sc (eta0 + a1 D_H + a2 Z_H).
// For a constant depth Hbar the operator L_Hbar - zeta is diagonal in
// Fourier space (the cross term C vanishes: centred differences commute),
// symbol -Hbar (s_x^2 + s_y^2) - zeta.  With the mean depth it is a
// preconditioner for the depth field; its shift is damped,
//   sigma = zeta + i beta |Re zeta| sign(Im zeta),  beta = 0.3,
// which keeps it bounded for the resonant poles (the shift inside the
// Laplacian's spectrum; undamped, the preconditioned iteration diverged at
// t rho = 5000 in the CPU/GPU prototype).  BiCGStab right-preconditioned:
//   p = r + beta (p - omega v);  ph = M^{-1} p;  v = K ph;  alpha = rho / <rh, v>
//   s = r - alpha v;  sh = M^{-1} s;  t = K sh;  omega = <t, s> / <t, t>
//   x += alpha ph + omega sh;  r = s - omega t;  rho' = <rh, r>
// with <a, b> = sum conj(a) b.  M^{-1} is a forward FFT (batch of the
// slots), a scale per mode and an inverse FFT.  Every vector kernel runs on
// all B slots (gridDim.y) and skips slots that are not iterating; the
// scalars of each slot come from block partial sums added in a fixed order
// by one block per slot (deterministic).
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "precond.h"

namespace rexii {

constexpr int kPcNT = 256;
constexpr int kPcBlocks = 256;   // blocks per slot of the vector kernels
constexpr int kPcParts = 8;      // doubles of partial sums per block

int pc_blocks() { return kPcBlocks; }

__device__ __forceinline__ double2 pc_ld2(const double2* p) { return uni(ldc(p)); }

// Sum of K values over the block (valid in thread 0), fixed order.
template <int K>
__device__ __forceinline__ void pc_block_sum(double (&v)[K], double* sh) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double a = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    v[k] = a;
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = 0.0;
      for (int q = 0; q < kPcNT / 64; ++q) a += sh[q * K + k];
      v[k] = a;
    }
}

__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// conj(a) b accumulated
__device__ __forceinline__ void c_dot(double& re, double& im, double2 a, double2 b) {
  re += a.x * b.x + a.y * b.y;
  im += a.x * b.y - a.y * b.x;
}

// b at point i of the problem for the slot's coefficients
__device__ __forceinline__ double2 pc_rhs(const PcProb& pb, size_t i, double2 sc, double2 a1, double2 a2) {
  double2 q = make_double2(pb.eta0[i], 0.0);
  if (pb.D0) {
    const double d = pb.D0[i], z = pb.Z0[i];
    q.x += a1.x * d + a2.x * z;
    q.y += a1.y * d + a2.y * z;
  }
  return c_mul(sc, q);
}

// K phi at (i, j) of one slot's field (periodic), the flux form of the
// slot engine's operator: cx [H_{i+1}(phi_{i+2} - phi_i) - H_{i-1}(phi_i - phi_{i-2})]
// + (y likewise) + gamma cxy [...] - zeta phi.
__device__ __forceinline__ double2 pc_kop(const double2* P, const PcProb& pb, int i, int j, double2 gamma,
                                          double2 zeta) {
  const int nx = pb.nx, ny = pb.ny;
  auto wx = [&](int a) { return a < 0 ? a + nx : (a >= nx ? a - nx : a); };
  auto wy = [&](int a) { return a < 0 ? a + ny : (a >= ny ? a - ny : a); };
  const size_t r0 = size_t(j) * nx, rn = size_t(wy(j + 1)) * nx, rs = size_t(wy(j - 1)) * nx;
  const size_t rnn = size_t(wy(j + 2)) * nx, rss = size_t(wy(j - 2)) * nx;
  const int ie = wx(i + 1), iw = wx(i - 1), iee = wx(i + 2), iww = wx(i - 2);
  const double2 c = P[r0 + i];
  const double2 e = P[r0 + iee], w = P[r0 + iww], n = P[rnn + i], s = P[rss + i];
  const double2 ne = P[rn + ie], nw = P[rn + iw], se = P[rs + ie], sw = P[rs + iw];
  const double* H = pb.H;
  const double hxp = H[r0 + ie], hxm = H[r0 + iw], hyp = H[rn + i], hym = H[rs + i];
  double2 lh, ch;
  lh.x = pb.cx * (hxp * (e.x - c.x) - hxm * (c.x - w.x)) + pb.cy * (hyp * (n.x - c.x) - hym * (c.x - s.x));
  lh.y = pb.cx * (hxp * (e.y - c.y) - hxm * (c.y - w.y)) + pb.cy * (hyp * (n.y - c.y) - hym * (c.y - s.y));
  ch.x = pb.cxy * (hxp * (ne.x - se.x) - hxm * (nw.x - sw.x) - hyp * (ne.x - nw.x) + hym * (se.x - sw.x));
  ch.y = pb.cxy * (hxp * (ne.y - se.y) - hxm * (nw.y - sw.y) - hyp * (ne.y - nw.y) + hym * (se.y - sw.y));
  return c_sub(c_add(lh, c_mul(gamma, ch)), c_mul(zeta, c));
}

#define PC_SLOT_LOOP                                                      \
  const int b = blockIdx.y;                                               \
  const size_t n = size_t(pb.nx) * pb.ny;                                 \
  const size_t base = size_t(b) * n;                                      \
  const size_t stride = size_t(gridDim.x) * kPcNT;

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPcNT) void k_pc_dir(PcVec w, PcProb pb) {
  __shared__ double sh[(kPcNT / 64) * 2];
  PC_SLOT_LOOP
  const int st = ldu(&w.slots[b].state);
  if (st != kPcIter && st != kPcStart) return;
  double acc[2] = {0.0, 0.0};
  if (st == kPcStart) {
    const double2 sc = pc_ld2(&w.slots[b].sc), a1 = pc_ld2(&w.slots[b].a1), a2 = pc_ld2(&w.slots[b].a2);
    for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += stride) {
      const double2 q = pc_rhs(pb, i, sc, a1, a2);
      w.x[base + i] = make_double2(0.0, 0.0);
      w.r[base + i] = q;
      w.rh[base + i] = q;
      w.p[base + i] = q;
      w.ph[base + i] = q;
      w.v[base + i] = make_double2(0.0, 0.0);
      acc[0] += q.x * q.x + q.y * q.y;
    }
  } else {
    const double2 beta = pc_ld2(&w.slots[b].beta), omega = pc_ld2(&w.slots[b].omega);
    for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += stride) {
      const double2 pv = c_add(w.r[base + i], c_mul(beta, c_sub(w.p[base + i], c_mul(omega, w.v[base + i]))));
      w.p[base + i] = pv;
      w.ph[base + i] = pv;
    }
  }
  pc_block_sum(acc, sh);
  if (threadIdx.x == 0 && st == kPcStart) {
    double* pp = w.part + (size_t(b) * kPcBlocks + blockIdx.x) * kPcParts;
    pp[0] = acc[0];
    pp[1] = 0.0;
  }
}

// vec *= 1 / (n (-hbar (s_x^2 + s_y^2) - sigma)) per mode of the full spectrum
__global__ __launch_bounds__(kPcNT) void k_pc_scale(double2* vec, PcVec w, PcProb pb) {
  PC_SLOT_LOOP
  const int st = ldu(&w.slots[b].state);
  if (st != kPcIter && st != kPcStart) return;
  const double2 sg = pc_ld2(&w.slots[b].sigma);
  const double inv_n = 1.0 / double(n);
  const double* sy = pb.sx + (pb.nx / 2 + 1);
  for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += stride) {
    const int kx = int(i % size_t(pb.nx)), ky = int(i / size_t(pb.nx));
    const double sxv = pb.sx[kx <= pb.nx / 2 ? kx : pb.nx - kx], syv = sy[ky];
    const double dr = -pb.hbar * (sxv * sxv + syv * syv) - sg.x, di = -sg.y;
    const double m = inv_n / (dr * dr + di * di);
    const double2 q = vec[base + i];
    // q / (dr + i di) = q (dr - i di) / |d|^2
    vec[base + i] = make_double2((q.x * dr + q.y * di) * m, (q.y * dr - q.x * di) * m);
  }
}

// out = K in; which 0: <rh, out> -> part[2..3]; which 1: <out, s>, |out|^2 -> part[4..6]
__global__ __launch_bounds__(kPcNT) void k_pc_matvec(const double2* in, double2* out, int which, PcVec w, PcProb pb) {
  __shared__ double sh[(kPcNT / 64) * 3];
  PC_SLOT_LOOP
  const int st = ldu(&w.slots[b].state);
  if (st != kPcIter && st != kPcStart) return;
  const double2 gamma = pc_ld2(&w.slots[b].gamma), zeta = pc_ld2(&w.slots[b].zeta);
  double acc[3] = {0.0, 0.0, 0.0};
  for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += stride) {
    const int x = int(i % size_t(pb.nx)), y = int(i / size_t(pb.nx));
    const double2 q = pc_kop(in + base, pb, x, y, gamma, zeta);
    out[base + i] = q;
    if (which == 0) {
      c_dot(acc[0], acc[1], w.rh[base + i], q);
    } else {
      c_dot(acc[0], acc[1], q, w.r[base + i]);
      acc[2] += q.x * q.x + q.y * q.y;
    }
  }
  pc_block_sum(acc, sh);
  if (threadIdx.x == 0) {
    double* pp = w.part + (size_t(b) * kPcBlocks + blockIdx.x) * kPcParts;
    if (which == 0) {
      pp[2] = acc[0];
      pp[3] = acc[1];
    } else {
      pp[4] = acc[0];
      pp[5] = acc[1];
      pp[6] = acc[2];
    }
  }
}

// s = r - alpha v (into r), sh = s
__global__ __launch_bounds__(kPcNT) void k_pc_s(PcVec w, PcProb pb) {
  PC_SLOT_LOOP
  const int st = ldu(&w.slots[b].state);
  if (st != kPcIter) return;
  const double2 alpha = pc_ld2(&w.slots[b].alpha);
  for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += stride) {
    const double2 sv = c_sub(w.r[base + i], c_mul(alpha, w.v[base + i]));
    w.r[base + i] = sv;
    w.sh[base + i] = sv;
  }
}

// x += alpha ph + omega sh, r = s - omega t (s is in r); partials <rh, r>, |r|^2
__global__ __launch_bounds__(kPcNT) void k_pc_xr(PcVec w, PcProb pb) {
  __shared__ double sh[(kPcNT / 64) * 3];
  PC_SLOT_LOOP
  const int st = ldu(&w.slots[b].state);
  if (st != kPcIter) return;
  const double2 alpha = pc_ld2(&w.slots[b].alpha), omega = pc_ld2(&w.slots[b].omega);
  double acc[3] = {0.0, 0.0, 0.0};
  for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += stride) {
    w.x[base + i] = c_add(w.x[base + i], c_add(c_mul(alpha, w.ph[base + i]), c_mul(omega, w.sh[base + i])));
    const double2 rv = c_sub(w.r[base + i], c_mul(omega, w.t[base + i]));
    w.r[base + i] = rv;
    c_dot(acc[0], acc[1], w.rh[base + i], rv);
    acc[2] += rv.x * rv.x + rv.y * rv.y;
  }
  pc_block_sum(acc, sh);
  if (threadIdx.x == 0) {
    double* pp = w.part + (size_t(b) * kPcBlocks + blockIdx.x) * kPcParts;
    pp[0] = acc[0];
    pp[1] = acc[1];
    pp[7] = acc[2];
  }
}

__device__ __forceinline__ bool c_ok(double2 a) { return isfinite(a.x) && isfinite(a.y) && (a.x != 0.0 || a.y != 0.0); }
__device__ __forceinline__ double2 c_div(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// One block per slot: the partials of the slot added in block order, then
// the scalars of the stage.
__global__ __launch_bounds__(kPcNT) void k_pc_scalars(PcVec w, int stage) {
  __shared__ double sh[(kPcNT / 64) * 4];
  const int b = blockIdx.x;
  PcSlot* S = w.slots + b;
  const int st = ldu(&S->state);
  const bool live = (st == kPcIter) || (stage <= 1 && st == kPcStart);
  if (!live) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < kPcBlocks; q += kPcNT) {
    const double* pp = w.part + (size_t(b) * kPcBlocks + q) * kPcParts;
    if (stage == 0) {
      acc[0] += pp[0];
    } else if (stage == 1) {
      acc[0] += pp[2];
      acc[1] += pp[3];
    } else if (stage == 2) {
      acc[0] += pp[4];
      acc[1] += pp[5];
      acc[2] += pp[6];
    } else {
      acc[0] += pp[0];
      acc[1] += pp[1];
      acc[2] += pp[7];
    }
  }
  pc_block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  if (stage == 0) {
    if (st != kPcStart) return;
    S->rho = make_double2(acc[0], 0.0);   // <b, b>
    S->bn2 = acc[0];
    S->rn2 = acc[0];
    S->it = 0;
    const double ref2 = ldc(&S->ref2);
    const double stop2 = ldc(&S->tol2) * (ref2 > 0.0 ? ref2 : acc[0]);
    S->stop2 = stop2;
    if (!(acc[0] <= stop2)) {
      S->state = kPcIter;     // alpha follows from <rh, v> at stage 1
    } else {
      S->state = kPcConv;     // b is (close to) zero: x = 0
    }
    return;
  }
  if (stage == 1) {
    const double2 rv = make_double2(acc[0], acc[1]);
    const double2 al = c_div(ldc(&S->rho), rv);
    if (!c_ok(rv) || !c_ok(al)) {
      S->state = kPcBreak;
      return;
    }
    S->alpha = al;
    if (st == kPcStart) S->state = kPcIter;
    return;
  }
  if (stage == 2) {
    const double tt = acc[2];
    const double2 om = make_double2(acc[0] / tt, acc[1] / tt);
    if (!(tt > 0.0) || !c_ok(om)) {
      S->state = kPcBreak;
      return;
    }
    S->omega = om;
    return;
  }
  // stage 3: new rho, beta, residual, stop test, cap
  const double2 rho1 = make_double2(acc[0], acc[1]);
  const double2 be = c_mul(c_div(rho1, ldc(&S->rho)), c_div(ldc(&S->alpha), ldc(&S->omega)));
  const int it = ldc(&S->it) + 1;
  S->rn2 = acc[2];
  S->it = it;
  if (acc[2] <= ldc(&S->stop2)) {
    S->state = kPcConv;
  } else if (!c_ok(rho1) || !c_ok(be) || !isfinite(acc[2])) {
    S->state = kPcBreak;
  } else if (it >= ldc(&S->max_it)) {
    S->state = kPcCap;
  }
  S->rho = rho1;
  S->beta = be;
}

// True residual of slots in state kPcConv / kPcCap: r = rh = p = b - K x, v = 0,
// partials <r, r> (part[0]).
__global__ __launch_bounds__(kPcNT) void k_pc_resid(PcVec w, PcProb pb) {
  __shared__ double sh[(kPcNT / 64) * 1];
  PC_SLOT_LOOP
  const int st = ldu(&w.slots[b].state);
  if (st != kPcConv && st != kPcCap && st != kPcBreak) return;
  const double2 gamma = pc_ld2(&w.slots[b].gamma), zeta = pc_ld2(&w.slots[b].zeta);
  const double2 sc = pc_ld2(&w.slots[b].sc), a1 = pc_ld2(&w.slots[b].a1), a2 = pc_ld2(&w.slots[b].a2);
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += stride) {
    const int x = int(i % size_t(pb.nx)), y = int(i / size_t(pb.nx));
    const double2 q = c_sub(pc_rhs(pb, i, sc, a1, a2), pc_kop(w.x + base, pb, x, y, gamma, zeta));
    w.r[base + i] = q;
    w.rh[base + i] = q;
    w.p[base + i] = q;
    w.v[base + i] = make_double2(0.0, 0.0);
    acc[0] += q.x * q.x + q.y * q.y;
  }
  pc_block_sum(acc, sh);
  if (threadIdx.x == 0) {
    double* pp = w.part + (size_t(b) * kPcBlocks + blockIdx.x) * kPcParts;
    pp[0] = acc[0];
  }
}

// After k_pc_resid: rn2 = |r|^2 of the true residual, rho = <rh, r> = rn2
// (one block per slot; the state is left for the host to decide).
__global__ __launch_bounds__(kPcNT) void k_pc_resid_sum(PcVec w) {
  __shared__ double sh[(kPcNT / 64) * 1];
  const int b = blockIdx.x;
  PcSlot* S = w.slots + b;
  const int st = ldu(&S->state);
  if (st != kPcConv && st != kPcCap && st != kPcBreak) return;
  double acc[1] = {0.0};
  for (int q = threadIdx.x; q < kPcBlocks; q += kPcNT) acc[0] += w.part[(size_t(b) * kPcBlocks + q) * kPcParts];
  pc_block_sum(acc, sh);
  if (threadIdx.x == 0) {
    S->rn2 = acc[0];
    S->rho = make_double2(acc[0], 0.0);
    S->beta = make_double2(0.0, 0.0);
    S->omega = make_double2(1.0, 0.0);
  }
}

// A_j += Re(c_j x) for one slot
__global__ __launch_bounds__(kPcNT) void k_pc_accum(const double2* x, double2 c0, double2 c1, double2 c2, double* A,
                                                    size_t n) {
  for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += size_t(gridDim.x) * kPcNT) {
    const double2 v = x[i];
    A[i] += c0.x * v.x - c0.y * v.y;
    A[n + i] += c1.x * v.x - c1.y * v.y;
    A[2 * n + i] += c2.x * v.x - c2.y * v.y;
  }
}

__global__ __launch_bounds__(kPcNT) void k_pc_sum(const double* H, size_t n, double* part) {
  __shared__ double sh[(kPcNT / 64) * 1];
  double acc[1] = {0.0};
  for (size_t i = blockIdx.x * size_t(kPcNT) + threadIdx.x; i < n; i += size_t(gridDim.x) * kPcNT) acc[0] += H[i];
  pc_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// ---------------------------------------------------------------------------
void launch_pc_dir(const PcVec& w, const PcProb& pb, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_dir, dim3(kPcBlocks, w.B), dim3(kPcNT), 0, s, w, pb);
}
void launch_pc_scale(double2* vec, const PcVec& w, const PcProb& pb, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_scale, dim3(kPcBlocks, w.B), dim3(kPcNT), 0, s, vec, w, pb);
}
void launch_pc_matvec(const double2* in, double2* out, int which, const PcVec& w, const PcProb& pb, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_matvec, dim3(kPcBlocks, w.B), dim3(kPcNT), 0, s, in, out, which, w, pb);
}
void launch_pc_s(const PcVec& w, const PcProb& pb, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_s, dim3(kPcBlocks, w.B), dim3(kPcNT), 0, s, w, pb);
}
void launch_pc_xr(const PcVec& w, const PcProb& pb, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_xr, dim3(kPcBlocks, w.B), dim3(kPcNT), 0, s, w, pb);
}
void launch_pc_scalars(const PcVec& w, int stage, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_scalars, dim3(w.B), dim3(kPcNT), 0, s, w, stage);
}
void launch_pc_resid(const PcVec& w, const PcProb& pb, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_resid, dim3(kPcBlocks, w.B), dim3(kPcNT), 0, s, w, pb);
  hipLaunchKernelGGL(k_pc_resid_sum, dim3(w.B), dim3(kPcNT), 0, s, w);
}
void launch_pc_accum(const PcVec& w, int slot, double2 c0, double2 c1, double2 c2, double* A, const PcProb& pb,
                     hipStream_t s) {
  const size_t n = size_t(pb.nx) * pb.ny;
  hipLaunchKernelGGL(k_pc_accum, dim3(1024), dim3(kPcNT), 0, s, w.x + size_t(slot) * n, c0, c1, c2, A, n);
}
void launch_pc_sum(const double* H, size_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_sum, dim3(kPcBlocks), dim3(kPcNT), 0, s, H, n, part);
}

}  // namespace rexii
