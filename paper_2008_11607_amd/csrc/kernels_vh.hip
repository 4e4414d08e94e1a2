// Variable-depth (flux form) shifted solves: BiCGStab on
//   K eta = (L_H + gamma C_H - zeta) eta = b        (see kernels.h)
// for every live slot, three passes per iteration, each followed by a
// one-block-per-slot scalar kernel (deterministic partial sums):
//   A: p = r + beta (p - omega v)  (p = r on the first iteration),  v = K p,
//      partial <r_hat, v>                       -> alpha = rho / <r_hat, v>
//   B: s = r - alpha v,  t = K s,  partials <t, s>, <t, t>
//                                               -> omega = <t, s> / <t, t>
//   C: s, t again,  x += alpha p + omega s,  r = s - omega t,
//      partials <r_hat, r>, |r|^2               -> beta = (rho'/rho)(alpha/omega)
// <a, b> = sum conj(a) b.  r, p, v are ping-pong buffers so that no pass
// reads (with a halo) what it writes.  The FP64 residual / refinement loop
// around the inner solve is shared with the COCG path (k_outer_update) plus
// the variable-coefficient residual below.
#include "device_util.h"
#include "kernels.h"

namespace rexii {

constexpr int kVW = kTX + 4, kVH = kTY + 4;   // field tile with halo 2
constexpr int kHW = kTX + 2, kHH = kTY + 2;   // depth tile with halo 1

// K phi at interior position (ly, lx) of a tile: phi tile with halo 2
// (row width kVW), depth tile with halo 1 (row width kHW).
template <typename V, typename S>
__device__ __forceinline__ V kop(const V* P, const S* Hs, int ly, int lx, S cx, S cy, S cxy, V gamma, V zeta) {
  const int y = ly + 2, x = lx + 2;
  const V c = P[y * kVW + x];
  const V e = P[y * kVW + x + 2], w = P[y * kVW + x - 2];
  const V n = P[(y + 2) * kVW + x], s = P[(y - 2) * kVW + x];
  const V ne = P[(y + 1) * kVW + x + 1], nw = P[(y + 1) * kVW + x - 1];
  const V se = P[(y - 1) * kVW + x + 1], sw = P[(y - 1) * kVW + x - 1];
  const S hxp = Hs[(ly + 1) * kHW + lx + 2], hxm = Hs[(ly + 1) * kHW + lx];
  const S hyp = Hs[(ly + 2) * kHW + lx + 1], hym = Hs[ly * kHW + lx + 1];
  V lh, ch;
  lh.x = cx * (hxp * (e.x - c.x) - hxm * (c.x - w.x)) + cy * (hyp * (n.x - c.x) - hym * (c.x - s.x));
  lh.y = cx * (hxp * (e.y - c.y) - hxm * (c.y - w.y)) + cy * (hyp * (n.y - c.y) - hym * (c.y - s.y));
  ch.x = cxy * (hxp * (ne.x - se.x) - hxm * (nw.x - sw.x) - hyp * (ne.x - nw.x) + hym * (se.x - sw.x));
  ch.y = cxy * (hxp * (ne.y - se.y) - hxm * (nw.y - sw.y) - hyp * (ne.y - nw.y) + hym * (se.y - sw.y));
  V q;
  q.x = lh.x + (gamma.x * ch.x - gamma.y * ch.y) - (zeta.x * c.x - zeta.y * c.y);
  q.y = lh.y + (gamma.x * ch.y + gamma.y * ch.x) - (zeta.x * c.y + zeta.y * c.x);
  return q;
}

template <typename T>
__device__ __forceinline__ void load_depth(T* Hs, const double* H, int x0, int y0, const Inst& I, bool big) {
  for (int k = threadIdx.x; k < kHH * kHW; k += kNT) {
    const int ly = k / kHW, lx = k - ly * kHW;
    Hs[k] = T(H[size_t(wrapc(y0 - 1 + ly, I.ny, big)) * I.nx + wrapc(x0 - 1 + lx, I.nx, big)]);
  }
}

struct SlotView {
  int slot, par;
  bool first;
  double2 alpha, beta, omega, gamma, zeta;
};

// Resolves work item w of the pass; returns false if the block has nothing
// to do for it (uniform across the block).
__device__ __forceinline__ bool bcg_item(const Eng& e, int w, int per, int total, int un, Item& it, SlotView& sv,
                                         Inst& I) {
  const int pos = xcd_pos(w, per);
  if (pos >= total) return false;
  it = item_of(e, pos, un);
  const Slot* S = &e.slots[it.slot];
  if (ldc(&S->status) != kInner) return false;
  I = ld_inst(&e.inst[ldc(&S->inst)]);
  sv.slot = it.slot;
  sv.par = ldc(&S->parity);
  sv.first = ldc(&S->prime) != 0;
  sv.alpha = ldc(&S->alpha);
  sv.beta = ldc(&S->beta);
  sv.omega = ldc(&S->omega);
  sv.gamma = ldc(&S->gamma);
  sv.zeta = ldc(&S->zeta);
  return true;
}

// ---- pass A ----------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_bcg_a(Eng e) {
  using V = typename C2<T>::t;
  __shared__ V PT[kVH * kVW];
  __shared__ T Hs[kHH * kHW];
  __shared__ double red[4 * 2];
  const int total = ldc(&e.tile_start[e.B]);
  const int un = ldc(&e.work[1]);
  const int per = (total + 7) >> 3;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int w = blockIdx.x; w < 8 * per; w += gridDim.x) {
    Item it;
    SlotView sv;
    Inst I;
    if (!bcg_item(e, w, per, total, un, it, sv, I)) continue;
    const size_t base = size_t(it.slot) * e.cap;
    const V* rs = reinterpret_cast<const V*>(sv.par ? e.r1 : e.r0) + base;
    const V* ps = reinterpret_cast<const V*>(sv.par ? e.p1 : e.p0) + base;
    const V* vs = reinterpret_cast<const V*>(sv.par ? e.v1 : e.v0) + base;
    V* pd = reinterpret_cast<V*>(sv.par ? e.p0 : e.p1) + base;
    V* vd = reinterpret_cast<V*>(sv.par ? e.v0 : e.v1) + base;
    const V* rh = reinterpret_cast<const V*>(e.rh) + base;
    const V beta = mk<V>(sv.beta.x, sv.beta.y), omega = mk<V>(sv.omega.x, sv.omega.y);
    const V gamma = mk<V>(sv.gamma.x, sv.gamma.y), zeta = mk<V>(sv.zeta.x, sv.zeta.y);
    const int x0 = (it.tile % I.tiles_x) * kTX, y0 = (it.tile / I.tiles_x) * kTY;
    const bool big = (I.nx >= kVW) && (I.ny >= kVH);
    __syncthreads();
    for (int k = threadIdx.x; k < kVH * kVW; k += kNT) {
      const int ly = k / kVW, lx = k - ly * kVW;
      const size_t gi = size_t(wrapc(y0 - 2 + ly, I.ny, big)) * I.nx + wrapc(x0 - 2 + lx, I.nx, big);
      V pn = rs[gi];
      if (!sv.first) pn = cadd(pn, cmul(beta, csub(ps[gi], cmul(omega, vs[gi]))));
      PT[k] = pn;
    }
    load_depth<T>(Hs, I.H, x0, y0, I, big);
    __syncthreads();
    double acc[2] = {0.0, 0.0};
    for (int j = 0; j < kTY / 4; ++j) {
      const int ly = ty + 4 * j;
      const int gx = x0 + tx, gy = y0 + ly;
      if (gx < I.nx && gy < I.ny) {
        const size_t gi = size_t(gy) * I.nx + gx;
        const V vn = kop<V, T>(PT, Hs, ly, tx, T(I.cx), T(I.cy), T(I.cxy), gamma, zeta);
        pd[gi] = PT[(ly + 2) * kVW + tx + 2];
        vd[gi] = vn;
        const V h = rh[gi];
        acc[0] += double(h.x) * vn.x + double(h.y) * vn.y;   // conj(h) vn
        acc[1] += double(h.x) * vn.y - double(h.y) * vn.x;
      }
    }
    double tot[2];
    block_sum_n<2>(acc, red, tot);
    if (threadIdx.x == 0) {
      double* pp = e.part + (size_t(it.slot) * e.cap_blk + it.tile) * kNDots;
      pp[0] = tot[0];
      pp[1] = tot[1];
    }
  }
}

// ---- pass B ----------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_bcg_b(Eng e) {
  using V = typename C2<T>::t;
  __shared__ V PT[kVH * kVW];
  __shared__ T Hs[kHH * kHW];
  __shared__ double red[4 * 3];
  const int total = ldc(&e.tile_start[e.B]);
  const int un = ldc(&e.work[1]);
  const int per = (total + 7) >> 3;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int w = blockIdx.x; w < 8 * per; w += gridDim.x) {
    Item it;
    SlotView sv;
    Inst I;
    if (!bcg_item(e, w, per, total, un, it, sv, I)) continue;
    const size_t base = size_t(it.slot) * e.cap;
    const V* rs = reinterpret_cast<const V*>(sv.par ? e.r1 : e.r0) + base;
    const V* vn = reinterpret_cast<const V*>(sv.par ? e.v0 : e.v1) + base;
    const V alpha = mk<V>(sv.alpha.x, sv.alpha.y);
    const V gamma = mk<V>(sv.gamma.x, sv.gamma.y), zeta = mk<V>(sv.zeta.x, sv.zeta.y);
    const int x0 = (it.tile % I.tiles_x) * kTX, y0 = (it.tile / I.tiles_x) * kTY;
    const bool big = (I.nx >= kVW) && (I.ny >= kVH);
    __syncthreads();
    for (int k = threadIdx.x; k < kVH * kVW; k += kNT) {
      const int ly = k / kVW, lx = k - ly * kVW;
      const size_t gi = size_t(wrapc(y0 - 2 + ly, I.ny, big)) * I.nx + wrapc(x0 - 2 + lx, I.nx, big);
      PT[k] = csub(rs[gi], cmul(alpha, vn[gi]));
    }
    load_depth<T>(Hs, I.H, x0, y0, I, big);
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < kTY / 4; ++j) {
      const int ly = ty + 4 * j;
      if (x0 + tx < I.nx && y0 + ly < I.ny) {
        const V t = kop<V, T>(PT, Hs, ly, tx, T(I.cx), T(I.cy), T(I.cxy), gamma, zeta);
        const V s = PT[(ly + 2) * kVW + tx + 2];
        acc[0] += double(t.x) * s.x + double(t.y) * s.y;   // conj(t) s
        acc[1] += double(t.x) * s.y - double(t.y) * s.x;
        acc[2] += double(t.x) * t.x + double(t.y) * t.y;
      }
    }
    double tot[3];
    block_sum_n<3>(acc, red, tot);
    if (threadIdx.x == 0) {
      double* pp = e.part + (size_t(it.slot) * e.cap_blk + it.tile) * kNDots;
      pp[0] = tot[0];
      pp[1] = tot[1];
      pp[2] = tot[2];
    }
  }
}

// ---- pass C ----------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_bcg_c(Eng e) {
  using V = typename C2<T>::t;
  __shared__ V PT[kVH * kVW];
  __shared__ T Hs[kHH * kHW];
  __shared__ double red[4 * 3];
  const int total = ldc(&e.tile_start[e.B]);
  const int un = ldc(&e.work[1]);
  const int per = (total + 7) >> 3;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int w = blockIdx.x; w < 8 * per; w += gridDim.x) {
    Item it;
    SlotView sv;
    Inst I;
    if (!bcg_item(e, w, per, total, un, it, sv, I)) continue;
    const size_t base = size_t(it.slot) * e.cap;
    const V* rs = reinterpret_cast<const V*>(sv.par ? e.r1 : e.r0) + base;
    V* rd = reinterpret_cast<V*>(sv.par ? e.r0 : e.r1) + base;
    const V* vn = reinterpret_cast<const V*>(sv.par ? e.v0 : e.v1) + base;
    const V* pn = reinterpret_cast<const V*>(sv.par ? e.p0 : e.p1) + base;
    const V* rh = reinterpret_cast<const V*>(e.rh) + base;
    V* d = reinterpret_cast<V*>(e.d) + base;
    const V alpha = mk<V>(sv.alpha.x, sv.alpha.y), omega = mk<V>(sv.omega.x, sv.omega.y);
    const V gamma = mk<V>(sv.gamma.x, sv.gamma.y), zeta = mk<V>(sv.zeta.x, sv.zeta.y);
    const int x0 = (it.tile % I.tiles_x) * kTX, y0 = (it.tile / I.tiles_x) * kTY;
    const bool big = (I.nx >= kVW) && (I.ny >= kVH);
    __syncthreads();
    for (int k = threadIdx.x; k < kVH * kVW; k += kNT) {
      const int ly = k / kVW, lx = k - ly * kVW;
      const size_t gi = size_t(wrapc(y0 - 2 + ly, I.ny, big)) * I.nx + wrapc(x0 - 2 + lx, I.nx, big);
      PT[k] = csub(rs[gi], cmul(alpha, vn[gi]));
    }
    load_depth<T>(Hs, I.H, x0, y0, I, big);
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < kTY / 4; ++j) {
      const int ly = ty + 4 * j;
      const int gx = x0 + tx, gy = y0 + ly;
      if (gx < I.nx && gy < I.ny) {
        const size_t gi = size_t(gy) * I.nx + gx;
        const V t = kop<V, T>(PT, Hs, ly, tx, T(I.cx), T(I.cy), T(I.cxy), gamma, zeta);
        const V s = PT[(ly + 2) * kVW + tx + 2];
        d[gi] = cadd(d[gi], cadd(cmul(alpha, pn[gi]), cmul(omega, s)));
        const V r = csub(s, cmul(omega, t));
        rd[gi] = r;
        const V h = rh[gi];
        acc[0] += double(h.x) * r.x + double(h.y) * r.y;   // conj(h) r
        acc[1] += double(h.x) * r.y - double(h.y) * r.x;
        acc[2] += double(r.x) * r.x + double(r.y) * r.y;
      }
    }
    double tot[3];
    block_sum_n<3>(acc, red, tot);
    if (threadIdx.x == 0) {
      double* pp = e.part + (size_t(it.slot) * e.cap_blk + it.tile) * kNDots;
      pp[0] = tot[0];
      pp[1] = tot[1];
      pp[2] = tot[2];
    }
  }
}

// ---- scalar kernels (one block per slot, partials in tile order) -----------
template <int N>
__device__ __forceinline__ bool slot_sums(const Eng& e, Slot* S, double (&tot)[N], double* red) {
  const int nblk = ldc(&e.inst[ldc(&S->inst)].nblk);
  double v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = 0.0;
  const double* pp = e.part + size_t(blockIdx.x) * e.cap_blk * kNDots;
  for (int b = threadIdx.x; b < nblk; b += kNT) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += ldc(&pp[size_t(b) * kNDots + k]);
  }
  block_sum_n<N>(v, red, tot);
  return threadIdx.x == 0;
}

__global__ __launch_bounds__(kNT) void k_bcg_sa(Eng e) {
  __shared__ double red[4 * 2];
  Slot* S = &e.slots[blockIdx.x];
  if (ldc(&S->status) != kInner) return;
  double tot[2];
  if (!slot_sums<2>(e, S, tot, red)) return;
  const double2 rv = make_double2(tot[0], tot[1]);
  if (!finite2(rv) || !(fabs(rv.x) + fabs(rv.y) > 0.0)) {
    S->status = kInnerDone;  // breakdown: restart from the FP64 residual
    return;
  }
  S->alpha = cdiv(ldc(&S->rr), rv);
}

__global__ __launch_bounds__(kNT) void k_bcg_sb(Eng e) {
  __shared__ double red[4 * 3];
  Slot* S = &e.slots[blockIdx.x];
  if (ldc(&S->status) != kInner) return;
  double tot[3];
  if (!slot_sums<3>(e, S, tot, red)) return;
  const double2 ts = make_double2(tot[0], tot[1]);
  const double tt = tot[2];
  S->omega = (tt > 0.0 && isfinite(tt) && finite2(ts)) ? make_double2(ts.x / tt, ts.y / tt) : make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(kNT) void k_bcg_sc(Eng e) {
  __shared__ double red[4 * 3];
  Slot* S = &e.slots[blockIdx.x];
  if (ldc(&S->status) != kInner) return;
  double tot[3];
  if (!slot_sums<3>(e, S, tot, red)) return;
  const double2 rr = make_double2(tot[0], tot[1]);
  const double n2 = tot[2];
  S->parity = ldc(&S->parity) ^ 1;
  S->prime = 0;
  S->it_inner = ldc(&S->it_inner) + 1;
  const int it_total = ldc(&S->it_total) + 1;
  S->it_total = it_total;
  const double2 om = ldc(&S->omega), al = ldc(&S->alpha), rho = ldc(&S->rr);
  const bool ok = isfinite(n2) && finite2(rr) && (fabs(rr.x) + fabs(rr.y) > 0.0) && (fabs(om.x) + fabs(om.y) > 0.0) &&
                  (fabs(rho.x) + fabs(rho.y) > 0.0);
  if (!ok || n2 <= ldc(&S->in_tol2) || it_total >= e.max_iter) {
    S->status = kInnerDone;
    return;
  }
  S->beta = cmul(cdiv(rr, rho), cdiv(al, om));
  S->rr = rr;
}

int prep_vh_blocks() { return 256; }

// ---- FP64 residual of the variable-coefficient system -----------------------
// r64 = sc (eta0 + a1 D + a2 Z) - K x64; r = r_hat = (T) r64, d = 0;
// partials |r64|^2 (index 0) and |r|^2 of the rounded residual (index 1).
template <typename T>
__global__ __launch_bounds__(kNT) void k_outer_residual_vh(Eng e) {
  using V = typename C2<T>::t;
  __shared__ double2 XT[kVH * kVW];
  __shared__ double Hs[kHH * kHW];
  __shared__ double red[4 * 2];
  const int total = ldc(&e.tile_start[e.B]);
  const int un = ldc(&e.work[1]);
  const int per = (total + 7) >> 3;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int w = blockIdx.x; w < 8 * per; w += gridDim.x) {
    const int pos = xcd_pos(w, per);
    if (pos >= total) continue;
    const Item it = item_of(e, pos, un);
    Slot* S = &e.slots[it.slot];
    const int st = ldc(&S->status);
    if (st != kInnerDone && st != kOuterPending) continue;
    const Inst I = ld_inst(&e.inst[ldc(&S->inst)]);
    const size_t base = size_t(it.slot) * e.cap;
    const double2* x = e.x64 + base;
    V* r = reinterpret_cast<V*>(ldc(&S->parity) ? e.r1 : e.r0) + base;
    V* rh = reinterpret_cast<V*>(e.rh) + base;
    V* d = reinterpret_cast<V*>(e.d) + base;
    const double2 zeta = ldc(&S->zeta), a1 = ldc(&S->a1), a2 = ldc(&S->a2);
    const double2 gamma = ldc(&S->gamma), sc = ldc(&S->sc);
    const bool zero_x = (ldc(&S->rounds) == 0);
    const int x0 = (it.tile % I.tiles_x) * kTX, y0 = (it.tile / I.tiles_x) * kTY;
    const bool big = (I.nx >= kVW) && (I.ny >= kVH);
    __syncthreads();
    if (!zero_x) {
      for (int k = threadIdx.x; k < kVH * kVW; k += kNT) {
        const int ly = k / kVW, lx = k - ly * kVW;
        XT[k] = x[size_t(wrapc(y0 - 2 + ly, I.ny, big)) * I.nx + wrapc(x0 - 2 + lx, I.nx, big)];
      }
      load_depth<double>(Hs, I.H, x0, y0, I, big);
    }
    __syncthreads();
    double acc[2] = {0.0, 0.0};
    for (int j = 0; j < kTY / 4; ++j) {
      const int ly = ty + 4 * j;
      const int gx = x0 + tx, gy = y0 + ly;
      if (gx < I.nx && gy < I.ny) {
        const size_t gi = size_t(gy) * I.nx + gx;
        double2 bv = make_double2(I.eta0[gi], 0.0);
        if (I.D0) {
          const double dv = I.D0[gi], zv = I.Z0[gi];
          bv.x += a1.x * dv + a2.x * zv;
          bv.y += a1.y * dv + a2.y * zv;
        }
        double2 rv = cmul(sc, bv);
        if (!zero_x) rv = csub(rv, kop<double2, double>(XT, Hs, ly, tx, I.cx, I.cy, I.cxy, gamma, zeta));
        const V rt = mk<V>(rv.x, rv.y);
        r[gi] = rt;
        rh[gi] = rt;
        d[gi] = mk<V>(0.0, 0.0);
        acc[0] += rv.x * rv.x + rv.y * rv.y;
        acc[1] += double(rt.x) * rt.x + double(rt.y) * rt.y;
      }
    }
    double tot[2];
    block_sum_n<2>(acc, red, tot);
    if (threadIdx.x == 0) {
      double* pp = e.part + (size_t(it.slot) * e.cap_blk + it.tile) * kNDots;
      pp[0] = tot[0];
      pp[1] = tot[1];
    }
  }
}

// ---- input preparation with a depth field ----------------------------------
// D_H = dx(H u0) + dy(H v0), Z_H = dx(H v0) - dy(H u0); flags: bit0
// non-finite state, bit1 non-zero velocity, bit2 non-zero divergence,
// bit3 non-finite or non-positive depth; per-block maxima of H.
__global__ __launch_bounds__(256) void k_prep_vh(const double* f, const double* H, int nx, int ny, double* D0,
                                                 double* Z0, int* flags, double* hmax_part) {
  __shared__ double sh[4];
  const size_t n = size_t(nx) * ny;
  int fl = 0;
  double hm = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int y = int(i / nx), x = int(i - size_t(y) * nx);
    const double* u = f + n;
    const double* v = f + 2 * n;
    const double e = f[i], uu = u[i], vv = v[i], hh = H[i];
    if (!isfinite(e) || !isfinite(uu) || !isfinite(vv)) fl |= 1;
    if (!isfinite(hh) || !(hh > 0.0)) fl |= 8;
    hm = fmax(hm, hh);
    if (uu != 0.0 || vv != 0.0) fl |= 2;
    const size_t xp = size_t(y) * nx + (x + 1 == nx ? 0 : x + 1);
    const size_t xm = size_t(y) * nx + (x == 0 ? nx - 1 : x - 1);
    const size_t yp = size_t(y + 1 == ny ? 0 : y + 1) * nx + x;
    const size_t ym = size_t(y == 0 ? ny - 1 : y - 1) * nx + x;
    const double hx = 0.5 * nx, hy = 0.5 * ny;
    const double div = hx * (H[xp] * u[xp] - H[xm] * u[xm]) + hy * (H[yp] * v[yp] - H[ym] * v[ym]);
    const double curl = hx * (H[xp] * v[xp] - H[xm] * v[xm]) - hy * (H[yp] * u[yp] - H[ym] * u[ym]);
    D0[i] = div;
    Z0[i] = curl;
    if (div != 0.0) fl |= 4;
  }
  if (fl) atomicOr(flags, fl);
  // block maximum (order-independent)
  for (int o = 32; o > 0; o >>= 1) hm = fmax(hm, __shfl_xor(hm, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = hm;
  __syncthreads();
  if (threadIdx.x == 0) hmax_part[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// per-block maxima of H and a validity flag (bit3: non-finite or <= 0)
__global__ __launch_bounds__(256) void k_hmax(const double* H, size_t n, int* flags, double* part) {
  __shared__ double sh[4];
  double hm = 0.0;
  int fl = 0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const double h = H[i];
    if (!isfinite(h) || !(h > 0.0)) fl |= 8;
    hm = fmax(hm, h);
  }
  if (fl) atomicOr(flags, fl);
  for (int o = 32; o > 0; o >>= 1) hm = fmax(hm, __shfl_xor(hm, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = hm;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ void k_fill_value(double* p, size_t n, double v) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) p[i] = v;
}

// ---- launchers -------------------------------------------------------------
void launch_hmax(const double* H, size_t n, int* flags, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_hmax, dim3(prep_vh_blocks()), dim3(256), 0, s, H, n, flags, part);
}
void launch_fill_value(double* p, size_t n, double v, hipStream_t s) {
  size_t bl = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_value, dim3(unsigned(bl > 8192 ? 8192 : (bl < 1 ? 1 : bl))), dim3(256), 0, s, p, n, v);
}
template <typename T>
void launch_bcg(const Eng& e, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_bcg_a<T>, dim3(grid), dim3(kNT), 0, s, e);
  hipLaunchKernelGGL(k_bcg_sa, dim3(e.B), dim3(kNT), 0, s, e);
  hipLaunchKernelGGL(k_bcg_b<T>, dim3(grid), dim3(kNT), 0, s, e);
  hipLaunchKernelGGL(k_bcg_sb, dim3(e.B), dim3(kNT), 0, s, e);
  hipLaunchKernelGGL(k_bcg_c<T>, dim3(grid), dim3(kNT), 0, s, e);
  hipLaunchKernelGGL(k_bcg_sc, dim3(e.B), dim3(kNT), 0, s, e);
}
template <typename T>
void launch_outer_residual_vh(const Eng& e, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_residual_vh<T>, dim3(grid), dim3(kNT), 0, s, e);
}
void launch_prep_vh(const double* f, const double* H, int nx, int ny, double* D0, double* Z0, int* flags,
                    double* hmax_part, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_vh, dim3(prep_vh_blocks()), dim3(256), 0, s, f, H, nx, ny, D0, Z0, flags, hmax_part);
}
int bcg_occupancy(int mixed) {
  int a = 0, b = 0;
  if (mixed) {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_bcg_a<float>, kNT, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_bcg_c<float>, kNT, 0);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_bcg_a<double>, kNT, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_bcg_c<double>, kNT, 0);
  }
  const int m = a < b ? a : b;
  return m > 0 ? m : 1;
}

template void launch_bcg<float>(const Eng&, int, hipStream_t);
template void launch_bcg<double>(const Eng&, int, hipStream_t);
template void launch_outer_residual_vh<float>(const Eng&, int, hipStream_t);
template void launch_outer_residual_vh<double>(const Eng&, int, hipStream_t);

}  // namespace rexii
