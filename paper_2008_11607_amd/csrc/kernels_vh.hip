// Variable-depth (flux form) shifted solves: BiCGStab on
//   K eta = (L_H + gamma C_H - zeta) eta = b        (see kernels.h)
// for every live slot, with <a, b> = sum conj(a) b and the shadow residual
// r_hat fixed to the first residual of each inner solve.  One iteration is
// three stencil passes and two one-block-per-slot scalar kernels
// (deterministic partial sums):
//
//   pass S  (alpha known):  s = r - alpha v (tile + halo 2), t = K s;
//           partials <t, s>, <t, t>, <s, s>, <r_hat, s>, <r_hat, t>
//   scalars: omega = <t, s>/<t, t> and, with no further pass,
//           rho' = <r_hat, r'> = <r_hat, s> - omega <r_hat, t>,
//           |r'|^2 = <s, s> - |<t, s>|^2/<t, t>  (stop test),
//           beta = (rho'/rho)(alpha/omega)
//   pass U1 (omega, beta known):  s and t again, then on the tile
//           d += alpha p + omega s, r' = s - omega t, p' = r' + beta (p - omega v)
//   pass U2: v' = K p',  partial <r_hat, v'>
//   scalars: alpha' = rho'/<r_hat, v'>
//
// The FP64 residual round of iterative refinement is folded into pass U1: a
// slot whose inner solve ended computes, with x = x64 + d (0 for a fresh
// solve), r64 = sc (eta0 + a1 D_H + a2 Z_H) - K x in FP64 and sets
// r = r_hat = p = (T) r64; pass U2 then forms v = K p and the scalar kernel
// decides convergence or restarts the inner solve.  As in the COCG pass,
// x64 and d are only read in a residual round; the first pass U1 of the next
// round moves d into x64.  A slot whose stop test fired in the scalars of
// pass S still gets its last update d += alpha p + omega s in pass U1
// (status kInnerLast) before its residual round.  r, p and v are ping-pong
// buffers so that no pass reads (with a halo) what another block of the
// same pass writes.
#include <algorithm>

#include "device_util.h"
#include "kernels.h"

namespace rexii {

// Tiles of kTX x TH points (TH = 16 or 32 rows, chosen per engine): row
// widths of the halo-2 tile, of the depth tile (halo 1), and the grid size
// from which the cheap periodic wrap is exact
constexpr int kBW = kTX + 4;   // tile with halo 2: TH + 4 rows
constexpr int kHW = kTX + 2;   // depth tile with halo 1: TH + 2 rows
constexpr int kSW = kTX + 8;   // with TH + 8 rows

// K phi at position (y, x) of a phi tile with row width PW; the same grid
// point is (y + DH, x + DH) of the depth tile (row width HW).
template <int PW, int HW, int DH, typename V, typename S, typename HT>
__device__ __forceinline__ V kop(const V* P, const HT* Hs, int y, int x, S cx, S cy, S cxy, V gamma, V zeta) {
  const V c = P[y * PW + x];
  const V e = P[y * PW + x + 2], w = P[y * PW + x - 2];
  const V n = P[(y + 2) * PW + x], s = P[(y - 2) * PW + x];
  const V ne = P[(y + 1) * PW + x + 1], nw = P[(y + 1) * PW + x - 1];
  const V se = P[(y - 1) * PW + x + 1], sw = P[(y - 1) * PW + x - 1];
  const int hy = y + DH, hx = x + DH;
  const S hxp = S(Hs[hy * HW + hx + 1]), hxm = S(Hs[hy * HW + hx - 1]);
  const S hyp = S(Hs[(hy + 1) * HW + hx]), hym = S(Hs[(hy - 1) * HW + hx]);
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

// conj(a) b accumulated in FP64
template <typename V>
__device__ __forceinline__ void cdot(double* acc, V a, V b) {
  acc[0] += double(a.x) * b.x + double(a.y) * b.y;
  acc[1] += double(a.x) * b.y - double(a.y) * b.x;
}

// Control fields of a slot, from one wavefront load of its record.
struct BcgCtl {
  int status, par, rounds, it_inner, discard, nx, ny, tiles_x;
  double cx, cy, cxy;
  const double* H;   // depth, FP64 (residual rounds)
  const void* Hin;   // depth in the inner-iteration type (passes S, U1, U2)
  double2 alpha, beta, omega, gamma, zeta;
};

__device__ __forceinline__ BcgCtl load_bctl(const Slot* S) {
  const SlotWords sw(S);
  BcgCtl c;
  c.status = sw.i32(SLOT_OFF(status));
  c.par = sw.i32(SLOT_OFF(parity));
  c.rounds = sw.i32(SLOT_OFF(rounds));
  c.it_inner = sw.i32(SLOT_OFF(it_inner));
  c.discard = sw.i32(SLOT_OFF(discard));
  c.nx = sw.i32(SLOT_OFF(nx));
  c.ny = sw.i32(SLOT_OFF(ny));
  c.tiles_x = sw.i32(SLOT_OFF(tiles_x));
  c.cx = sw.f64(SLOT_OFF(cx));
  c.cy = sw.f64(SLOT_OFF(cy));
  c.cxy = sw.f64(SLOT_OFF(cxy));
  c.H = sw.ptr<const double>(SLOT_OFF(H));
  c.Hin = sw.ptr<const void>(SLOT_OFF(Hin));
  c.alpha = sw.c64(SLOT_OFF(alpha));
  c.beta = sw.c64(SLOT_OFF(beta));
  c.omega = sw.c64(SLOT_OFF(omega));
  c.gamma = sw.c64(SLOT_OFF(gamma));
  c.zeta = sw.c64(SLOT_OFF(zeta));
  return c;
}

// ---- pass S ----------------------------------------------------------------
template <typename T, int TH>
struct LdsS {
  using V = typename C2<T>::t;
  static constexpr size_t kBytes = sizeof(V) * (TH + 4) * kBW + sizeof(T) * (TH + 2) * kHW;
};

template <typename T, int TH>
__device__ __forceinline__ void bcg_s(const Eng& e, const BcgCtl& c, int slot, int tile, unsigned char* lds,
                                      double (&acc)[8]) {
  using V = typename C2<T>::t;
  V* ST = reinterpret_cast<V*>(lds);
  T* Hs = reinterpret_cast<T*>(lds + sizeof(V) * (TH + 4) * kBW);
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const V* rs = reinterpret_cast<const V*>(c.par ? e.r1 : e.r0) + base;
  const V* vs = reinterpret_cast<const V*>(c.par ? e.v1 : e.v0) + base;
  const V* rh = reinterpret_cast<const V*>(e.rh) + base;
  const V alpha = mk<V>(c.alpha.x, c.alpha.y);
  const V gamma = mk<V>(c.gamma.x, c.gamma.y), zeta = mk<V>(c.zeta.x, c.zeta.y);
  const T cx = T(c.cx), cy = T(c.cy), cxy = T(c.cxy);
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * TH;
  const bool big = (nx >= kSW) && (ny >= (TH + 8));
  // pure loads first, then the tile whose values are formed as they
  // arrive (s = r - alpha v), so that every load is in flight before the
  // first wait
  const T* Hi = static_cast<const T*>(c.Hin);
  RowTile<T, 1, TH> hr;
  hr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) { return Hi[ro + col]; });
  const unsigned col = unsigned(wrapc(x0 + tx, nx, big));
  V hv[TH / 4];
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) hv[j] = (rh + size_t(wrapc(y0 + ty + 4 * j, ny, big)) * size_t(nx))[col];
  RowTile<V, 2, TH> sr;
  sr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) {
    const size_t g = ro + col;
    return csub(rs[g], cmul(alpha, vs[g]));
  });
  __syncthreads();  // LDS of the previous work item is free
  sr.store(ST);
  hr.store(Hs);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) {
    const int ly = ty + 4 * j;
    if (x0 + tx < nx && y0 + ly < ny) {
      const V t = kop<kBW, kHW, -1>(ST, Hs, ly + 2, tx + 2, cx, cy, cxy, gamma, zeta);
      const V s = ST[(ly + 2) * kBW + tx + 2];
      cdot(acc + 0, t, s);
      acc[2] += double(t.x) * t.x + double(t.y) * t.y;
      acc[3] += double(s.x) * s.x + double(s.y) * s.y;
      cdot(acc + 4, hv[j], s);
      cdot(acc + 6, hv[j], t);
    }
  }
}

// ---- pass U1: updates ------------------------------------------------------
// Inner step: s = r - alpha v (tile + halo 2), t = K s, then on the tile
// d += alpha p + omega s, r' = s - omega t, p' = r' + beta (p - omega v).
template <typename T, int TH>
__device__ __forceinline__ void bcg_u1_inner(const Eng& e, const BcgCtl& c, int slot, int tile, unsigned char* lds) {
  using V = typename C2<T>::t;
  V* ST = reinterpret_cast<V*>(lds);
  T* Hs = reinterpret_cast<T*>(lds + sizeof(V) * (TH + 4) * kBW);
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const V* rs = reinterpret_cast<const V*>(c.par ? e.r1 : e.r0) + base;
  V* rd = reinterpret_cast<V*>(c.par ? e.r0 : e.r1) + base;
  const V* ps = reinterpret_cast<const V*>(c.par ? e.p1 : e.p0) + base;
  V* pd = reinterpret_cast<V*>(c.par ? e.p0 : e.p1) + base;
  const V* vs = reinterpret_cast<const V*>(c.par ? e.v1 : e.v0) + base;
  V* d = reinterpret_cast<V*>(e.d) + base;
  double2* x64 = e.x64 + base;
  const bool first = c.it_inner == 1;                      // d restarts this pass
  const bool fold = first && c.rounds >= 2 && !c.discard;  // ... after x64 += d
  const V alpha = mk<V>(c.alpha.x, c.alpha.y), beta = mk<V>(c.beta.x, c.beta.y);
  const V omega = mk<V>(c.omega.x, c.omega.y);
  const V gamma = mk<V>(c.gamma.x, c.gamma.y), zeta = mk<V>(c.zeta.x, c.zeta.y);
  const T cx = T(c.cx), cy = T(c.cy), cxy = T(c.cxy);
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * TH;
  const bool big = (nx >= kSW) && (ny >= (TH + 8));
  // pure loads first (depth tile, p, v, d; rows are wavefront-uniform, so
  // row offsets sit in scalar registers and one column offset serves every
  // load), then the tile formed as it arrives (s = r - alpha v)
  const T* Hi = static_cast<const T*>(c.Hin);
  RowTile<T, 1, TH> hr;
  hr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) { return Hi[ro + col]; });
  const unsigned col = unsigned(wrapc(x0 + tx, nx, big));
  size_t ro[TH / 4];
  V pv[TH / 4], vv[TH / 4], dv[TH / 4];
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) {
    ro[j] = size_t(wrapc(y0 + ty + 4 * j, ny, big)) * size_t(nx);
    pv[j] = (ps + ro[j])[col];
    vv[j] = (vs + ro[j])[col];
    if (!first) dv[j] = nt_load(&(d + ro[j])[col]);
  }
  RowTile<V, 2, TH> sr;
  sr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) {
    const size_t g = ro + col;
    return csub(rs[g], cmul(alpha, vs[g]));
  });
  __syncthreads();  // LDS of the previous work item is free
  sr.store(ST);
  hr.store(Hs);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) {
    const int ly = ty + 4 * j;
    if (x0 + tx < nx && y0 + ly < ny) {
      const V t = kop<kBW, kHW, -1>(ST, Hs, ly + 2, tx + 2, cx, cy, cxy, gamma, zeta);
      const V sv = ST[(ly + 2) * kBW + tx + 2];
      const V r1 = csub(sv, cmul(omega, t));
      const V p1 = cadd(r1, cmul(beta, csub(pv[j], cmul(omega, vv[j]))));
      const V upd = cadd(cmul(alpha, pv[j]), cmul(omega, sv));
      if (fold) {
        // once per round: the previous round's correction moves into x64
        const V dold = (d + ro[j])[col];
        const double2 xo = (x64 + ro[j])[col];
        (x64 + ro[j])[col] = make_double2(xo.x + double(dold.x), xo.y + double(dold.y));
      }
      nt_store(first ? upd : cadd(dv[j], upd), &(d + ro[j])[col]);
      (rd + ro[j])[col] = r1;
      (pd + ro[j])[col] = p1;
    }
  }
}

// last update of an inner solve (no halo): d += alpha p + omega (r - alpha v)
template <typename T, int TH>
__device__ __forceinline__ void bcg_u1_last(const Eng& e, const BcgCtl& c, int slot, int tile) {
  using V = typename C2<T>::t;
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const V* rs = reinterpret_cast<const V*>(c.par ? e.r1 : e.r0) + base;
  const V* ps = reinterpret_cast<const V*>(c.par ? e.p1 : e.p0) + base;
  const V* vs = reinterpret_cast<const V*>(c.par ? e.v1 : e.v0) + base;
  V* d = reinterpret_cast<V*>(e.d) + base;
  double2* x64 = e.x64 + base;
  const bool first = c.it_inner == 1;
  const bool fold = first && c.rounds >= 2 && !c.discard;
  const V alpha = mk<V>(c.alpha.x, c.alpha.y), omega = mk<V>(c.omega.x, c.omega.y);
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * TH;
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) {
    const int gx = x0 + tx, gy = y0 + ty + 4 * j;
    if (gx < nx && gy < ny) {
      const size_t ro = size_t(gy) * size_t(nx);
      const V s = csub((rs + ro)[gx], cmul(alpha, (vs + ro)[gx]));
      const V upd = cadd(cmul(alpha, (ps + ro)[gx]), cmul(omega, s));
      const V dold = (d + ro)[gx];
      if (fold) {
        const double2 xo = (x64 + ro)[gx];
        (x64 + ro)[gx] = make_double2(xo.x + double(dold.x), xo.y + double(dold.y));
      }
      (d + ro)[gx] = first ? upd : cadd(dold, upd);
    }
  }
}

// FP64 residual round: with x = x64 + d (0 for a fresh solve) on tile +
// halo 2, r64 = sc (eta0 + a1 D_H + a2 Z_H) - K x on the tile;
// r = r_hat = p = (T) r64; partials |r64|^2 (index 2) and |r|^2 (index 3).
template <typename T, int TH>
__device__ __forceinline__ void bcg_u1_outer(const Eng& e, const BcgCtl& c, int slot, int tile, unsigned char* lds,
                                             double (&acc)[2]) {
  using V = typename C2<T>::t;
  double2* XT = reinterpret_cast<double2*>(lds);
  double* Hs = reinterpret_cast<double*>(lds + sizeof(double2) * (TH + 4) * kBW);
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const double2* x64 = e.x64 + base;
  const V* d = reinterpret_cast<const V*>(e.d) + base;
  V* rd = reinterpret_cast<V*>(c.par ? e.r0 : e.r1) + base;
  V* pd = reinterpret_cast<V*>(c.par ? e.p0 : e.p1) + base;
  V* rh = reinterpret_cast<V*>(e.rh) + base;
  const bool zero_x = c.rounds == 0;  // fresh solve: x = 0, d holds nothing
  const bool use_d = !c.discard;   // else the iterate is x64 alone
  const SlotWords sw(&e.slots[slot]);  // right-hand side fields, needed only here
  const double2 a1 = sw.c64(SLOT_OFF(a1)), a2 = sw.c64(SLOT_OFF(a2)), sc = sw.c64(SLOT_OFF(sc));
  const double* eta0 = sw.ptr<const double>(SLOT_OFF(eta0));
  const double* D0 = sw.ptr<const double>(SLOT_OFF(D0));
  const double* Z0 = sw.ptr<const double>(SLOT_OFF(Z0));
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * TH;
  const bool big = (nx >= kSW) && (ny >= (TH + 8));
  // every load of the work item in one round: the right-hand side fields
  // (interior) and the depth (halo 1) first, then x = x64 + d (halo 2),
  // formed as it arrives (d is read even when discarded, then not used)
  const unsigned col = unsigned(wrapc(x0 + tx, nx, big));
  double bre[TH / 4], bdz[TH / 4], bzz[TH / 4];
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) {
    const size_t ro = size_t(wrapc(y0 + ty + 4 * j, ny, big)) * size_t(nx);
    bre[j] = (eta0 + ro)[col];
    if (D0) {
      bdz[j] = (D0 + ro)[col];
      bzz[j] = (Z0 + ro)[col];
    }
  }
  // x64 and d as two tiles of pure loads, added in registers once all have
  // been issued (the block runs at two per CU for its LDS: registers are
  // not what limits it)
  RowTile<double2, 2, TH> xr;
  RowTile<V, 2, TH> dr;
  RowTile<double, 1, TH> hr;
  if (!zero_x) {
    hr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) { return c.H[ro + col]; });
    xr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) { return x64[ro + col]; });
    dr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) { return d[ro + col]; });
    if (use_d) {  // a discarded d may hold non-finite values: not added
#pragma unroll
      for (int m = 0; m < RowTile<double2, 2, TH>::kRows; ++m) {
        xr.mainv[m].x += double(dr.mainv[m].x);
        xr.mainv[m].y += double(dr.mainv[m].y);
      }
      xr.sidev.x += double(dr.sidev.x);
      xr.sidev.y += double(dr.sidev.y);
    }
  }
  __syncthreads();  // LDS of the previous work item is free
  if (!zero_x) {
    xr.store(XT);
    hr.store(Hs);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) {
    const int ly = ty + 4 * j;
    const int gx = x0 + tx, gy = y0 + ly;
    if (gx < nx && gy < ny) {
      const size_t ro = size_t(gy) * size_t(nx);
      double2 bv = make_double2(bre[j], 0.0);
      if (D0) {
        bv.x += a1.x * bdz[j] + a2.x * bzz[j];
        bv.y += a1.y * bdz[j] + a2.y * bzz[j];
      }
      double2 rv = cmul(sc, bv);
      if (!zero_x) rv = csub(rv, kop<kBW, kHW, -1>(XT, Hs, ly + 2, tx + 2, c.cx, c.cy, c.cxy, c.gamma, c.zeta));
      const V rt = mk<V>(rv.x, rv.y);
      (rd + ro)[gx] = rt;
      (pd + ro)[gx] = rt;
      (rh + ro)[gx] = rt;
      acc[0] += rv.x * rv.x + rv.y * rv.y;
      acc[1] += double(rt.x) * rt.x + double(rt.y) * rt.y;
    }
  }
}

// ---- pass U2: v' = K p' and <r_hat, v'> -------------------------------------
template <typename T, int TH>
__device__ __forceinline__ void bcg_u2(const Eng& e, const BcgCtl& c, int slot, int tile, unsigned char* lds,
                                       double (&acc)[2]) {
  using V = typename C2<T>::t;
  V* PT = reinterpret_cast<V*>(lds);
  T* Hs = reinterpret_cast<T*>(lds + sizeof(V) * (TH + 4) * kBW);
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  // p' was written by pass U1 into the buffers of the next parity
  const V* pn = reinterpret_cast<const V*>(c.par ? e.p0 : e.p1) + base;
  V* vd = reinterpret_cast<V*>(c.par ? e.v0 : e.v1) + base;
  const V* rh = reinterpret_cast<const V*>(e.rh) + base;
  const V gamma = mk<V>(c.gamma.x, c.gamma.y), zeta = mk<V>(c.zeta.x, c.zeta.y);
  const T cx = T(c.cx), cy = T(c.cy), cxy = T(c.cxy);
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * TH;
  const bool big = (nx >= kSW) && (ny >= (TH + 8));
  RowTile<V, 2, TH> pr;
  pr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) {
    const size_t g = ro + col;
    return pn[g];
  });
  const T* Hi = static_cast<const T*>(c.Hin);
  RowTile<T, 1, TH> hr;
  hr.fetch(x0, y0, nx, ny, big, [&](size_t ro, unsigned col) { return Hi[ro + col]; });
  const unsigned col = unsigned(wrapc(x0 + tx, nx, big));
  V hv[TH / 4];
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) hv[j] = (rh + size_t(wrapc(y0 + ty + 4 * j, ny, big)) * size_t(nx))[col];
  __syncthreads();  // LDS of the previous work item is free
  pr.store(PT);
  hr.store(Hs);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < TH / 4; ++j) {
    const int ly = ty + 4 * j;
    if (x0 + tx < nx && y0 + ly < ny) {
      const V v1 = kop<kBW, kHW, -1>(PT, Hs, ly + 2, tx + 2, cx, cy, cxy, gamma, zeta);
      (vd + size_t(y0 + ly) * size_t(nx))[x0 + tx] = v1;
      cdot(acc, hv[j], v1);
    }
  }
}

template <typename T, int TH>
__device__ __forceinline__ void bcg_pass_s(const Eng& e) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LdsS<T, TH>::kBytes];
  __shared__ double red[4 * 8];
  const WorkMap m = load_work_map(e);
  const int span = work_span(m);
  for (int w = blockIdx.x; w < span; w += gridDim.x) {
    Item it;
    if (!work_item(e, m, w, it)) continue;
    const BcgCtl c = load_bctl(&e.slots[it.slot]);
    if (c.status != kInner) continue;
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    bcg_s<T, TH>(e, c, it.slot, it.tile, lds, acc);
    store_block_sums<8>(acc, red, item_part(e, it.slot, it.tile));
  }
}

template <typename T, int TH>
struct LdsU1 {
  static constexpr size_t kX = sizeof(double2) * (TH + 4) * kBW + sizeof(double) * (TH + 2) * kHW;  // residual round
};

template <typename T, int TH>
__device__ __forceinline__ void bcg_pass_u1(const Eng& e) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LdsS<T, TH>::kBytes];
  const WorkMap m = load_work_map(e);
  const int span = work_span(m);
  for (int w = blockIdx.x; w < span; w += gridDim.x) {
    Item it;
    if (!work_item(e, m, w, it)) continue;
    const BcgCtl c = load_bctl(&e.slots[it.slot]);
    if (c.status == kInner)
      bcg_u1_inner<T, TH>(e, c, it.slot, it.tile, lds);
    else if (c.status == kInnerLast)
      bcg_u1_last<T, TH>(e, c, it.slot, it.tile);
  }
}

// the FP64 residual rounds (a kernel of their own: sharing pass U1 would
// raise its register count for a step that runs once per round)
template <typename T, int TH>
__device__ __forceinline__ void bcg_pass_outer(const Eng& e) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LdsU1<T, TH>::kX];
  __shared__ double red[4 * 2];
  __shared__ int st[kMaxSlots];
  __shared__ int any;
  // the statuses of all slots in one round of loads; most launches find no
  // slot in a residual round and end here
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < e.B; q += kNT) {
    const int v = ldc(&e.slots[q].status);
    st[q] = v;
    if (v == kOuterPending || v == kInnerDone) any = 1;
  }
  __syncthreads();
  if (!any) return;
  const WorkMap m = load_work_map(e);
  const int span = work_span(m);
  for (int w = blockIdx.x; w < span; w += gridDim.x) {
    Item it;
    if (!work_item(e, m, w, it)) continue;
    if (st[it.slot] != kOuterPending && st[it.slot] != kInnerDone) continue;
    const BcgCtl c = load_bctl(&e.slots[it.slot]);
    double acc[2] = {0.0, 0.0};
    bcg_u1_outer<T, TH>(e, c, it.slot, it.tile, lds, acc);
    store_block_sums<2, 2>(acc, red, item_part(e, it.slot, it.tile));
  }
}

template <typename T, int TH>
__device__ __forceinline__ void bcg_pass_u2(const Eng& e) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LdsS<T, TH>::kBytes];
  __shared__ double red[4 * 2];
  const WorkMap m = load_work_map(e);
  const int span = work_span(m);
  for (int w = blockIdx.x; w < span; w += gridDim.x) {
    Item it;
    if (!work_item(e, m, w, it)) continue;
    const BcgCtl c = load_bctl(&e.slots[it.slot]);
    if (c.status != kInner && c.status != kOuterPending && c.status != kInnerDone) continue;
    double acc[2] = {0.0, 0.0};
    bcg_u2<T, TH>(e, c, it.slot, it.tile, lds, acc);
    store_block_sums<2>(acc, red, item_part(e, it.slot, it.tile));
  }
}

// 64 x 32 tiles (the default) and 64 x 16 tiles (suffix _h16)
__global__ __launch_bounds__(kNT) void k_bcg_s_f32(Eng e) { bcg_pass_s<float, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_s_f64(Eng e) { bcg_pass_s<double, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u1_f32(Eng e) { bcg_pass_u1<float, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u1_f64(Eng e) { bcg_pass_u1<double, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_outer_f32(Eng e) { bcg_pass_outer<float, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_outer_f64(Eng e) { bcg_pass_outer<double, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u2_f32(Eng e) { bcg_pass_u2<float, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u2_f64(Eng e) { bcg_pass_u2<double, 32>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_s_f32_h16(Eng e) { bcg_pass_s<float, 16>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_s_f64_h16(Eng e) { bcg_pass_s<double, 16>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u1_f32_h16(Eng e) { bcg_pass_u1<float, 16>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u1_f64_h16(Eng e) { bcg_pass_u1<double, 16>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_outer_f32_h16(Eng e) { bcg_pass_outer<float, 16>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_outer_f64_h16(Eng e) { bcg_pass_outer<double, 16>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u2_f32_h16(Eng e) { bcg_pass_u2<float, 16>(e); }
__global__ __launch_bounds__(kNT) void k_bcg_u2_f64_h16(Eng e) { bcg_pass_u2<double, 16>(e); }

// ---- scalar kernels (one block per slot, partials in tile order) -----------
template <int N>
__device__ __forceinline__ bool slot_sums(const Eng& e, const Slot* S, double (&tot)[N], double* red) {
  slot_sums_n<N>(e.part + size_t(blockIdx.x) * e.cap_blk * kNDots, ldc(&S->nblk), tot, red);
  return threadIdx.x == 0;
}

__device__ __forceinline__ bool nonzero(double2 v) { return fabs(v.x) + fabs(v.y) > 0.0; }

// after pass S: omega, rho', beta and the stop test
__global__ __launch_bounds__(kSNT) void k_bcg_scalars_s(Eng e) {
  __shared__ double red[kSNT / 64 * 8];
  Slot* S = &e.slots[blockIdx.x];
  if (ldc(&S->status) != kInner) return;
  double tot[8];
  if (!slot_sums<8>(e, S, tot, red)) return;
  const double2 ts = make_double2(tot[0], tot[1]);
  const double tt = tot[2], ss = tot[3];
  const double2 hs = make_double2(tot[4], tot[5]), ht = make_double2(tot[6], tot[7]);
  S->it_inner = ldc(&S->it_inner) + 1;
  const int it_total = ldc(&S->it_total) + 1;
  S->it_total = it_total;
  const bool ok_t = tt > 0.0 && isfinite(tt) && finite2(ts) && isfinite(ss) && finite2(hs) && finite2(ht);
  if (!ok_t) {
    // breakdown: keep the BiCG half step (d += alpha p) and restart
    S->omega = make_double2(0.0, 0.0);
    S->status = kInnerLast;
    return;
  }
  const double2 om = make_double2(ts.x / tt, ts.y / tt);
  if (!(fabs(om.x) + fabs(om.y) < 1e30)) {
    // omega outside the inner precision's range: keep the half step
    S->omega = make_double2(0.0, 0.0);
    S->status = kInnerLast;
    return;
  }
  S->omega = om;
  const double2 rho1 = csub(hs, cmul(om, ht));
  const double n2 = fmax(ss - (ts.x * ts.x + ts.y * ts.y) / tt, 0.0);
  const double2 rho = ldc(&S->rr), al = ldc(&S->alpha);
  const bool ok = nonzero(om) && nonzero(rho1) && nonzero(rho) && finite2(rho1);
  if (!ok || n2 <= ldc(&S->in_tol2) || it_total >= ldc(&S->max_it)) {
    S->status = kInnerLast;
    return;
  }
  S->beta = cmul(cdiv(rho1, rho), cdiv(al, om));
  S->rr = rho1;
}

// after pass U: alpha of the next iteration; end of the last update; or the
// decision of an FP64 residual round
__global__ __launch_bounds__(kSNT) void k_bcg_scalars_u(Eng e) {
  __shared__ double red[kSNT / 64 * 4];
  Slot* S = &e.slots[blockIdx.x];
  const int status = ldc(&S->status);
  if (status == kInnerLast) {
    if (threadIdx.x == 0) {
      if (ldc(&S->it_inner) == 1) S->discard = 0;  // pass U1 restarted d
      S->status = kInnerDone;
    }
    return;
  }
  const bool outer = (status == kOuterPending || status == kInnerDone);
  if (status != kInner && !outer) return;
  double tot[4];
  if (!slot_sums<4>(e, S, tot, red)) return;
  const double2 hv = make_double2(tot[0], tot[1]);
  S->parity = ldc(&S->parity) ^ 1;
  double2 rho = ldc(&S->rr);
  if (outer) {
    const double rn2 = tot[2];
    const int rounds0 = ldc(&S->rounds);
    double bn2 = ldc(&S->bn2);
    if (rounds0 == 0) {
      bn2 = rn2;
      S->bn2 = rn2;
    }
    if (!isfinite(rn2) && rounds0 >= 1 && !ldc(&S->discard)) {
      // the last inner round went non-finite: drop its correction d and
      // take the residual of x64 alone in the next residual round
      S->discard = 1;
      return;
    }
    const int rounds = rounds0 + 1;
    S->rounds = rounds;
    const double prev = ldc(&S->prev_rn2);
    const double ref2 = ldc(&S->ref2);
    // stop threshold on |b - K x|^2: tol2 times the fixed reference, or
    // times |b|^2 (relative residual)
    const double thr = ldc(&S->tol2) * (ref2 > 0.0 ? ref2 : bn2);
    S->rn2 = rn2;
    S->prev_rn2 = rn2;
    if (!isfinite(rn2)) {
      S->status = e.retry ? kRetry : kFailBreakdown;
      return;
    }
    if (rn2 <= thr) {
      S->status = kDone;
      return;
    }
    if (rounds >= 3 && rn2 > 0.25 * prev) {
      // a whole inner solve did not halve the FP64 residual.  Mixed
      // precision: the FP32 inner solves stalled or diverged, FP64 retry.
      // FP64: the iterate sits at its rounding floor, above the requested
      // tolerance; the achieved residual enters the reported error bound.
      if (e.retry) {
        S->status = kRetry;
        return;
      }
      S->status = kDone;
      S->stagnated = 1;
      if (rn2 > prev) {
        // the last correction made the iterate worse (an inner solve that
        // diverged): x64 holds the previous iterate, of residual prev
        S->discard = 1;
        S->rn2 = prev;
      }
      return;
    }
    if (ldc(&S->it_total) >= ldc(&S->max_it)) {
      S->status = e.retry ? kRetry : kFailMaxIter;
      return;
    }
    // restart: r_hat = r, rho = <r_hat, r> = |r|^2 of the rounded residual
    rho = make_double2(tot[3], 0.0);
    S->rr = rho;
    S->it_inner = 0;
    S->in_tol2 = fmax(e.inner_eta2 * rn2, 0.0625 * thr);
    S->status = kInner;
  }
  const double2 al = (finite2(hv) && nonzero(hv) && nonzero(rho)) ? cdiv(rho, hv) : make_double2(NAN, NAN);
  if (!(fabs(al.x) + fabs(al.y) < 1e30)) {
    if (!outer) {
      // breakdown inside the inner solve: restart from the FP64 residual
      S->status = kInnerDone;
    } else if (e.retry) {
      // no usable restart in the inner precision: FP64 retry
      S->status = kRetry;
    } else if (ldc(&S->rounds) >= 2) {
      // no usable restart from a finite residual above the tolerance: the
      // solve stops at its current iterate (its residual enters the
      // reported error bound)
      S->status = kDone;
      S->stagnated = 1;
    } else {
      S->status = kFailBreakdown;
    }
    return;
  }
  if (!outer && ldc(&S->it_inner) == 1) S->discard = 0;  // pass U1 restarted d
  S->alpha = al;
}

int prep_vh_blocks() { return 256; }

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
__global__ void k_to_f32(const double* p, float* q, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    q[i] = float(p[i]);
}
void launch_to_f32(const double* p, float* q, size_t n, hipStream_t s) {
  size_t bl = (n + 255) / 256;
  hipLaunchKernelGGL(k_to_f32, dim3(unsigned(bl > 8192 ? 8192 : (bl < 1 ? 1 : bl))), dim3(256), 0, s, p, q, n);
}
void launch_fill_value(double* p, size_t n, double v, hipStream_t s) {
  size_t bl = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_value, dim3(unsigned(bl > 8192 ? 8192 : (bl < 1 ? 1 : bl))), dim3(256), 0, s, p, n, v);
}
template <typename T>
void launch_bcg(const Eng& e, int grid, hipStream_t s, hipEvent_t* ev) {
  const bool f32 = sizeof(T) == 4, h16 = e.th == 16;
  using K = void (*)(Eng);
  const K outer = f32 ? (h16 ? k_bcg_outer_f32_h16 : k_bcg_outer_f32) : (h16 ? k_bcg_outer_f64_h16 : k_bcg_outer_f64);
  const K u1 = f32 ? (h16 ? k_bcg_u1_f32_h16 : k_bcg_u1_f32) : (h16 ? k_bcg_u1_f64_h16 : k_bcg_u1_f64);
  const K u2 = f32 ? (h16 ? k_bcg_u2_f32_h16 : k_bcg_u2_f32) : (h16 ? k_bcg_u2_f64_h16 : k_bcg_u2_f64);
  const K sp = f32 ? (h16 ? k_bcg_s_f32_h16 : k_bcg_s_f32) : (h16 ? k_bcg_s_f64_h16 : k_bcg_s_f64);
  int k = 0;
  auto mark = [&]() {
    if (ev) (void)hipEventRecord(ev[k++], s);
  };
  mark();
  hipLaunchKernelGGL(outer, dim3(std::min(grid, e.grid_small)), dim3(kNT), 0, s, e);
  mark();
  hipLaunchKernelGGL(u1, dim3(grid), dim3(kNT), 0, s, e);
  mark();
  hipLaunchKernelGGL(u2, dim3(grid), dim3(kNT), 0, s, e);
  mark();
  hipLaunchKernelGGL(k_bcg_scalars_u, dim3(e.B), dim3(kSNT), 0, s, e);
  mark();
  hipLaunchKernelGGL(sp, dim3(grid), dim3(kNT), 0, s, e);
  mark();
  hipLaunchKernelGGL(k_bcg_scalars_s, dim3(e.B), dim3(kSNT), 0, s, e);
  mark();
}
void launch_prep_vh(const double* f, const double* H, int nx, int ny, double* D0, double* Z0, int* flags,
                    double* hmax_part, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_vh, dim3(prep_vh_blocks()), dim3(256), 0, s, f, H, nx, ny, D0, Z0, flags, hmax_part);
}
int bcg_occupancy(int mixed, int th) {
  const bool h16 = th == 16;
  int a = 0, b = 0;
  if (mixed) {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, h16 ? k_bcg_u1_f32_h16 : k_bcg_u1_f32, kNT, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, h16 ? k_bcg_s_f32_h16 : k_bcg_s_f32, kNT, 0);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, h16 ? k_bcg_u1_f64_h16 : k_bcg_u1_f64, kNT, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, h16 ? k_bcg_s_f64_h16 : k_bcg_s_f64, kNT, 0);
  }
  const int m = a < b ? a : b;
  return m > 0 ? m : 1;
}

template void launch_bcg<float>(const Eng&, int, hipStream_t, hipEvent_t*);
template void launch_bcg<double>(const Eng&, int, hipStream_t, hipEvent_t*);

}  // namespace rexii
