// gfx950 kernels of the REXII shifted-solve path (see kernels.h for the
// mathematics and the slot scheme).
//
// Determinism: every block writes its partial sums to a fixed place; the
// last block of a slot adds them in index order; wavefront sums use a fixed
// xor-shuffle tree over the 64 lanes.  Accumulation into the FP64 outputs
// walks the slots in index order.  Results are therefore bitwise
// reproducible for a given slot count and chunk length.
//
// Work mapping: the pass kernels are persistent (grid-stride) over work items
// (slot, tile).  Work items are numbered so that each of the 8 XCDs (block b
// runs on XCD b % 8) walks one contiguous range of tiles, keeping the halo
// rows of neighbouring tiles in that XCD's L2.
#include "kernels.h"
#include "device_util.h"

namespace rexii {


// Stencil (L - zeta) v at LDS position (y, x) of a tile with row width W.
template <typename V, typename S, int W>
__device__ __forceinline__ V helm(const V* t, int y, int x, S cx, S cy, V zeta) {
  const V c = t[y * W + x];
  const V e = t[y * W + x + 2];
  const V w = t[y * W + x - 2];
  const V n = t[(y + 2) * W + x];
  const V s = t[(y - 2) * W + x];
  V q;
  q.x = cx * (e.x + w.x - S(2) * c.x) + cy * (n.x + s.x - S(2) * c.x) - (zeta.x * c.x - zeta.y * c.y);
  q.y = cx * (e.y + w.y - S(2) * c.y) + cy * (n.y + s.y - S(2) * c.y) - (zeta.x * c.y + zeta.y * c.x);
  return q;
}

// ---------------------------------------------------------------------------
// The COCG pass.  Each launch advances every live slot by one step; what the
// step is depends on the slot's state.
//
// Inner step (status kInner), input (x_i = d, r_i, p_i) with alpha_i, beta_i:
//   q_i = (L - zeta) p_i                      (tile + halo 2, from p with halo 4)
//   d  += alpha_i p_i,  r_{i+1} = r_i - alpha_i q_i,  p_{i+1} = r_{i+1} + beta_i p_i
//   (the d update as d += dcp p_i + dcr r_i, or none at all: see DMode)
//   q_{i+1} = (L - zeta) p_{i+1}              (tile)
//   partial sums: p_{i+1}^T q_{i+1}, q_{i+1}^T r_{i+1}, q_{i+1}^T q_{i+1},
//                 r_{i+1}^T r_{i+1}, |r_{i+1}|^2
// k_pass_scalars then sets alpha_{i+1} = rr_{i+1} / pq_{i+1} and
// beta_{i+1} = (rr_{i+1} - 2 alpha qr + alpha^2 qq) / rr_{i+1}.
//
// Residual step (status kOuterPending or kInnerDone): the FP64 residual
// round of iterative refinement, folded into the same launch.  With the
// current iterate x = x64 + d (x = 0 for a fresh solve; x with halo 2)
//   r64 = b - (L - zeta) x   in FP64 on the tile,   r = p = (T) r64,
// partial sum |r64|^2; k_pass_scalars decides convergence.  If the solve
// goes on, a prime step (status kPrime) forms q = (L - zeta) p from r with
// halo 2 and the sums of the restarted COCG, which give alpha and beta of
// the first inner step.  x64 and d are only read in a residual step (other
// blocks read them as halo); the first inner step of the round then folds d
// into x64 (x64 += d, point by point) and restarts d = alpha p.  The
// solution of a finished solve is therefore x64 + d once it has run at
// least one inner round.
// ---------------------------------------------------------------------------
constexpr int kPW = kTX + 8, kPH = kTY + 8;   // tile with halo 4
constexpr int kNW = kTX + 4, kNH = kTY + 4;   // tile with halo 2


// Control fields of a slot, from one wavefront load of its record.
struct SlotCtl {
  int status, par, rounds, it_inner, nx, ny, tiles_x, dmode;
  double cx, cy;
  double2 alpha, beta, zeta, dcp, dcr;
};

__device__ __forceinline__ SlotCtl load_ctl(const Slot* S) {
  const SlotWords sw(S);
  SlotCtl c;
  c.status = sw.i32(SLOT_OFF(status));
  c.par = sw.i32(SLOT_OFF(parity));
  c.rounds = sw.i32(SLOT_OFF(rounds));
  c.it_inner = sw.i32(SLOT_OFF(it_inner));
  c.nx = sw.i32(SLOT_OFF(nx));
  c.ny = sw.i32(SLOT_OFF(ny));
  c.tiles_x = sw.i32(SLOT_OFF(tiles_x));
  c.cx = sw.f64(SLOT_OFF(cx));
  c.cy = sw.f64(SLOT_OFF(cy));
  c.dmode = sw.i32(SLOT_OFF(dmode));
  c.alpha = sw.c64(SLOT_OFF(alpha));
  c.beta = sw.c64(SLOT_OFF(beta));
  c.zeta = sw.c64(SLOT_OFF(zeta));
  c.dcp = sw.c64(SLOT_OFF(dcp));
  c.dcr = sw.c64(SLOT_OFF(dcr));
  return c;
}

// LDS of the pass: a T tile with halo 2 (p_{i+1}, or r in a prime step)
// and a T tile of p with halo 4 (inner step), or an FP64 tile of x with
// halo 2 (residual step).
template <typename T>
struct PassLds {
  using V = typename C2<T>::t;
  static constexpr size_t kN = sizeof(V) * kNH * kNW;
  static constexpr size_t kInner = kN + sizeof(V) * kPH * kPW;
  static constexpr size_t kOuter = sizeof(double2) * kNH * kNW;   // residual round
  static constexpr size_t kBytes = kInner > kOuter ? kInner : kOuter;
};

// Partial sums of one thread's points in the inner precision T (FP32: the
// products and the four-point sums; the block and slot sums are FP64).
template <typename T, typename V>
__device__ __forceinline__ void cocg_dots_t(T (&s)[kNDots], V p, V r, V q) {
  s[0] += p.x * q.x - p.y * q.y;
  s[1] += p.x * q.y + p.y * q.x;
  s[2] += q.x * r.x - q.y * r.y;
  s[3] += q.x * r.y + q.y * r.x;
  s[4] += q.x * q.x - q.y * q.y;
  s[5] += T(2) * q.x * q.y;
  s[6] += r.x * r.x - r.y * r.y;
  s[7] += T(2) * r.x * r.y;
  s[8] += r.x * r.x + r.y * r.y;
}


// Flat tile mapping (element k of a tile to thread k mod 256): used for the
// FP64 inner precision, where it measured faster than the row mapping below;
// it takes the d updates of DMode (deferred every other step).
constexpr int kRing = kNW * kNH - kTX * kTY;  // halo-2 ring points
__device__ __forceinline__ void ring_pos(int e, int& y, int& x) {
  // rows 0,1 and kNH-2, kNH-1 (full width), then columns 0,1,kNW-2,kNW-1
  if (e < 2 * kNW) {
    y = e / kNW;
    x = e - y * kNW;
  } else if (e < 4 * kNW) {
    e -= 2 * kNW;
    y = kNH - 2 + e / kNW;
    x = e - (e / kNW) * kNW;
  } else {
    e -= 4 * kNW;
    y = 2 + (e >> 2);
    const int c = e & 3;
    x = (c < 2) ? c : kNW - 4 + c;
  }
}

template <typename T>
__device__ __forceinline__ void cocg_inner_flat(const Eng& e, const SlotCtl& c, int slot, int tile, unsigned char* lds,
                                           T (&a)[kNDots]) {
  using V = typename C2<T>::t;
  V* PN = reinterpret_cast<V*>(lds);
  V* PT = reinterpret_cast<V*>(lds + PassLds<T>::kN);
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const V* rs = reinterpret_cast<const V*>(c.par ? e.r1 : e.r0) + base;
  V* rd = reinterpret_cast<V*>(c.par ? e.r0 : e.r1) + base;
  const V* ps = reinterpret_cast<const V*>(c.par ? e.p1 : e.p0) + base;
  V* pd = reinterpret_cast<V*>(c.par ? e.p0 : e.p1) + base;
  V* d = reinterpret_cast<V*>(e.d) + base;
  double2* x64 = e.x64 + base;
  const bool first = c.it_inner == 0;        // d restarts this step
  const bool fold = first && c.rounds >= 2;  // ... after x64 += d
  const bool skip = c.dmode == kDSkip;       // d is left alone this step
  const V alpha = mk<V>(c.alpha.x, c.alpha.y);
  const V beta = mk<V>(c.beta.x, c.beta.y);
  const V zeta = mk<V>(c.zeta.x, c.zeta.y);
  const V dcp = mk<V>(c.dcp.x, c.dcp.y), dcr = mk<V>(c.dcr.x, c.dcr.y);
  const T cx = T(c.cx), cy = T(c.cy);
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * kTY;
  const bool big = (nx >= kPW) && (ny >= kPH);

  // every global load of the step is issued before the first wait:
  // r and d (interior), r (halo-2 ring) and p (halo 4) into registers
  size_t gi[kTY / 4];
  V rv[kTY / 4], dv[kTY / 4];
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    gi[j] = size_t(wrapc(y0 + ty + 4 * j, ny, big)) * nx + wrapc(x0 + tx, nx, big);
    rv[j] = rs[gi[j]];
    if (!first && !skip) dv[j] = nt_load(&d[gi[j]]);
  }
  constexpr int kRingPerThread = (kRing + kNT - 1) / kNT;
  V rr_[kRingPerThread];
  int rly[kRingPerThread], rlx[kRingPerThread];
#pragma unroll
  for (int m = 0; m < kRingPerThread; ++m) {
    const int k = threadIdx.x + m * kNT;
    rly[m] = -1;
    if (k < kRing) {
      ring_pos(k, rly[m], rlx[m]);
      rr_[m] = rs[size_t(wrapc(y0 - 2 + rly[m], ny, big)) * nx + wrapc(x0 - 2 + rlx[m], nx, big)];
    }
  }
  TileRegs<V, kPH, kPW> pt;
  pt.fetch([&](int ly, int lx) {
    const unsigned g = unsigned(wrapc(y0 - 4 + ly, ny, big)) * unsigned(nx) + unsigned(wrapc(x0 - 4 + lx, nx, big)); return ps[g]; });
  __syncthreads();  // LDS of the previous work item is free
  pt.store(PT);
  __syncthreads();
  // interior: rows ty + 4j, column tx
  V rn[kTY / 4], pn[kTY / 4];
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    const int ly = ty + 4 * j;
    const bool in = (x0 + tx < nx) && (y0 + ly < ny);
    const V pc = PT[(ly + 4) * kPW + tx + 4];
    const V q = helm<V, T, kPW>(PT, ly + 4, tx + 4, cx, cy, zeta);
    const V r1 = csub(rv[j], cmul(alpha, q));
    const V p1 = cadd(r1, cmul(beta, pc));
    if (in) {
      if (fold) {
        // once per round: the previous round's correction moves into x64
        const V dold = d[gi[j]];
        const double2 xo = x64[gi[j]];
        x64[gi[j]] = make_double2(xo.x + double(dold.x), xo.y + double(dold.y));
      }
      if (!skip) {
        const V dd = cadd(cmul(dcp, pc), cmul(dcr, rv[j]));
        nt_store(first ? dd : cadd(dv[j], dd), &d[gi[j]]);
      }
      rd[gi[j]] = r1;
      pd[gi[j]] = p1;
    }
    PN[(ly + 2) * kNW + tx + 2] = p1;
    rn[j] = r1;
    pn[j] = p1;
  }
  // halo ring of p_{i+1}
#pragma unroll
  for (int m = 0; m < kRingPerThread; ++m) {
    if (rly[m] < 0) continue;
    const int ly = rly[m], lx = rlx[m];
    const V pc = PT[(ly + 2) * kPW + lx + 2];
    const V q = helm<V, T, kPW>(PT, ly + 2, lx + 2, cx, cy, zeta);
    PN[ly * kNW + lx] = cadd(csub(rr_[m], cmul(alpha, q)), cmul(beta, pc));
  }
  __syncthreads();
  // sums over the thread's four points (and over the wavefront) in T;
  // the block and slot sums are FP64
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    const int ly = ty + 4 * j;
    if (x0 + tx < nx && y0 + ly < ny) {
      const V qv = helm<V, T, kNW>(PN, ly + 2, tx + 2, cx, cy, zeta);
      cocg_dots_t(a, pn[j], rn[j], qv);
    }
  }
}

// Row mapping: used for the FP32 inner precision (every step updates d:
// the scalars never choose kDSkip for FP32 vectors).
template <typename T>
__device__ __forceinline__ void cocg_inner(const Eng& e, const SlotCtl& c, int slot, int tile, unsigned char* lds,
                                           T (&a)[kNDots]) {
  using V = typename C2<T>::t;
  V* PN = reinterpret_cast<V*>(lds);
  V* PT = reinterpret_cast<V*>(lds + PassLds<T>::kN);
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const V* rs = reinterpret_cast<const V*>(c.par ? e.r1 : e.r0) + base;
  V* rd = reinterpret_cast<V*>(c.par ? e.r0 : e.r1) + base;
  const V* ps = reinterpret_cast<const V*>(c.par ? e.p1 : e.p0) + base;
  V* pd = reinterpret_cast<V*>(c.par ? e.p0 : e.p1) + base;
  V* d = reinterpret_cast<V*>(e.d) + base;
  double2* x64 = e.x64 + base;
  const bool first = c.it_inner == 0;        // d restarts this step
  const bool fold = first && c.rounds >= 2;  // ... after x64 += d
  const V alpha = mk<V>(c.alpha.x, c.alpha.y);
  const V beta = mk<V>(c.beta.x, c.beta.y);
  const V zeta = mk<V>(c.zeta.x, c.zeta.y);
  const T cx = T(c.cx), cy = T(c.cy);
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * kTY;
  const bool big = (nx >= kPW) && (ny >= kPH);

  // Thread (tx, wave w) owns column x0 + tx of rows w, w + 4, w + 8, w + 12;
  // a row is uniform across a wavefront, so row offsets live in scalar
  // registers and one column offset serves every load of the thread.
  const int w = __builtin_amdgcn_readfirstlane(ty);
  const unsigned col = unsigned(wrapc(x0 + tx, nx, big));
  auto row_off = [&](int y) { return size_t(wrapc(y, ny, big)) * size_t(nx); };
  // every global load of the step is issued before the first wait:
  // r and d (interior), r (halo-2 ring) and p (halo 4) into registers
  size_t ro[kTY / 4];
  V rv[kTY / 4], dv[kTY / 4];
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    ro[j] = row_off(y0 + w + 4 * j);
    rv[j] = (rs + ro[j])[col];
    if (!first) dv[j] = nt_load(&(d + ro[j])[col]);
  }
  // ring of the halo-2 tile: rows 0, 1, kNH-2, kNH-1 at columns 2..65 (one
  // per thread: row index w -> 0, 1, kNH-2, kNH-1), and columns 0, 1,
  // kNW-2, kNW-1 of all kNH rows (threads 0..4 kNH-1)
  const int rrow = (w < 2) ? w : kNH - 4 + w;
  const V rtop = (rs + row_off(y0 - 2 + rrow))[col];
  const bool side = threadIdx.x < 4 * kNH;
  const int sly = threadIdx.x >> 2, sc = threadIdx.x & 3;
  const int slx = (sc < 2) ? sc : kNW - 4 + sc;
  V rside;
  if (side) rside = rs[row_off(y0 - 2 + sly) + unsigned(wrapc(x0 - 2 + slx, nx, big))];
  // p with halo 4: rows w + 4m at columns 4..67 of the tile, and the 8 halo
  // columns of all kPH rows (threads 0..8 kPH-1)
  V pm[kPH / 4];
#pragma unroll
  for (int m = 0; m < kPH / 4; ++m) pm[m] = (ps + row_off(y0 - 4 + w + 4 * m))[col];
  const bool pside = threadIdx.x < 8 * kPH;
  const int ply = threadIdx.x >> 3, pc8 = threadIdx.x & 7;
  const int plx = (pc8 < 4) ? pc8 : kTX + pc8;
  V pside_v, pside_w;
  if (pside) pside_v = ps[row_off(y0 - 4 + ply) + unsigned(wrapc(x0 - 4 + plx, nx, big))];
  // taller tiles: the side columns need a second element for some threads
  constexpr int kPSide2 = 8 * kPH - kNT;
  if (kPSide2 > 0 && int(threadIdx.x) < kPSide2)
    pside_w = ps[row_off(y0 - 4 + ply + kNT / 8) + unsigned(wrapc(x0 - 4 + plx, nx, big))];
  __syncthreads();  // LDS of the previous work item is free
#pragma unroll
  for (int m = 0; m < kPH / 4; ++m) PT[(w + 4 * m) * kPW + tx + 4] = pm[m];
  if (pside) PT[ply * kPW + plx] = pside_v;
  if (kPSide2 > 0 && int(threadIdx.x) < kPSide2) PT[(ply + kNT / 8) * kPW + plx] = pside_w;
  __syncthreads();
  // interior: rows w + 4j, column tx
  V rn[kTY / 4], pn[kTY / 4];
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    const int ly = w + 4 * j;
    const bool in = (x0 + tx < nx) && (y0 + ly < ny);
    const V pc = PT[(ly + 4) * kPW + tx + 4];
    const V q = helm<V, T, kPW>(PT, ly + 4, tx + 4, cx, cy, zeta);
    const V r1 = csub(rv[j], cmul(alpha, q));
    const V p1 = cadd(r1, cmul(beta, pc));
    if (in) {
      if (fold) {
        // once per round: the previous round's correction moves into x64
        const V dold = (d + ro[j])[col];
        const double2 xo = (x64 + ro[j])[col];
        (x64 + ro[j])[col] = make_double2(xo.x + double(dold.x), xo.y + double(dold.y));
      }
      nt_store(first ? cmul(alpha, pc) : cadd(dv[j], cmul(alpha, pc)), &(d + ro[j])[col]);
      (rd + ro[j])[col] = r1;
      (pd + ro[j])[col] = p1;
    }
    PN[(ly + 2) * kNW + tx + 2] = p1;
    rn[j] = r1;
    pn[j] = p1;
  }
  // halo ring of p_{i+1}
  {
    const V pc = PT[(rrow + 2) * kPW + tx + 4];
    const V q = helm<V, T, kPW>(PT, rrow + 2, tx + 4, cx, cy, zeta);
    PN[rrow * kNW + tx + 2] = cadd(csub(rtop, cmul(alpha, q)), cmul(beta, pc));
  }
  if (side) {
    const V pc = PT[(sly + 2) * kPW + slx + 2];
    const V q = helm<V, T, kPW>(PT, sly + 2, slx + 2, cx, cy, zeta);
    PN[sly * kNW + slx] = cadd(csub(rside, cmul(alpha, q)), cmul(beta, pc));
  }
  __syncthreads();
  // sums over the thread's four points (and over the wavefront) in T;
  // the block and slot sums are FP64
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    const int ly = w + 4 * j;
    if (x0 + tx < nx && y0 + ly < ny) {
      const V qv = helm<V, T, kNW>(PN, ly + 2, tx + 2, cx, cy, zeta);
      cocg_dots_t(a, pn[j], rn[j], qv);
    }
  }
}

template <typename T>
__device__ __forceinline__ void cocg_residual(const Eng& e, const SlotCtl& c, int slot, int tile, unsigned char* lds,
                                              double& n2) {
  using V = typename C2<T>::t;
  double2* XT = reinterpret_cast<double2*>(lds);  // x = x64 + d with halo 2, FP64
  const int tx = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const double2* x64 = e.x64 + base;
  const V* d = reinterpret_cast<const V*>(e.d) + base;
  // r and p of the current parity: no other block reads them in this launch
  V* rc = reinterpret_cast<V*>(c.par ? e.r1 : e.r0) + base;
  V* pc = reinterpret_cast<V*>(c.par ? e.p1 : e.p0) + base;
  const bool zero_x = c.rounds == 0;  // fresh solve: x = 0, d holds nothing
  // right-hand side b = eta0 + a1 D0 + a2 Z0 (a second read of the slot
  // record: the fields are needed only here)
  const SlotWords sw(&e.slots[slot]);
  const double2 a1 = sw.c64(SLOT_OFF(a1)), a2 = sw.c64(SLOT_OFF(a2));
  const double* eta0 = sw.ptr<const double>(SLOT_OFF(eta0));
  const double* D0 = sw.ptr<const double>(SLOT_OFF(D0));
  const double* Z0 = sw.ptr<const double>(SLOT_OFF(Z0));
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * kTY;
  const bool big = (nx >= kPW) && (ny >= kPH);
  const unsigned col = unsigned(wrapc(x0 + tx, nx, big));
  // the right-hand side fields first (pure loads), then x = x64 + d with
  // halo 2, formed as it arrives: every load is issued before the first wait
  double bv[kTY / 4], dz[kTY / 4], zz[kTY / 4];
  size_t ro[kTY / 4];
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    ro[j] = size_t(wrapc(y0 + w + 4 * j, ny, big)) * size_t(nx);
    bv[j] = (eta0 + ro[j])[col];
    if (D0) {
      dz[j] = (D0 + ro[j])[col];
      zz[j] = (Z0 + ro[j])[col];
    }
  }
  RowTile<double2, 2> xr;
  if (!zero_x) xr.fetch(x0, y0, nx, ny, big, [&](size_t rofs, unsigned cx_) {
    const size_t g = rofs + cx_;
    const V dv = d[g];
    const double2 xv = x64[g];
    return make_double2(xv.x + double(dv.x), xv.y + double(dv.y));
  });
  __syncthreads();  // LDS of the previous work item is free
  if (!zero_x) xr.store(XT);
  __syncthreads();
  // r64 = b - (L - zeta) x on the tile; r = p = (T) r64
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    const int ly = w + 4 * j;
    if (x0 + tx < nx && y0 + ly < ny) {
      double2 rv = make_double2(bv[j], 0.0);
      if (D0) {
        rv.x += a1.x * dz[j] + a2.x * zz[j];
        rv.y += a1.y * dz[j] + a2.y * zz[j];
      }
      if (!zero_x) rv = csub(rv, helm<double2, double, kNW>(XT, ly + 2, tx + 2, c.cx, c.cy, c.zeta));
      const V rt = mk<V>(rv.x, rv.y);
      (rc + ro[j])[col] = rt;
      (pc + ro[j])[col] = rt;
      n2 += rv.x * rv.x + rv.y * rv.y;
    }
  }
}

// First step of an inner solve: p = r (the rounded residual), q = (L - zeta) p
// on the tile (r with halo 2 from LDS) and the COCG partial sums, in FP64
// (alpha and beta of the first step set the course of the whole inner solve:
// FP32 sums here slowed the hardest solves several-fold).
template <typename T>
__device__ __forceinline__ void cocg_prime(const Eng& e, const SlotCtl& c, int slot, int tile, unsigned char* lds,
                                           double (&a)[kNDots]) {
  using V = typename C2<T>::t;
  V* RN = reinterpret_cast<V*>(lds);
  const int tx = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nx = c.nx, ny = c.ny;
  const size_t base = size_t(slot) * e.cap;
  const V* rc = reinterpret_cast<const V*>(c.par ? e.r1 : e.r0) + base;
  const V zeta = mk<V>(c.zeta.x, c.zeta.y);
  const T cx = T(c.cx), cy = T(c.cy);
  const int x0 = (tile % c.tiles_x) * kTX, y0 = (tile / c.tiles_x) * kTY;
  const bool big = (nx >= kPW) && (ny >= kPH);
  TileRegs<V, kNH, kNW> rr;
  rr.fetch([&](int ly, int lx) {
    return rc[unsigned(wrapc(y0 - 2 + ly, ny, big)) * unsigned(nx) + unsigned(wrapc(x0 - 2 + lx, nx, big))];
  });
  __syncthreads();  // LDS of the previous work item is free
  rr.store(RN);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kTY / 4; ++j) {
    const int ly = w + 4 * j;
    if (x0 + tx < nx && y0 + ly < ny) {
      const V rt = RN[(ly + 2) * kNW + tx + 2];
      const V q = helm<V, T, kNW>(RN, ly + 2, tx + 2, cx, cy, zeta);
      cocg_dots_t(a, make_double2(rt.x, rt.y), make_double2(rt.x, rt.y), make_double2(q.x, q.y));
    }
  }
}

template <typename T>
__device__ __forceinline__ void cocg_pass(const Eng& e) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[PassLds<T>::kBytes];
  __shared__ double red[4 * kNDots];
  const WorkMap m = load_work_map(e);
  const int span = work_span(m);
  for (int w = blockIdx.x; w < span; w += gridDim.x) {
    Item it;
    if (!work_item(e, m, w, it)) continue;
    const SlotCtl c = load_ctl(&e.slots[it.slot]);
    if (c.status == kInner) {
      T a[kNDots];
#pragma unroll
      for (int k = 0; k < kNDots; ++k) a[k] = T(0);
      if (sizeof(T) == 4)
        cocg_inner<T>(e, c, it.slot, it.tile, lds, a);
      else
        cocg_inner_flat<T>(e, c, it.slot, it.tile, lds, a);
      store_block_sums<kNDots>(a, red, item_part(e, it.slot, it.tile));
    } else if (c.status == kPrime) {
      double a[kNDots];
#pragma unroll
      for (int k = 0; k < kNDots; ++k) a[k] = 0.0;
      cocg_prime<T>(e, c, it.slot, it.tile, lds, a);
      store_block_sums<kNDots>(a, red, item_part(e, it.slot, it.tile));
    } else if (c.status == kOuterPending || c.status == kInnerDone) {
      double n2[1] = {0.0};
      cocg_residual<T>(e, c, it.slot, it.tile, lds, n2[0]);
      store_block_sums<1, 8>(n2, red, item_part(e, it.slot, it.tile));
    }
  }
}

// FP32 inner precision at 5 waves per SIMD (<= 96 VGPRs); FP64 as compiled
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(5))) void k_pass_f32(Eng e) {
  cocg_pass<float>(e);
}
__global__ __launch_bounds__(kNT) void k_pass_f64(Eng e) { cocg_pass<double>(e); }

// One block per slot after each pass: add the partial sums of the slot's
// tiles in index order.  Inner step: set alpha_{i+1}, beta_{i+1} or end the
// inner solve.  Residual step: decide done / stagnated / failed, or go on
// to a prime step.  Prime step: alpha, beta of the first inner step.
__global__ __launch_bounds__(kSNT) void k_pass_scalars(Eng e) {
  __shared__ double red[kSNT / 64 * kNDots];
  Slot* S = &e.slots[blockIdx.x];
  const int status = ldc(&S->status);
  const bool outer = (status == kOuterPending || status == kInnerDone);
  if (status != kInner && status != kPrime && !outer) return;
  double tot[kNDots];
  slot_sums_n<kNDots>(e.part + size_t(blockIdx.x) * e.cap_blk * kNDots, ldc(&S->nblk), tot, red);
  if (threadIdx.x != 0) return;
  const double n2 = tot[8];
  if (outer) {
    // n2 is the FP64 residual |b - K x|^2 of the current iterate
    const int rounds0 = ldc(&S->rounds);
    double bn2 = ldc(&S->bn2);
    if (rounds0 == 0) {
      bn2 = n2;
      S->bn2 = n2;
    }
    const int rounds = rounds0 + 1;
    S->rounds = rounds;
    const double prev = ldc(&S->prev_rn2);
    const double ref2 = ldc(&S->ref2);
    // stop threshold on |b - K x|^2: tol2 times the fixed reference, or
    // times |b|^2 (relative residual)
    const double thr = ldc(&S->tol2) * (ref2 > 0.0 ? ref2 : bn2);
    S->rn2 = n2;
    S->prev_rn2 = n2;
    const bool capped = ldc(&S->it_total) >= ldc(&S->max_it);
    if (!isfinite(n2)) {
      // an inner round went non-finite: in mixed precision the solve is run
      // again in FP64
      S->status = e.retry ? kRetry : kFailBreakdown;
    } else if (n2 <= thr) {
      S->status = kDone;
    } else if (rounds >= 3 && n2 > 0.25 * prev) {
      // a whole inner solve did not halve the FP64 residual.  In mixed
      // precision the FP32 inner solves stalled or diverged: FP64 retry.  In
      // FP64 the iterate sits at its rounding floor, above the requested
      // tolerance; the achieved residual enters the reported error bound.
      if (e.retry) {
        S->status = kRetry;
      } else {
        S->status = kDone;
        S->stagnated = 1;
        if (n2 > prev) {
          // the last correction made the iterate worse (an inner solve that
          // diverged): x64 holds the previous iterate, of residual prev
          S->discard = 1;
          S->rn2 = prev;
        }
      }
    } else if (capped) {
      S->status = e.retry ? kRetry : kFailMaxIter;
    } else {
      S->status = kPrime;
      S->it_inner = 0;
      // the requested reduction of this residual, never below a quarter of
      // the final tolerance
      S->in_tol2 = fmax(e.inner_eta2 * n2, 0.0625 * thr);
    }
    return;
  }
  const double2 pq = make_double2(tot[0], tot[1]);
  const double2 qr = make_double2(tot[2], tot[3]);
  const double2 qq = make_double2(tot[4], tot[5]);
  const double2 rr = make_double2(tot[6], tot[7]);
  const bool ok = finite2(pq) && finite2(qr) && finite2(qq) && finite2(rr) && (fabs(pq.x) + fabs(pq.y) > 0.0) &&
                  (fabs(rr.x) + fabs(rr.y) > 0.0);
  // alpha and beta of the next step from the sums of this one
  auto next_scalars = [&](double2& al, double2& be) {
    al = cdiv(rr, pq);
    // rr_{i+2} = rr - 2 alpha qr + alpha^2 qq
    const double2 a2 = make_double2(al.x * al.x - al.y * al.y, 2.0 * al.x * al.y);
    const double2 aqr = make_double2(al.x * qr.x - al.y * qr.y, al.x * qr.y + al.y * qr.x);
    const double2 aqq = make_double2(a2.x * qq.x - a2.y * qq.y, a2.x * qq.y + a2.y * qq.x);
    const double2 rr2 = make_double2(rr.x - 2.0 * aqr.x + aqq.x, rr.y - 2.0 * aqr.y + aqq.y);
    be = cdiv(rr2, rr);
  };
  double2 al, be;
  if (status == kPrime) {
    if (!ok) {
      S->status = e.retry ? kRetry : kFailBreakdown;
      return;
    }
    S->status = kInner;
    next_scalars(al, be);
    // the first step of a round restarts d = alpha p
    S->dmode = kDUpdate;
    S->fin = 0;
    S->dcp = al;
    S->dcr = make_double2(0.0, 0.0);
  } else {
    // inner step: r and p were written to the other buffers
    S->parity = ldc(&S->parity) ^ 1;
    S->it_inner = ldc(&S->it_inner) + 1;
    const int it_total = ldc(&S->it_total) + 1;
    S->it_total = it_total;
    const bool skipped = ldc(&S->dmode) == kDSkip;
    if (skipped) S->skips = ldc(&S->skips) + 1;
    // alpha_i / beta_i of the step just taken, for a deferred update
    const double2 ab = skipped ? cdiv(ldc(&S->alpha), ldc(&S->beta)) : make_double2(0.0, 0.0);
    const bool good = ok && isfinite(n2);
    if (!good || n2 <= ldc(&S->in_tol2) || it_total >= ldc(&S->max_it) || ldc(&S->fin)) {
      if (!skipped) {
        S->status = kInnerDone;
        S->fin = 0;
        return;
      }
      // one more step adds the deferred term to d, then the round ends
      // (with alpha = beta = 0 if the scalars are unusable: only d changes)
      if (good) {
        next_scalars(al, be);
      } else {
        al = be = make_double2(0.0, 0.0);
      }
      S->alpha = al;
      S->beta = be;
      S->rr = rr;
      S->dmode = kDUpdate;
      S->dcp = make_double2(al.x + ab.x, al.y + ab.y);
      S->dcr = make_double2(-ab.x, -ab.y);
      S->fin = 1;
      return;
    }
    next_scalars(al, be);
    if (skipped) {
      S->dmode = kDUpdate;
      S->dcp = make_double2(al.x + ab.x, al.y + ab.y);
      S->dcr = make_double2(-ab.x, -ab.y);
    } else if (!e.d_is_f32 && be.x * be.x + be.y * be.y >= kDeferBeta * kDeferBeta) {
      S->dmode = kDSkip;
    } else {
      S->dmode = kDUpdate;
      S->dcp = al;
      S->dcr = make_double2(0.0, 0.0);
    }
  }
  S->alpha = al;
  S->beta = be;
  S->rr = rr;
}

// ---------------------------------------------------------------------------
// scheduler
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finished(int st) {
  return st == kDone || st == kFailMaxIter || st == kFailBreakdown || st == kRetry;
}

// Exclusive prefix sum of one int per thread over a block of kSchedNT
// threads (4 wavefronts); *total receives the block total.
constexpr int kSchedNT = 256;
constexpr int kSchedPer = kMaxSlots / kSchedNT;  // slots per thread
__device__ __forceinline__ int block_scan_excl(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();  // sh free
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  int off = 0;
  for (int k = 0; k < wid; ++k) off += sh[k];
  *total = sh[0] + sh[1] + sh[2] + sh[3];
  return off + x - v;
}

// Finished slots, in index order, into list[0 .. *n) (whole block).
__device__ __forceinline__ void finished_slots(const Eng& e, int* list, int* sh, int* n) {
  int st[kSchedPer];
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < kSchedPer; ++j) {
    const int s = threadIdx.x * kSchedPer + j;
    st[j] = (s < e.B) ? ldc(&e.slots[s].status) : kIdle;
    cnt += finished(st[j]) ? 1 : 0;
  }
  int pos = block_scan_excl(cnt, sh, n);
#pragma unroll
  for (int j = 0; j < kSchedPer; ++j)
    if (finished(st[j])) list[pos++] = threadIdx.x * kSchedPer + j;
  __syncthreads();
}

// Finished slots: A[inst] += Re(c_j x64) (or copy x64 out), then x64 = 0.
// Each point walks the finished slots in index order.
__global__ __launch_bounds__(kSchedNT) void k_retire(Eng e) {
  if (ldc(&e.counter[3]) == 0) return;  // nothing finished in the previous chunk
  __shared__ int list[kMaxSlots];
  __shared__ int sh[4];
  int nfin = 0;
  finished_slots(e, list, sh, &nfin);
  for (int q = 0; q < nfin; ++q) {
    const int s = list[q];
    const Slot* S = &e.slots[s];
    const Inst I = ld_inst(&e.inst[ldc(&S->inst)]);
    const int n = I.nx * I.ny;
    if (ldc(&S->status) == kRetry) {
      // solved again in FP64 by the host: nothing is kept from this attempt
      for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        e.x64[size_t(s) * e.cap + i] = make_double2(0.0, 0.0);
      continue;
    }
    // the last inner correction d is still to be added (once the solve has
    // run an inner round)
    const bool add_d = ldc(&S->rounds) >= 2 && ldc(&S->discard) == 0;
    const int sv = ldc(&S->solve);
    const double2 c0 = ldc(&e.solves[sv].c0), c1 = ldc(&e.solves[sv].c1), c2 = ldc(&e.solves[sv].c2);
    const size_t yrow = e.yout ? size_t(ldc(&e.solves[sv].yidx)) * e.ystride : 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      double2* xp = e.x64 + size_t(s) * e.cap + i;
      double2 x = *xp;
      if (add_d) {
        if (e.d_is_f32) {
          const float2 dv = reinterpret_cast<const float2*>(e.d)[size_t(s) * e.cap + i];
          x.x += double(dv.x);
          x.y += double(dv.y);
        } else {
          const double2 dv = reinterpret_cast<const double2*>(e.d)[size_t(s) * e.cap + i];
          x.x += dv.x;
          x.y += dv.y;
        }
      }
      if (e.yout) e.yout[yrow + i] = x;
      I.A[i] += c0.x * x.x - c0.y * x.y;
      I.A[n + i] += c1.x * x.x - c1.y * x.y;
      I.A[2 * n + i] += c2.x * x.x - c2.y * x.y;
      *xp = make_double2(0.0, 0.0);
    }
  }
}

// Next solve of the queue into slot s.
__device__ __forceinline__ void assign_solve(Eng& e, int s, int next) {
  Slot* S = &e.slots[s];
  const SolveDev* D = &e.solves[next];
  const int dinst = ldc(&D->inst);
  S->zeta = ldc(&D->zeta);
  S->a1 = ldc(&D->a1);
  S->a2 = ldc(&D->a2);
  S->gamma = ldc(&D->gamma);
  S->sc = ldc(&D->sc);
  S->omega = make_double2(0.0, 0.0);
  S->tol2 = ldc(&D->tol2);
  S->ref2 = ldc(&D->ref2);
  S->rr = S->alpha = S->beta = make_double2(0.0, 0.0);
  S->bn2 = S->rn2 = S->prev_rn2 = S->in_tol2 = 0.0;
  S->status = kOuterPending;
  S->parity = 0;
  S->prime = 0;
  S->it_total = S->it_inner = S->rounds = 0;
  S->solve = next;
  S->inst = dinst;
  const Inst* I = &e.inst[dinst];
  S->nx = ldc(&I->nx);
  S->ny = ldc(&I->ny);
  S->tiles_x = ldc(&I->tiles_x);
  S->nblk = ldc(&I->nblk);
  S->cx = ldc(&I->cx);
  S->cy = ldc(&I->cy);
  S->cxy = ldc(&I->cxy);
  S->H = ldc_ptr(&I->H);
  S->Hin = ldc_ptr(&I->Hin);
  S->eta0 = ldc_ptr(&I->eta0);
  S->D0 = ldc_ptr(&I->D0);
  S->Z0 = ldc_ptr(&I->Z0);
  S->stagnated = 0;
  S->discard = 0;
  S->max_it = ldc(&D->max_it);
  S->dcp = S->dcr = make_double2(0.0, 0.0);
  S->dmode = kDUpdate;
  S->fin = 0;
  S->skips = 0;
}

// One block: record finished solves, hand out the next ones in queue order
// (the k-th idle slot in index order takes queue entry next + k), rebuild
// the work list (working slots in index order, the common tile count if
// any) and the host-visible counts; then, when tile counts differ, write
// the (slot, tile) table of the work positions as 8 band lists (one per
// XCD).
// Every slot is handled by its own thread; the orders are those of a
// sequential walk over the slots.
__global__ __launch_bounds__(kSchedNT) void k_assign(Eng e) {
  __shared__ int sh[4];
  __shared__ int s_nb[kMaxSlots];
  __shared__ int s_bo[kMaxSlots];
  __shared__ int s_min, s_max;
  const int next0 = ldc(e.next);
#ifdef REXII_DEBUG_CHECKS
  if (threadIdx.x == 0) {
    int fin = 0;
    for (int s = 0; s < e.B; ++s) fin += finished(ldc(&e.slots[s].status)) ? 1 : 0;
    if (fin != ldc(&e.counter[3])) atomicAdd(&e.dbg[1], 1);
    if (fin > 0 && ldc(&e.counter[3]) == 0) atomicAdd(&e.dbg[2], 1);
  }
  __syncthreads();
#endif
  if (threadIdx.x == 0) {
    s_min = 1 << 30;
    s_max = 0;
  }
  int st[kSchedPer];
  int nidle = 0;
#pragma unroll
  for (int j = 0; j < kSchedPer; ++j) {
    const int s = threadIdx.x * kSchedPer + j;
    st[j] = -1;  // no such slot
    if (s >= e.B) continue;
    Slot* S = &e.slots[s];
    st[j] = ldc(&S->status);
    if (finished(st[j])) {
      SolveStat& ss = e.stats[ldc(&S->solve)];
      ss.rn2 = ldc(&S->rn2);
      ss.bn2 = ldc(&S->bn2);
      ss.it_total = ldc(&S->it_total);
      ss.rounds = ldc(&S->rounds);
      ss.status = st[j];
      ss.stagnated = ldc(&S->stagnated);
      ss.skips = ldc(&S->skips);
      st[j] = kIdle;
      S->status = kIdle;
    }
    nidle += (st[j] == kIdle) ? 1 : 0;
  }
  int total_idle = 0;
  int rank = block_scan_excl(nidle, sh, &total_idle);
  int nwork = 0, ntiles = 0, nband = 0;
  int nb[kSchedPer];
#pragma unroll
  for (int j = 0; j < kSchedPer; ++j) {
    const int s = threadIdx.x * kSchedPer + j;
    nb[j] = 0;
    if (st[j] < 0) continue;
    if (st[j] == kIdle) {
      const int q = next0 + rank++;
      if (q < e.S) {
        assign_solve(e, s, q);
        st[j] = kOuterPending;
        nb[j] = ldc(&e.inst[ldc(&e.solves[q].inst)].nblk);
      }
    } else {
      nb[j] = ldc(&e.inst[ldc(&e.slots[s].inst)].nblk);
    }
    if (st[j] != kIdle) {
      ++nwork;
      ntiles += nb[j];
      nband += (nb[j] + 7) >> 3;
    }
  }
  const int next = min(next0 + total_idle, e.S);
  int working = 0, total = 0, per = 0;
  int wpos = block_scan_excl(nwork, sh, &working);
  (void)block_scan_excl(ntiles, sh, &total);
  int bpos = block_scan_excl(nband, sh, &per);
  int lmin = 1 << 30, lmax = 0;
#pragma unroll
  for (int j = 0; j < kSchedPer; ++j) {
    const int s = threadIdx.x * kSchedPer + j;
    if (st[j] < 0) continue;
    s_bo[s] = bpos;
    s_nb[s] = (st[j] != kIdle) ? nb[j] : 0;
    if (st[j] != kIdle) {
      e.work[2 + wpos++] = s;
      bpos += (nb[j] + 7) >> 3;
      lmin = min(lmin, nb[j]);
      lmax = max(lmax, nb[j]);
    }
  }
  atomicMin(&s_min, lmin);
  atomicMax(&s_max, lmax);
  __syncthreads();
  const int uniform = (working > 0 && s_min == s_max) ? s_max : 0;
  if (threadIdx.x == 0) {
    // list length: the working tiles, or 8 band lists of per entries each
    e.work[0] = (uniform > 0) ? total : 8 * per;
    e.work[1] = uniform | ((working == e.B && uniform > 0) ? kWorkIdentity : 0);
    *e.next = next;
    e.counter[0] = working + (next < e.S ? 1 : 0);
    e.counter[1] = next;
  }
  if (uniform > 0) return;
  // band lists: list x holds band x of every working slot in slot order
  // (tiles x bs .. x bs + bs - 1, bs = ceil(nb / 8)); positions past a
  // slot's last tile hold slot -1
  for (int s = 0; s < e.B; ++s) {
    const int n = s_nb[s];
    if (n == 0) continue;
    const int bs = (n + 7) >> 3, bo = s_bo[s];
    for (int k = threadIdx.x; k < 8 * bs; k += blockDim.x) {
      const int x = k / bs, j = k - x * bs, t = x * bs + j;
      e.items[size_t(x) * per + bo + j] = (t < n) ? make_int2(s, t) : make_int2(-1, -1);
    }
  }
}

// Count of slots that finished during the chunk (read by the next retire).
__global__ __launch_bounds__(kSchedNT) void k_count_finished(Eng e) {
  __shared__ int sh[4];
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < kSchedPer; ++j) {
    const int s = threadIdx.x * kSchedPer + j;
    if (s < e.B) cnt += finished(ldc(&e.slots[s].status)) ? 1 : 0;
  }
  int fin = 0;
  (void)block_scan_excl(cnt, sh, &fin);
  if (threadIdx.x == 0) e.counter[3] = fin;
}

// ---------------------------------------------------------------------------
// problem-level kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_zero(double* p, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_copy(const double* s, double* d, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    d[i] = s[i];
}

// D0 = dx u0 + dy v0, Z0 = dx v0 - dy u0; flags: bit0 non-finite input,
// bit1 non-zero velocity, bit2 non-zero divergence
__global__ void k_prep(const double* f, int nx, int ny, double* D0, double* Z0, int* flags) {
  const size_t n = size_t(nx) * ny;
  int fl = 0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int y = int(i / nx), x = int(i - size_t(y) * nx);
    const double* u = f + n;
    const double* v = f + 2 * n;
    const double e = f[i], uu = u[i], vv = v[i];
    if (!isfinite(e) || !isfinite(uu) || !isfinite(vv)) fl |= 1;
    if (uu != 0.0 || vv != 0.0) fl |= 2;
    const size_t xp = size_t(y) * nx + (x + 1 == nx ? 0 : x + 1);
    const size_t xm = size_t(y) * nx + (x == 0 ? nx - 1 : x - 1);
    const size_t yp = size_t(y + 1 == ny ? 0 : y + 1) * nx + x;
    const size_t ym = size_t(y == 0 ? ny - 1 : y - 1) * nx + x;
    const double hx = 0.5 * nx, hy = 0.5 * ny;
    const double div = hx * (u[xp] - u[xm]) + hy * (v[yp] - v[ym]);
    const double curl = hx * (v[xp] - v[xm]) - hy * (u[yp] - u[ym]);
    D0[i] = div;
    Z0[i] = curl;
    if (div != 0.0) fl |= 4;
  }
  if (fl) atomicOr(flags, fl);
}

// u_eta = A0;  (u, v) = S1 (u0, v0) + S2 J(u0, v0) + t g (grad A1 + J grad A2),
// J(a, b) = (b, -a)
__global__ void k_reconstruct(const double* f, const double* A, int nx, int ny, double S1, double S2,
                              double tg, int has_vel, double* u) {
  const size_t n = size_t(nx) * ny;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int y = int(i / nx), x = int(i - size_t(y) * nx);
    const size_t xp = size_t(y) * nx + (x + 1 == nx ? 0 : x + 1);
    const size_t xm = size_t(y) * nx + (x == 0 ? nx - 1 : x - 1);
    const size_t yp = size_t(y + 1 == ny ? 0 : y + 1) * nx + x;
    const size_t ym = size_t(y == 0 ? ny - 1 : y - 1) * nx + x;
    const double hx = 0.5 * nx, hy = 0.5 * ny;
    const double* A1 = A + n;
    const double* A2 = A + 2 * n;
    const double a1x = hx * (A1[xp] - A1[xm]), a1y = hy * (A1[yp] - A1[ym]);
    const double a2x = hx * (A2[xp] - A2[xm]), a2y = hy * (A2[yp] - A2[ym]);
    double uu = tg * (a1x + a2y), vv = tg * (a1y - a2x);
    if (has_vel) {
      const double u0 = f[n + i], v0 = f[2 * n + i];
      uu += S1 * u0 + S2 * v0;
      vv += S1 * v0 - S2 * u0;
    }
    u[i] = A[i];
    u[n + i] = uu;
    u[2 * n + i] = vv;
  }
}

// Full per-pole solution x = (eta, u, v) from the Helmholtz solution y:
// eta = y / sigma, (u, v) = M ((u0, v0) + t g grad eta), M = m1 I + m2 J.
__global__ void k_expand(const double2* y, const double* f, int nx, int ny, double2 is, double2 M1, double2 M2,
                         double tg, int has_vel, double2* o) {
  const size_t n = size_t(nx) * ny;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int yy = int(i / nx), x = int(i - size_t(yy) * nx);
    const size_t xp = size_t(yy) * nx + (x + 1 == nx ? 0 : x + 1);
    const size_t xm = size_t(yy) * nx + (x == 0 ? nx - 1 : x - 1);
    const size_t yp = size_t(yy + 1 == ny ? 0 : yy + 1) * nx + x;
    const size_t ym = size_t(yy == 0 ? ny - 1 : yy - 1) * nx + x;
    const double hx = 0.5 * nx, hy = 0.5 * ny;
    const double2 gx = cmul(is, csub(y[xp], y[xm])), gy = cmul(is, csub(y[yp], y[ym]));
    double2 wu = make_double2(tg * hx * gx.x, tg * hx * gx.y);
    double2 wv = make_double2(tg * hy * gy.x, tg * hy * gy.y);
    if (has_vel) {
      wu.x += f[n + i];
      wv.x += f[2 * n + i];
    }
    o[i] = cmul(is, y[i]);
    o[n + i] = cadd(cmul(M1, wu), cmul(M2, wv));
    o[2 * n + i] = csub(cmul(M1, wv), cmul(M2, wu));
  }
}

__global__ void k_scale3(const double* src, double* dst, size_t n, double s0, double s1, double s2) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    dst[i] = s0 * src[i];
    dst[n + i] = s1 * src[n + i];
    dst[2 * n + i] = s2 * src[2 * n + i];
  }
}

// partial sums of the adjoint dots: block b of dot k covers points
// b, b + nblk*256, ... (fixed assignment), then a fixed-order reduction
__global__ __launch_bounds__(256) void k_adj_dots(const AdjDot* dd, const double2* yout, int cap, const double* eta0,
                                                  const double* D0, const double* Z0, int nx, int ny, double tg,
                                                  int has_vel, double2* part, int nblk) {
  __shared__ double red[8];
  const AdjDot a = dd[blockIdx.y];
  const size_t n = size_t(nx) * ny;
  const double2* y = yout + size_t(a.jf) * cap;
  const double2* ya = yout + size_t(a.ja) * cap;
  double sr = 0.0, si = 0.0;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(nblk) * 256) {
    double2 r = make_double2(eta0[i], 0.0);
    double2 div = make_double2(0.0, 0.0);
    if (has_vel) {
      const double dv = D0[i], zv = Z0[i];
      r.x += a.a1.x * dv + a.a2.x * zv;
      r.y += a.a1.y * dv + a.a2.y * zv;
      div.x = a.m1.x * dv + a.m2.x * zv;
      div.y = a.m1.y * dv + a.m2.y * zv;
    }
    const double2 ly = cmul(cadd(r, cmul(a.zeta, y[i])), a.isig);   // L eta
    const double2 t = cmul(a.m1, ly);
    div.x += tg * t.x;
    div.y += tg * t.y;
    double2 yy = ya[i];
    if (a.conj) yy.y = -yy.y;
    const double2 Y = cmul(yy, a.ysc);
    sr += Y.x * div.x - Y.y * div.y;
    si += Y.x * div.y + Y.y * div.x;
  }
  double v[2] = {sr, si}, tot[2];
  block_sum_n<2>(v, red, tot);
  if (threadIdx.x == 0) part[size_t(blockIdx.y) * nblk + blockIdx.x] = make_double2(tot[0], tot[1]);
}

__global__ __launch_bounds__(256) void k_adj_reduce(const double2* part, int nblk, double2* out) {
  __shared__ double red[8];
  double v[2] = {0.0, 0.0}, tot[2];
  for (int b = threadIdx.x; b < nblk; b += 256) {
    v[0] += part[size_t(blockIdx.x) * nblk + b].x;
    v[1] += part[size_t(blockIdx.x) * nblk + b].y;
  }
  block_sum_n<2>(v, red, tot);
  if (threadIdx.x == 0) out[blockIdx.x] = make_double2(tot[0], tot[1]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
__global__ void k_scale1(double* p, size_t n, double v) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) p[i] *= v;
}
void launch_scale1(double* p, size_t n, double v, hipStream_t s) {
  size_t bl = (n + 255) / 256;
  hipLaunchKernelGGL(k_scale1, dim3(unsigned(bl > 8192 ? 8192 : (bl < 1 ? 1 : bl))), dim3(256), 0, s, p, n, v);
}
void launch_scale3(const double* src, double* dst, size_t n, double s0, double s1, double s2, hipStream_t s) {
  size_t bl = (n + 255) / 256;
  hipLaunchKernelGGL(k_scale3, dim3(unsigned(bl > 8192 ? 8192 : (bl < 1 ? 1 : bl))), dim3(256), 0, s, src, dst, n,
                     s0, s1, s2);
}
int adj_dot_blocks(size_t n) {
  size_t b = (n + 255) / 256;
  return int(b > 64 ? 64 : (b < 1 ? 1 : b));
}
void launch_adj_dots(const AdjDot* d, int nd, const double2* yout, int cap, const double* eta0, const double* D0,
                     const double* Z0, int nx, int ny, double tg, int has_vel, double2* part, int nblk, double2* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_adj_dots, dim3(nblk, nd), dim3(256), 0, s, d, yout, cap, eta0, D0, Z0, nx, ny, tg, has_vel,
                     part, nblk);
  hipLaunchKernelGGL(k_adj_reduce, dim3(nd), dim3(256), 0, s, part, nblk, out);
}
constexpr int kWnBlocks = 256;
__global__ __launch_bounds__(256) void k_wnorm2(const double* f, const double* H, double H0, double g, size_t n,
                                                double* part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(kWnBlocks) * 256) {
    const double eta = f[i], u = f[n + i], v = f[2 * n + i];
    const double h = H ? H[i] : H0;
    acc += g * eta * eta + h * (u * u + v * v);
  }
  double v[1] = {acc}, tot[1];
  block_sum_n<1>(v, red, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot[0];
}
int wnorm_blocks() { return kWnBlocks; }
void launch_wnorm2(const double* f, const double* H, double H0, double g, size_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_wnorm2, dim3(kWnBlocks), dim3(256), 0, s, f, H, H0, g, n, part);
}

static inline unsigned flat_blocks(size_t n) {
  size_t bl = (n + 255) / 256;
  return unsigned(bl > 8192 ? 8192 : (bl < 1 ? 1 : bl));
}

template <typename T>
void launch_pass(const Eng& e, int grid, hipStream_t s) {
  if (sizeof(T) == 4)
    hipLaunchKernelGGL(k_pass_f32, dim3(grid), dim3(kNT), 0, s, e);
  else
    hipLaunchKernelGGL(k_pass_f64, dim3(grid), dim3(kNT), 0, s, e);
}
void launch_pass_scalars(const Eng& e, hipStream_t s) {
  hipLaunchKernelGGL(k_pass_scalars, dim3(e.B), dim3(kSNT), 0, s, e);
}
void launch_retire(const Eng& e, hipStream_t s) {
  hipLaunchKernelGGL(k_retire, dim3(flat_blocks(size_t(e.cap))), dim3(kSchedNT), 0, s, e);
}
void launch_assign(const Eng& e, hipStream_t s) {
  hipLaunchKernelGGL(k_assign, dim3(1), dim3(kSchedNT), 0, s, e);
}
void launch_count_finished(const Eng& e, hipStream_t s) {
  hipLaunchKernelGGL(k_count_finished, dim3(1), dim3(kSchedNT), 0, s, e);
}
void launch_fill_zero(double* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(flat_blocks(n)), dim3(256), 0, s, p, n);
}
void launch_copy(const double* src, double* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(flat_blocks(n)), dim3(256), 0, s, src, dst, n);
}
void launch_prep(const double* f, int nx, int ny, double* D0, double* Z0, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(flat_blocks(size_t(nx) * ny)), dim3(256), 0, s, f, nx, ny, D0, Z0, flags);
}
void launch_reconstruct(const double* f, const double* A, int nx, int ny, double S1, double S2, double tg,
                        int has_vel, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_reconstruct, dim3(flat_blocks(size_t(nx) * ny)), dim3(256), 0, s, f, A, nx, ny, S1, S2, tg,
                     has_vel, u);
}
void launch_expand(const double2* y, const double* f, int nx, int ny, double2 is, double2 m1, double2 m2,
                   double tg, int has_vel, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_expand, dim3(flat_blocks(size_t(nx) * ny)), dim3(256), 0, s, y, f, nx, ny, is, m1, m2, tg,
                     has_vel, out);
}

int pass_occupancy(int mixed) {
  int occ = 0;
  hipError_t err = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_pass_f32, kNT, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_pass_f64, kNT, 0);
  return err == hipSuccess ? occ : 1;
}

template void launch_pass<float>(const Eng&, int, hipStream_t);
template void launch_pass<double>(const Eng&, int, hipStream_t);

}  // namespace rexii
