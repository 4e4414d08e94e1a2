// gfx950 kernels of the REXII shifted-solve path (see kernels.h for the
// mathematics).  All reductions are deterministic: every block writes one
// partial in a fixed order, wavefront sums use xor-shuffles over the 64
// lanes, and the per-slot scalar kernels add the partials in index order.
#include "kernels.h"

namespace rexii {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename V>
__device__ __forceinline__ V cadd(V a, V b) {
  V r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename V>
__device__ __forceinline__ V csub(V a, V b) {
  V r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  double2 r;
  r.x = (a.x * b.x + a.y * b.y) / den;
  r.y = (a.y * b.x - a.x * b.y) / den;
  return r;
}
template <typename V>
__device__ __forceinline__ V mk(double x, double y) {
  V r;
  r.x = static_cast<decltype(r.x)>(x);
  r.y = static_cast<decltype(r.y)>(y);
  return r;
}

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// ---------------------------------------------------------------------------
// deterministic block reductions (256 threads = 4 wavefronts of 64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums v over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return s;
}

// ---------------------------------------------------------------------------
// stencil tile in LDS: (kTY + 4) x (kTX + 4) complex values, periodic wrap
// ---------------------------------------------------------------------------
constexpr int kLW = kTX + 2 * kHalo;
constexpr int kLH = kTY + 2 * kHalo;

// (L - zeta) v at LDS position (ly, lx) (interior coordinates)
template <typename V, typename S>
__device__ __forceinline__ V helm(const V (*t)[kLW], int ly, int lx, S cx, S cy, V zeta, V* centre) {
  const V c = t[ly + kHalo][lx + kHalo];
  const V e = t[ly + kHalo][lx + kHalo + 2];
  const V w = t[ly + kHalo][lx + kHalo - 2];
  const V n = t[ly + kHalo + 2][lx + kHalo];
  const V s = t[ly + kHalo - 2][lx + kHalo];
  V q;
  q.x = cx * (e.x + w.x - S(2) * c.x) + cy * (n.x + s.x - S(2) * c.x) - (zeta.x * c.x - zeta.y * c.y);
  q.y = cx * (e.y + w.y - S(2) * c.y) + cy * (n.y + s.y - S(2) * c.y) - (zeta.x * c.y + zeta.y * c.x);
  *centre = c;
  return q;
}

struct TileIdx {
  int x0, y0;
};
__device__ __forceinline__ TileIdx tile_of(const Geo& g) {
  TileIdx t;
  t.x0 = (blockIdx.x % g.tiles_x) * kTX;
  t.y0 = (blockIdx.x / g.tiles_x) * kTY;
  return t;
}

// ---------------------------------------------------------------------------
// inner COCG: p_new = r + beta p_old, partial sums of p_new^T (L - zeta) p_new
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_inner_mv(Batch b) {
  using V = typename C2<T>::t;
  const int slot = blockIdx.y;
  Slot* S = &b.slots[slot];
  if (S->status != kInner) return;
  const Geo g = b.geo;
  const size_t n = size_t(g.nx) * g.ny;
  const V* r = reinterpret_cast<const V*>(b.r) + slot * n;
  const int parity = S->parity;
  const V* pold = reinterpret_cast<const V*>(parity ? b.p1 : b.p0) + slot * n;
  V* pnew = reinterpret_cast<V*>(parity ? b.p0 : b.p1) + slot * n;
  const bool first = (S->it_inner == 0);
  const V beta = mk<V>(S->beta.x, S->beta.y);
  const V zeta = mk<V>(S->zeta.x, S->zeta.y);

  __shared__ V tile[kLH][kLW];
  __shared__ double red[8];
  const TileIdx ti = tile_of(g);
  for (int e = threadIdx.x; e < kLH * kLW; e += kNT) {
    const int ly = e / kLW, lx = e - ly * kLW;
    const size_t gi = size_t(wrap(ti.y0 - kHalo + ly, g.ny)) * g.nx + wrap(ti.x0 - kHalo + lx, g.nx);
    V v = r[gi];
    if (!first) v = cadd(v, cmul(beta, pold[gi]));
    tile[ly][lx] = v;
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const T cx = T(g.cx), cy = T(g.cy);
  T ar = 0, ai = 0;
#pragma unroll
  for (int k = 0; k < kTY / 4; ++k) {
    const int ly = ty + 4 * k;
    const int gx = ti.x0 + tx, gy = ti.y0 + ly;
    if (gx < g.nx && gy < g.ny) {
      V c;
      const V q = helm<V, T>(tile, ly, tx, cx, cy, zeta, &c);
      pnew[size_t(gy) * g.nx + gx] = c;
      ar += c.x * q.x - c.y * q.y;
      ai += c.x * q.y + c.y * q.x;
    }
  }
  const double sr = block_sum(double(ar), red);
  const double si = block_sum(double(ai), red + 4);
  if (threadIdx.x == 0) b.part_a[size_t(slot) * g.nblk + blockIdx.x] = make_double2(sr, si);
}

// d += alpha p, r -= alpha (L - zeta) p; partial sums of r^T r and |r|^2
template <typename T>
__global__ __launch_bounds__(kNT) void k_inner_up(Batch b) {
  using V = typename C2<T>::t;
  const int slot = blockIdx.y;
  Slot* S = &b.slots[slot];
  if (S->status != kInner) return;
  const Geo g = b.geo;
  const size_t n = size_t(g.nx) * g.ny;
  const int parity = S->parity;
  const V* p = reinterpret_cast<const V*>(parity ? b.p0 : b.p1) + slot * n;
  V* r = reinterpret_cast<V*>(b.r) + slot * n;
  V* d = reinterpret_cast<V*>(b.d) + slot * n;
  const V alpha = mk<V>(S->alpha.x, S->alpha.y);
  const V zeta = mk<V>(S->zeta.x, S->zeta.y);

  __shared__ V tile[kLH][kLW];
  __shared__ double red[12];
  const TileIdx ti = tile_of(g);
  for (int e = threadIdx.x; e < kLH * kLW; e += kNT) {
    const int ly = e / kLW, lx = e - ly * kLW;
    const size_t gi = size_t(wrap(ti.y0 - kHalo + ly, g.ny)) * g.nx + wrap(ti.x0 - kHalo + lx, g.nx);
    tile[ly][lx] = p[gi];
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const T cx = T(g.cx), cy = T(g.cy);
  T ar = 0, ai = 0, an = 0;
#pragma unroll
  for (int k = 0; k < kTY / 4; ++k) {
    const int ly = ty + 4 * k;
    const int gx = ti.x0 + tx, gy = ti.y0 + ly;
    if (gx < g.nx && gy < g.ny) {
      V c;
      const V q = helm<V, T>(tile, ly, tx, cx, cy, zeta, &c);
      const size_t gi = size_t(gy) * g.nx + gx;
      d[gi] = cadd(d[gi], cmul(alpha, c));
      const V rn = csub(r[gi], cmul(alpha, q));
      r[gi] = rn;
      ar += rn.x * rn.x - rn.y * rn.y;
      ai += T(2) * rn.x * rn.y;
      an += rn.x * rn.x + rn.y * rn.y;
    }
  }
  const double sr = block_sum(double(ar), red);
  const double si = block_sum(double(ai), red + 4);
  const double sn = block_sum(double(an), red + 8);
  if (threadIdx.x == 0) {
    b.part_a[size_t(slot) * g.nblk + blockIdx.x] = make_double2(sr, si);
    b.part_c[size_t(slot) * g.nblk + blockIdx.x] = sn;
  }
}

// ---------------------------------------------------------------------------
// FP64 outer step: x64 += d (after an inner solve) ...
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_outer_update(Batch b) {
  using V = typename C2<T>::t;
  const int slot = blockIdx.y;
  const Slot* S = &b.slots[slot];
  if (S->status != kInnerDone) return;
  const Geo g = b.geo;
  const size_t n = size_t(g.nx) * g.ny;
  const V* d = reinterpret_cast<const V*>(b.d) + slot * n;
  double2* x = b.x64 + slot * n;
  const TileIdx ti = tile_of(g);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int k = 0; k < kTY / 4; ++k) {
    const int gx = ti.x0 + tx, gy = ti.y0 + ty + 4 * k;
    if (gx < g.nx && gy < g.ny) {
      const size_t gi = size_t(gy) * g.nx + gx;
      const V dv = d[gi];
      double2 xv = x[gi];
      xv.x += double(dv.x);
      xv.y += double(dv.y);
      x[gi] = xv;
    }
  }
}

// ... then r64 = b - (L - zeta) x64 in FP64; r = (T) r64, d = 0;
// partial sums |r64|^2 (part_c) and r^T r of the rounded r (part_a).
template <typename T>
__global__ __launch_bounds__(kNT) void k_outer_residual(Batch b, Rhs rhs) {
  using V = typename C2<T>::t;
  const int slot = blockIdx.y;
  const Slot* S = &b.slots[slot];
  if (S->status != kInnerDone && S->status != kOuterPending) return;
  const Geo g = b.geo;
  const size_t n = size_t(g.nx) * g.ny;
  const double2* x = b.x64 + slot * n;
  V* r = reinterpret_cast<V*>(b.r) + slot * n;
  V* d = reinterpret_cast<V*>(b.d) + slot * n;
  const double2 zeta = S->zeta, a1 = S->a1, a2 = S->a2;
  const bool zero_x = (S->rounds == 0);

  __shared__ double2 tile[kLH][kLW];
  __shared__ double red[12];
  const TileIdx ti = tile_of(g);
  if (!zero_x) {
    for (int e = threadIdx.x; e < kLH * kLW; e += kNT) {
      const int ly = e / kLW, lx = e - ly * kLW;
      const size_t gi = size_t(wrap(ti.y0 - kHalo + ly, g.ny)) * g.nx + wrap(ti.x0 - kHalo + lx, g.nx);
      tile[ly][lx] = x[gi];
    }
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  double ar = 0, ai = 0, an = 0;
#pragma unroll
  for (int k = 0; k < kTY / 4; ++k) {
    const int ly = ty + 4 * k;
    const int gx = ti.x0 + tx, gy = ti.y0 + ly;
    if (gx < g.nx && gy < g.ny) {
      const size_t gi = size_t(gy) * g.nx + gx;
      double2 bv = make_double2(rhs.eta0[gi], 0.0);
      if (rhs.D0) {
        const double dv = rhs.D0[gi], zv = rhs.Z0[gi];
        bv.x += a1.x * dv + a2.x * zv;
        bv.y += a1.y * dv + a2.y * zv;
      }
      double2 rv = bv;
      if (!zero_x) {
        double2 c;
        const double2 q = helm<double2, double>(tile, ly, tx, g.cx, g.cy, zeta, &c);
        rv = csub(bv, q);
      }
      const V rt = mk<V>(rv.x, rv.y);
      r[gi] = rt;
      d[gi] = mk<V>(0.0, 0.0);
      an += rv.x * rv.x + rv.y * rv.y;
      const double tr = double(rt.x), tim = double(rt.y);
      ar += tr * tr - tim * tim;
      ai += 2.0 * tr * tim;
    }
  }
  const double sr = block_sum(ar, red);
  const double si = block_sum(ai, red + 4);
  const double sn = block_sum(an, red + 8);
  if (threadIdx.x == 0) {
    b.part_a[size_t(slot) * g.nblk + blockIdx.x] = make_double2(sr, si);
    b.part_c[size_t(slot) * g.nblk + blockIdx.x] = sn;
  }
}

// ---------------------------------------------------------------------------
// per-slot scalar kernels: one block per slot, partials added in index order
// ---------------------------------------------------------------------------
__device__ double2 reduce_parts2(const double2* p, int m, double* sh) {
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < m; i += kNT) {
    sx += p[i].x;
    sy += p[i].y;
  }
  const double rx = block_sum(sx, sh);
  const double ry = block_sum(sy, sh + 4);
  return make_double2(rx, ry);
}
__device__ double reduce_parts1(const double* p, int m, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += kNT) s += p[i];
  return block_sum(s, sh);
}

__device__ __forceinline__ bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__global__ __launch_bounds__(kNT) void k_scalars_outer(Batch b) {
  const int slot = blockIdx.x;
  Slot* S = &b.slots[slot];
  const int st = S->status;
  if (st != kInnerDone && st != kOuterPending) return;
  __shared__ double sh[12];
  const int m = b.geo.nblk;
  const double2 rr = reduce_parts2(b.part_a + size_t(slot) * m, m, sh);
  const double rn2 = reduce_parts1(b.part_c + size_t(slot) * m, m, sh + 8);
  if (threadIdx.x != 0) return;
  if (S->rounds == 0) S->bn2 = rn2;
  S->rounds += 1;
  const double prev = S->prev_rn2;
  S->rn2 = rn2;
  S->prev_rn2 = rn2;
  if (!isfinite(rn2) || !finite2(rr)) {
    S->status = kFailBreakdown;
  } else if (rn2 <= S->tol2 * S->bn2) {
    S->status = kDone;
  } else if (S->rounds >= 3 && rn2 > 0.25 * prev) {
    // a whole inner solve did not halve the true residual: the FP64
    // rounding floor of the residual is above the requested tolerance
    S->status = kDone;
    S->stagnated = 1;
  } else if (S->it_total >= S->max_iter) {
    S->status = kFailMaxIter;
  } else {
    S->status = kInner;
    S->rr = rr;
    S->it_inner = 0;
    S->beta = make_double2(0.0, 0.0);
    // inner target: the requested reduction of this residual, but never
    // below a quarter of the final tolerance
    S->in_tol2 = fmax(S->inner_eta2 * rn2, 0.0625 * S->tol2 * S->bn2);
  }
}

__global__ __launch_bounds__(kNT) void k_scalars_mv(Batch b) {
  const int slot = blockIdx.x;
  Slot* S = &b.slots[slot];
  if (S->status != kInner) return;
  __shared__ double sh[8];
  const int m = b.geo.nblk;
  const double2 pq = reduce_parts2(b.part_a + size_t(slot) * m, m, sh);
  if (threadIdx.x != 0) return;
  const double mag = fabs(pq.x) + fabs(pq.y);
  if (!(mag > 0.0) || !finite2(pq)) {
    // breakdown of the bilinear form: hand the slot back to the FP64
    // residual step, which restarts the iteration from the true residual
    S->status = (S->it_inner == 0) ? kFailBreakdown : kInnerDone;
    return;
  }
  S->alpha = cdiv(S->rr, pq);
}

__global__ __launch_bounds__(kNT) void k_scalars_up(Batch b) {
  const int slot = blockIdx.x;
  Slot* S = &b.slots[slot];
  if (S->status != kInner) return;
  __shared__ double sh[12];
  const int m = b.geo.nblk;
  const double2 rr = reduce_parts2(b.part_a + size_t(slot) * m, m, sh);
  const double rn2 = reduce_parts1(b.part_c + size_t(slot) * m, m, sh + 8);
  if (threadIdx.x != 0) return;
  S->parity ^= 1;
  S->it_inner += 1;
  S->it_total += 1;
  const bool ok = isfinite(rn2) && finite2(rr) && (fabs(S->rr.x) + fabs(S->rr.y) > 0.0);
  if (ok) S->beta = cdiv(rr, S->rr);
  S->rr = rr;
  if (!ok || rn2 <= S->in_tol2 || S->it_total >= S->max_iter) S->status = kInnerDone;
}

__global__ void k_count(Batch b) {
  // counter[0]: slots still working; [1]: done; [2]: failed
  __shared__ int c[3];
  if (threadIdx.x < 3) c[threadIdx.x] = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < b.B; s += blockDim.x) {
    const int st = b.slots[s].status;
    if (st == kOuterPending || st == kInner || st == kInnerDone) atomicAdd(&c[0], 1);
    else if (st == kDone) atomicAdd(&c[1], 1);
    else if (st == kFailMaxIter || st == kFailBreakdown) atomicAdd(&c[2], 1);
  }
  __syncthreads();
  if (threadIdx.x < 3) b.counter[threadIdx.x] = c[threadIdx.x];
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

// A[j] += Re(c_j[s] * x64[s]) for j = 0, 1, 2, slots in index order
__global__ void k_accumulate(Batch b, const double2* c0, const double2* c1, const double2* c2, int ns, double* A) {
  const size_t n = size_t(b.geo.nx) * b.geo.ny;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    double s0 = A[i], s1 = A[n + i], s2 = A[2 * n + i];
    for (int s = 0; s < ns; ++s) {
      const double2 x = b.x64[size_t(s) * n + i];
      s0 += c0[s].x * x.x - c0[s].y * x.y;
      s1 += c1[s].x * x.x - c1[s].y * x.y;
      s2 += c2[s].x * x.x - c2[s].y * x.y;
    }
    A[i] = s0;
    A[n + i] = s1;
    A[2 * n + i] = s2;
  }
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

// Full per-pole solution x_k = (eta_k, u_k, v_k) from y_k:
// eta = y / sigma, (u, v) = M ((u0, v0) + t g grad eta), M = m1 I + m2 J.
__global__ void k_expand(Batch b, const double* f, int ns, const double2* inv_sigma, const double2* m1,
                         const double2* m2, double tg, int has_vel, double2* out) {
  const int nx = b.geo.nx, ny = b.geo.ny;
  const size_t n = size_t(nx) * ny;
  const int s = blockIdx.y;
  if (s >= ns) return;
  const double2* y = b.x64 + size_t(s) * n;
  const double2 is = inv_sigma[s], M1 = m1[s], M2 = m2[s];
  double2* o = out + size_t(s) * 3 * n;
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline dim3 slot_grid(const Batch& b) { return dim3(b.geo.nblk, b.B); }
static inline unsigned flat_blocks(size_t n) {
  size_t bl = (n + 255) / 256;
  return unsigned(bl > 8192 ? 8192 : (bl < 1 ? 1 : bl));
}

template <typename T>
void launch_outer_update(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_update<T>, slot_grid(b), dim3(kNT), 0, s, b);
}
template <typename T>
void launch_outer_residual(const Batch& b, const Rhs& rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_residual<T>, slot_grid(b), dim3(kNT), 0, s, b, rhs);
}
void launch_scalars_outer(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_scalars_outer, dim3(b.B), dim3(kNT), 0, s, b);
}
template <typename T>
void launch_inner_mv(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_mv<T>, slot_grid(b), dim3(kNT), 0, s, b);
}
void launch_scalars_mv(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_scalars_mv, dim3(b.B), dim3(kNT), 0, s, b);
}
template <typename T>
void launch_inner_up(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_up<T>, slot_grid(b), dim3(kNT), 0, s, b);
}
void launch_scalars_up(const Batch& b, hipStream_t s) {
  hipLaunchKernelGGL(k_scalars_up, dim3(b.B), dim3(kNT), 0, s, b);
}
void launch_count(const Batch& b, hipStream_t s) { hipLaunchKernelGGL(k_count, dim3(1), dim3(256), 0, s, b); }
void launch_fill_zero(double* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(flat_blocks(n)), dim3(256), 0, s, p, n);
}
void launch_copy(const double* src, double* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(flat_blocks(n)), dim3(256), 0, s, src, dst, n);
}
void launch_prep(const double* f, int nx, int ny, double* D0, double* Z0, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(flat_blocks(size_t(nx) * ny)), dim3(256), 0, s, f, nx, ny, D0, Z0, flags);
}
void launch_accumulate(const Batch& b, const double2* c0, const double2* c1, const double2* c2, int ns, double* A,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate, dim3(flat_blocks(size_t(b.geo.nx) * b.geo.ny)), dim3(256), 0, s, b, c0, c1, c2,
                     ns, A);
}
void launch_reconstruct(const double* f, const double* A, int nx, int ny, double S1, double S2, double tg,
                        int has_vel, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_reconstruct, dim3(flat_blocks(size_t(nx) * ny)), dim3(256), 0, s, f, A, nx, ny, S1, S2, tg,
                     has_vel, u);
}
void launch_expand(const Batch& b, const double* f, int ns, const double2* inv_sigma, const double2* m1,
                   const double2* m2, double tg, int has_vel, double2* out, hipStream_t s) {
  size_t n = size_t(b.geo.nx) * b.geo.ny;
  unsigned bx = unsigned(n / 256 + 1 > 1024 ? 1024 : n / 256 + 1);
  hipLaunchKernelGGL(k_expand, dim3(bx, ns), dim3(256), 0, s, b, f, ns, inv_sigma, m1, m2, tg, has_vel, out);
}

template void launch_outer_update<float>(const Batch&, hipStream_t);
template void launch_outer_update<double>(const Batch&, hipStream_t);
template void launch_outer_residual<float>(const Batch&, const Rhs&, hipStream_t);
template void launch_outer_residual<double>(const Batch&, const Rhs&, hipStream_t);
template void launch_inner_mv<float>(const Batch&, hipStream_t);
template void launch_inner_mv<double>(const Batch&, hipStream_t);
template void launch_inner_up<float>(const Batch&, hipStream_t);
template void launch_inner_up<double>(const Batch&, hipStream_t);

}  // namespace rexii
