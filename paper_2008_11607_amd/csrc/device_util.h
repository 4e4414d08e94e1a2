// Device helpers shared by the REXII kernel sources: complex arithmetic,
// coherent loads of control data, periodic indexing, deterministic block
// reductions and the (slot, tile) work mapping.
#ifndef REXII_DEVICE_UTIL_H
#define REXII_DEVICE_UTIL_H

#include <cstddef>

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
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
template <typename V>
__device__ __forceinline__ V mk(double x, double y) {
  V r;
  r.x = static_cast<decltype(r.x)>(x);
  r.y = static_cast<decltype(r.y)>(y);
  return r;
}
__device__ __forceinline__ bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }

// streaming (non-temporal) access to complex values
typedef float nf2 __attribute__((ext_vector_type(2)));
typedef double nd2 __attribute__((ext_vector_type(2)));
#ifdef REXII_NO_NT
__device__ __forceinline__ float2 nt_load(const float2* p) { return *p; }
__device__ __forceinline__ double2 nt_load(const double2* p) { return *p; }
__device__ __forceinline__ void nt_store(float2 a, float2* p) { *p = a; }
__device__ __forceinline__ void nt_store(double2 a, double2* p) { *p = a; }
#else
__device__ __forceinline__ float2 nt_load(const float2* p) {
  const nf2 v = __builtin_nontemporal_load(reinterpret_cast<const nf2*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 nt_load(const double2* p) {
  const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void nt_store(float2 a, float2* p) {
  nf2 v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, reinterpret_cast<nf2*>(p));
}
__device__ __forceinline__ void nt_store(double2 a, double2* p) {
  nd2 v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, reinterpret_cast<nd2*>(p));
}
#endif

// Control data (slot state, tile table, counters, partial sums) is written
// by one kernel and read by later ones.  Reads go through agent-scope
// atomic loads: a plain uniform load may be served from the scalar cache,
// which is not kept coherent with vector stores of earlier launches.
__device__ __forceinline__ int ldc(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ double ldc(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 ldc(const double2* p) { return make_double2(ldc(&p->x), ldc(&p->y)); }
template <typename P>
__device__ __forceinline__ P* ldc_ptr(P* const* p) {
  const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  return reinterpret_cast<P*>(v);
}
// Coherent load of a value at a block-uniform address, returned in scalar
// registers (the atomic load itself is a vector load).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double2 uni(double2 v) { return make_double2(uni(v.x), uni(v.y)); }
__device__ __forceinline__ unsigned long long uni(unsigned long long v) {
  const unsigned int lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned int>(v & 0xffffffffull));
  const unsigned int hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned int>(v >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}
template <typename P>
__device__ __forceinline__ P* uni(P* v) {
  return reinterpret_cast<P*>(uni(reinterpret_cast<unsigned long long>(v)));
}
template <typename X>
__device__ __forceinline__ X ldu(const X* p) { return uni(ldc(p)); }

// A slot record read by one vector load per wavefront: lane k loads the k-th
// 8-byte word (a lane-dependent address, so the load never goes through the
// scalar cache; the record was written by an earlier launch), and fields
// are moved to scalar registers by readlane.  One request per cache line
// instead of one per field keeps the record's lines from becoming a hot
// spot when thousands of blocks read the same slot.
constexpr int kSlotWords = int(sizeof(Slot) / 8);
static_assert(sizeof(Slot) % 8 == 0 && kSlotWords <= 64, "slot record must fit one wavefront load");
struct SlotWords {
  unsigned long long w;
  __device__ __forceinline__ explicit SlotWords(const Slot* S) {
    const int lane = int(threadIdx.x & 63);
    w = (lane < kSlotWords) ? reinterpret_cast<const unsigned long long*>(S)[lane] : 0ull;
  }
  __device__ __forceinline__ unsigned lo(int k) const {
    return unsigned(__builtin_amdgcn_readlane(int(unsigned(w)), k));
  }
  __device__ __forceinline__ unsigned hi(int k) const {
    return unsigned(__builtin_amdgcn_readlane(int(unsigned(w >> 32)), k));
  }
  __device__ __forceinline__ unsigned long long u64(int off) const {
    return (static_cast<unsigned long long>(hi(off / 8)) << 32) | lo(off / 8);
  }
  __device__ __forceinline__ int i32(int off) const { return int((off % 8) ? hi(off / 8) : lo(off / 8)); }
  __device__ __forceinline__ double f64(int off) const { return __longlong_as_double((long long)u64(off)); }
  __device__ __forceinline__ double2 c64(int off) const { return make_double2(f64(off), f64(off + 8)); }
  template <typename P>
  __device__ __forceinline__ P* ptr(int off) const {
    return reinterpret_cast<P*>(u64(off));
  }
};
#define SLOT_OFF(f) int(offsetof(Slot, f))

// Problem and solve tables are uploaded once per call into reused workspace
// addresses: read them the same way.
__device__ __forceinline__ Inst ld_inst(const Inst* p) {
  Inst I;
  I.nx = ldc(&p->nx);
  I.ny = ldc(&p->ny);
  I.tiles_x = ldc(&p->tiles_x);
  I.nblk = ldc(&p->nblk);
  I.cx = ldc(&p->cx);
  I.cy = ldc(&p->cy);
  I.cxy = ldc(&p->cxy);
  I.H = ldc_ptr(&p->H);
  I.eta0 = ldc_ptr(&p->eta0);
  I.D0 = ldc_ptr(&p->D0);
  I.Z0 = ldc_ptr(&p->Z0);
  I.A = ldc_ptr(&p->A);
  return I;
}

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}
// Periodic index for i in [-n, 2n): one conditional add or subtract.
__device__ __forceinline__ int wrap1(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}
// Either form, chosen once per tile (block-uniform): the single-step form
// is exact when the tile with its halo is no larger than the grid.
__device__ __forceinline__ int wrapc(int i, int n, bool big) { return big ? wrap1(i, n) : wrap(i, n); }

// ---------------------------------------------------------------------------
// deterministic reductions (256 threads = 4 wavefronts of 64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduces v[0..N) over the block into out[0..N) (valid in thread 0).
template <int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double* sh, double (&out)[N]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) sh[wid * N + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = (sh[k] + sh[N + k]) + (sh[2 * N + k] + sh[3 * N + k]);
  }
}

// Wavefront sum by DPP lane moves (no LDS): adjacent lanes, pairs of lanes,
// rotations by 4 and 8 within each row of 16, then the row totals are
// carried across rows; the total ends in lane 63.  Fixed order, so the
// result is reproducible.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double wave_total63(double v) {
  v += dpp_f64<0xb1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4e, 0xf>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x124, 0xf>(v);  // row_ror 4
  v += dpp_f64<0x128, 0xf>(v);  // row_ror 8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast 15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast 31 into rows 2 and 3
  return v;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_total63(float v) {
  v += dpp_f32<0xb1, 0xf>(v);
  v += dpp_f32<0x4e, 0xf>(v);
  v += dpp_f32<0x124, 0xf>(v);
  v += dpp_f32<0x128, 0xf>(v);
  v += dpp_f32<0x142, 0xa>(v);
  v += dpp_f32<0x143, 0xc>(v);
  return v;
}

// Block sums of v[0..N) (DPP within each wavefront in the type of v, then
// the four wavefront totals in FP64, in fixed order, through LDS) stored by
// thread 0 at dst[OFF..OFF+N).
template <int N, int OFF = 0, typename A>
__device__ __forceinline__ void store_block_sums(A (&v)[N], double* red, double* dst) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_total63(v[k]);
  if ((threadIdx.x & 63) == 63) {
#pragma unroll
    for (int k = 0; k < N; ++k) red[(threadIdx.x >> 6) * N + k] = double(v[k]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) dst[OFF + k] = (red[k] + red[N + k]) + (red[2 * N + k] + red[3 * N + k]);
  }
}

// Slot sums of N partials over nblk tiles by a block of kSNT threads: each
// thread adds its tiles in index order, then DPP within each wavefront and
// the kSNT/64 wavefront totals in fixed order (valid in thread 0).  The
// partials were written by the previous kernel on the stream, so plain
// loads see them; a thread issues the loads of four tiles before adding.
constexpr int kSNT = 512;
template <int N>
__device__ __forceinline__ void slot_sums_n(const double* pp, int nblk, double (&tot)[N], double* red) {
  constexpr int kU = 4;
  double v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = 0.0;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += kU * kSNT) {
    double t[kU][N];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = b0 + u * kSNT;
#pragma unroll
      for (int k = 0; k < N; ++k) t[u][k] = (b < nblk) ? pp[size_t(b) * kNDots + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] += t[u][k];
    }
  }
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_total63(v[k]);
  if ((threadIdx.x & 63) == 63) {
#pragma unroll
    for (int k = 0; k < N; ++k) red[(threadIdx.x >> 6) * N + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double a = 0.0;
      for (int q = 0; q < kSNT / 64; ++q) a += red[q * N + k];
      tot[k] = a;
    }
  }
}

// partial sums of work item (slot, tile): [slot][tile][kNDots]
__device__ __forceinline__ double* item_part(const Eng& e, int slot, int tile) {
  return e.part + (size_t(slot) * e.cap_blk + tile) * kNDots;
}

// ---------------------------------------------------------------------------
// LDS tile staging.  fetch() issues all of a thread's global loads of a tile
// (element k of the TH x TW tile comes from f(k / TW, k % TW)) before any
// of them is used, so the tile costs one memory round trip; store() then
// writes the registers to LDS (after the caller's barrier).
// ---------------------------------------------------------------------------
template <typename V, int TH, int TW>
struct TileRegs {
  static constexpr int kN = TH * TW;
  static constexpr int kPer = (kN + kNT - 1) / kNT;
  V v[kPer];
  template <typename F>
  __device__ __forceinline__ void fetch(F f) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int k = threadIdx.x + m * kNT;
      if (k < kN) {
        const int ly = k / TW;
        v[m] = f(ly, k - ly * TW);
      }
    }
  }
  __device__ __forceinline__ void store(V* lds) const {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int k = threadIdx.x + m * kNT;
      if (k < kN) lds[k] = v[m];
    }
  }
};

// Row-mapped tile with halo HALO, (TH + 2 HALO) x (kTX + 2 HALO): thread
// (tx, wave w) loads rows w, w + 4, ... at tile column tx + HALO (grid column
// x0 + tx, the same for every row, while each row is uniform across the
// wavefront), and threads 0 .. 2 HALO (TH + 2 HALO) - 1 load one point of
// the 2 HALO side columns.  f(row_offset, column) returns the value of a
// grid point (row_offset = wrapped row * nx).
template <typename V, int HALO, int TH = kTY>
struct RowTile {
  static constexpr int kH = TH + 2 * HALO, kW = kTX + 2 * HALO;
  static constexpr int kRows = (kH + 3) / 4, kSide = 2 * HALO * kH;
  V mainv[kRows];
  V sidev;
  int sly, slx;
  template <typename F>
  __device__ __forceinline__ void fetch(int x0, int y0, int nx, int ny, bool big, F f) {
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const unsigned col = unsigned(wrapc(x0 + tx, nx, big));
    // row offsets first (scalar, with the wrap's branches), then the loads
    // in straight-line code, so that every load is issued before the first
    // value is used (when the tile height is a multiple of 4 no row test
    // is needed: w < 4)
    size_t ro[kRows];
#pragma unroll
    for (int m = 0; m < kRows; ++m) ro[m] = size_t(wrapc(y0 - HALO + w + 4 * m, ny, big)) * size_t(nx);
#pragma unroll
    for (int m = 0; m < kRows; ++m) {
      if (kH % 4 == 0 || w + 4 * m < kH) mainv[m] = f(ro[m], col);
    }
    // the side coordinates are formed here, not hoisted out of a caller's
    // work-item loop (where they would occupy registers across every code
    // path of a pass and can be spilled): the empty asm makes the thread
    // index opaque to loop-invariant code motion
    int tid = int(threadIdx.x);
    asm volatile("" : "+v"(tid));
    sly = tid / (2 * HALO);
    const int c = tid - sly * 2 * HALO;
    slx = (c < HALO) ? c : kTX + c;
    if (tid < kSide)
      sidev = f(size_t(wrapc(y0 - HALO + sly, ny, big)) * size_t(nx), unsigned(wrapc(x0 - HALO + slx, nx, big)));
  }
  __device__ __forceinline__ void store(V* lds) const {
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
#pragma unroll
    for (int m = 0; m < kRows; ++m) {
      if (kH % 4 == 0 || w + 4 * m < kH) lds[(w + 4 * m) * kW + tx + HALO] = mainv[m];
    }
    if (int(threadIdx.x) < kSide) lds[sly * kW + slx] = sidev;
  }
};

// ---------------------------------------------------------------------------
// work items (slot, tile)
// ---------------------------------------------------------------------------
struct Item {
  int slot, tile;
};

constexpr int kWorkIdentity = 1 << 30;

// Head of the work list (one 8-byte coherent load): list length (the
// working tiles when they share one tile count un, else the length of the 8
// band lists together), un (0 when counts differ), identity flag.
struct WorkHead {
  int total, un;
  bool ident;
};
__device__ __forceinline__ WorkHead load_work_head(const Eng& e) {
  const unsigned long long v = uni(static_cast<unsigned long long>(
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(e.work), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
  WorkHead h;
  h.total = int(v & 0xffffffffull);
  const int w1 = int(v >> 32);
  h.un = w1 & (kWorkIdentity - 1);
  h.ident = (w1 & kWorkIdentity) != 0;
  return h;
}

// Work mapping.  A pass kernel's blocks take loop indices w = b, b + G, ...
// (G a multiple of 8), and index w runs on XCD w % 8 (workgroups are dealt
// to the XCDs in turn).  When every working slot has the same tile count
// un, XCD x takes band x of every slot: the tiles x bs .. (x + 1) bs - 1
// (bs = ceil(un / 8), row-major tiles, so a band is a run of tile rows whose
// halo rows stay in that XCD's L2 except at the band edges).  Every XCD then
// holds an equal share of every slot, whatever state each slot is in.  With
// differing tile counts the assignment kernel writes the same bands as 8
// lists of (slot, tile) entries of equal length, list x for XCD x.
struct WorkMap {
  WorkHead h;
  int per;  // loop indices per XCD
  int bs;   // band of tiles per slot and XCD (uniform case), else 0
};
__device__ __forceinline__ WorkMap load_work_map(const Eng& e) {
  WorkMap m;
  m.h = load_work_head(e);
  if (m.h.un > 0) {
    m.bs = (m.h.un + 7) >> 3;
    m.per = (m.h.total / m.h.un) * m.bs;
  } else {
    m.bs = 0;
    m.per = m.h.total >> 3;  // 8 band lists of equal length
  }
  return m;
}
// loop bound: indices 0 .. span - 1
__device__ __forceinline__ int work_span(const WorkMap& m) { return 8 * m.per; }
// (slot, tile) of loop index w; false when w maps to no item
__device__ __forceinline__ bool work_item(const Eng& e, const WorkMap& m, int w, Item& it) {
  const int x = w & 7, i = w >> 3;
  if (m.bs > 0) {
    const int k = i / m.bs;
    const int t = x * m.bs + (i - k * m.bs);
    if (t >= m.h.un) return false;
    it.slot = m.h.ident ? k : ldu(&e.work[2 + k]);
    it.tile = t;
    return true;
  }
  const size_t pos = size_t(x) * m.per + i;
  const unsigned long long v = uni(static_cast<unsigned long long>(__hip_atomic_load(
      reinterpret_cast<const unsigned long long*>(e.items + pos), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
  it.slot = int(v & 0xffffffffull);
  it.tile = int(v >> 32);
  return it.slot >= 0;
}

}  // namespace rexii

#endif
