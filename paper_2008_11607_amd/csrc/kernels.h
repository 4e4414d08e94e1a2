// Device-side data structures and kernel launchers of the REXII solver.
//
// Each pole k of the REXII sum (Sec. 2.2) needs x_k = (tA - z_k I)^{-1} f.
// Eliminating the velocities (Sec. 4, eqs. lswVelocities and lswEta, here
// with centred differences, gravity g, depth H and Coriolis f_c) leaves one
// complex Helmholtz equation per pole for the height:
//   (L - zeta_k) y_k = eta0 + a1_k div(u0,v0) + a2_k curl(u0,v0),
//   L = dx dx + dy dy (a 5-point stencil with stride 2),
//   den = z^2 + t^2 f_c^2,  m1 = -z/den,  m2 = -t f_c/den,
//   sigma = t^2 g H z / den,  zeta = z / sigma,
//   a1 = t H m1, a2 = t H m2,  eta_k = y_k / sigma_k,
//   (u, v)_k = M_k ((u0, v0) + t g grad eta_k),  M = m1 I + m2 J, J(a,b) = (b,-a).
//
// Solver organisation ("slots"): B slots each hold one shifted system at a
// time.  A slot runs COCG (conjugate orthogonal CG for complex-symmetric
// matrices) on L - zeta in the inner precision T (FP32 or FP64), inside an
// FP64 loop of true residuals and refinement.  When its solve is finished
// the slot's solution is added, in FP64, to the three accumulators of its
// problem (A0 = Re sum c0 y, A1 = Re sum c1 y, A2 = Re sum c2 y) and the slot
// takes the next solve from the queue, so every launch works on B live
// solves until the queue is empty.  Slots of one launch may belong to
// different problems (grid sizes).
//
// One COCG iteration is one pass over x, r and p (the pass also forms
// the next search direction, with beta from the recurrence
// r'^T r' = r^T r - 2 alpha q^T r + alpha^2 q^T q), and each slot's scalars
// are reduced by a one-block-per-slot kernel after the pass (a kernel
// boundary makes the partial sums of all XCDs visible; a device-scope fence
// per block would write back the whole L2 each time).
#ifndef REXII_KERNELS_H
#define REXII_KERNELS_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rexii {

// Stencil tile: 64 x 16 points, 256 threads (64 x 4), 4 rows per thread.
constexpr int kTX = 64;
constexpr int kTY = 16;    // tile height of the COCG passes
constexpr int kTYB = 32;   // default tile height of the BiCGStab passes (16 also built)
constexpr int kNT = 256;
constexpr int kNDots = 9;   // pq(2) qr(2) qq(2) rr(2) |r|^2(1)
constexpr int kMaxSlots = 1024;

enum SlotStatus : int {
  kIdle = 0,          // slot holds no solve
  kOuterPending = 1,  // needs an FP64 residual (the first one is the RHS)
  kInner = 2,         // running inner Krylov passes
  kInnerDone = 3,     // inner solve finished: x64 += d, then a residual
  kDone = 4,          // converged (waiting to be accumulated)
  kFailMaxIter = 5,   // stopped at max_iter (x64 holds the best iterate)
  kFailBreakdown = 6, // non-finite scalars
  kInnerLast = 7,     // BiCGStab: stop test fired, last update of d pending
  kPrime = 8,         // COCG: residual taken, first step (p = r) pending
  kRetry = 9,         // mixed precision: stopped without reaching its tolerance
                      // (an inner round went non-finite or diverged, the FP64
                      // residual stagnated, or the inner-precision iteration
                      // cap was hit); not accumulated, the host solves it
                      // again in FP64
};

// One problem (an initial state on a grid) of the launch.
struct Inst {
  int nx, ny, tiles_x, nblk;
  double cx, cy;          // (nx/2)^2, (ny/2)^2
  double cxy;             // nx ny / 4 (cross term of the variable-depth operator)
  const double* H;        // depth field [ny][nx] (BiCGStab path) or nullptr
  const void* Hin;        // the depth in the inner-iteration type (float or double)
  const double* eta0;     // [ny][nx]
  const double* D0;       // div(u0, v0) or nullptr
  const double* Z0;       // curl(u0, v0) or nullptr
  double* A;              // accumulators [3][ny][nx]
};

// One shifted system (device table, read by the scheduler).
struct SolveDev {
  double2 zeta, a1, a2;   // shift and RHS coefficients
  double2 gamma, sc;      // BiCGStab path: cross-term factor, RHS scale
  double2 c0, c1, c2;     // accumulation weights
  double tol2;            // done when ||b - K x||^2 <= tol2 ref2
  double ref2;            // reference of the stop test: > 0 a fixed value
                          // (||f||_W^2 / (g scale^2), so that the test
                          // bounds the solve's share of the error of the
                          // weighted sum), 0: ||b||^2 (relative residual)
  int inst;
  int max_it;             // cap on this solve's Krylov iterations
  int yidx;               // row of Eng::yout that receives its solution
  int pad;
};

// Per-solve outcome (for the report).
struct SolveStat {
  double rn2, bn2;
  int it_total, rounds, status, stagnated;
  int skips, pad;   // COCG inner steps that left d alone (see Slot::dmode)
};

struct Slot {
  double2 zeta, a1, a2;
  double2 gamma, sc; // BiCGStab path (see SolveDev)
  double2 rr;        // COCG: r^T r; BiCGStab: rho = <r_hat, r>
  double2 alpha, beta;
  double2 dcp, dcr;  // COCG: d += dcp p + dcr r in the next inner step (see dmode)
  double2 omega;     // BiCGStab
  double bn2;        // ||b||^2
  double rn2;        // latest FP64 true residual ||b - K x||^2
  double prev_rn2;   // residual of the previous FP64 round
  double in_tol2;    // inner stop: recursive ||r||^2 <= in_tol2
  double tol2;       // final relative tolerance^2 of this solve
  double ref2;       // reference norm^2 of the stop test (see SolveDev)
  double cx, cy, cxy;  // stencil coefficients of the solve's problem
  const double* H;     // its depth field (BiCGStab path) or nullptr
  const void* Hin;     // the same in the inner-iteration type
  const double* eta0;  // its right-hand side fields (see Inst)
  const double* D0;
  const double* Z0;
  int nx, ny, tiles_x, nblk;  // its grid (copied at assignment so a pass
                              // reads every control field in one round)
  int status;
  int parity;        // which r/p buffers hold the current iterate
  int prime;         // 1: next pass only forms p = r and its dots
  int it_total;      // inner iterations over all rounds
  int it_inner;
  int rounds;        // FP64 residual evaluations
  int solve;         // index into the SolveDev table
  int inst;
  int stagnated;
  int discard;       // BiCGStab: d holds no usable correction (its last
                     // inner round went non-finite); the iterate is x64
  int max_it;        // iteration cap of the solve (from SolveDev)
  int dmode;         // COCG: kDUpdate or kDSkip for the next inner step
  int fin;           // COCG: the inner round ends after the next step
  int skips;         // COCG: inner steps with dmode = kDSkip
  int pad2;
};

// COCG correction updates.  An inner step with alpha_i, beta_i adds
// alpha_i p_i to d.  Every other step may leave d alone (kDSkip, when
// |beta_i| >= kDeferBeta): p_{i+1} = r_{i+1} + beta_i p_i, so the next step,
// which reads p_{i+1} and r_{i+1} anyway, adds both terms at once as
//   alpha_{i+1} p_{i+1} + (alpha_i / beta_i) (p_{i+1} - r_{i+1})
// (dcp = alpha_{i+1} + alpha_i / beta_i, dcr = -alpha_i / beta_i).  A round
// never ends on a skipped step: one more step adds the deferred term first.
// The skipped steps neither read nor write d: 4 vector accesses instead of 6.
// FP64 inner precision only: with FP32 vectors the rounding of p - r, scaled
// by 1 / beta_i, slowed the FP64 refinement (more iterations, solves re-run
// in FP64) for a few per cent less pass time.
enum DMode { kDUpdate = 0, kDSkip = 1 };
constexpr double kDeferBeta = 0.1;

// Everything the kernels of one engine need (passed by value).
struct Eng {
  int B;                 // slots
  int S;                 // solves in the queue
  int cap;               // points per slot vector (max over instances)
  int cap_blk;           // partial-sum slots per slot (max tiles)
  double inner_eta2;     // relative reduction^2 of one inner solve
  int retry;             // 1: a solve that fails in the inner precision
                         // ends as kRetry (mixed precision), 0: it ends
                         // stagnated (kDone) or failed
  int method;            // 0: COCG on the constant-depth Helmholtz; 1: BiCGStab (flux form)
  int d_is_f32;          // inner precision of d, r, p (1: FP32, 0: FP64)
  int grid_small;        // persistent grid of kernels that mostly find no work
  int th;                // rows of a work tile (kTY, or 16 / 32 on the BiCGStab path)
  Slot* slots;           // [B]
  const Inst* inst;      // [ninst]
  const SolveDev* solves;// [S]
  SolveStat* stats;      // [S]
  int* next;             // [1] next solve to hand out
  int* work;             // [B + 2]: [0] work items (tiles of working slots),
                         // [1] their common tile count (0 if they differ;
                         // bit 30 set when every slot works, so the list is
                         // 0, 1, ..., B-1), [2..] working slot indices
  int* counter;          // [4] host-visible counts
  int2* items;           // [B * (cap_blk + 7)] (slot, tile): 8 band lists when tile counts differ
                         // (filled when the working slots' tile counts differ)
  double* part;          // [B][cap_blk][kNDots]
  double2* x64;          // [B][cap]
  void* d;               // [B][cap] T2
  void* r0;              // [B][cap] T2, ping-pong
  void* r1;
  void* p0;
  void* p1;
  void* v0;              // BiCGStab: v = K p (ping-pong) and the shadow residual
  void* v1;
  void* rh;
  double2* yout;         // nullptr: accumulate; else solutions, row
                         // SolveDev::yidx of [*][ystride]
  int ystride;           // row stride of yout (points)
  int pad_e;
  int* dbg;              // [16] consistency counters (debug builds only)
};

// Per-pole bilinear dot of the depth derivative (adjoint): for a forward
// Helmholtz solution y (pole with m1, m2, a1, a2, zeta, 1/sigma) and the
// partner adjoint solution y',
//   div = m1 D0 + m2 Z0 + t g m1 (r + zeta y) / sigma,  r = eta0 + a1 D0 + a2 Z0
//   (the divergence of the pole's velocity: L eta = (r + zeta y) / sigma),
//   dot = sum_points Y . div,  Y = (conj ? conj(y') : y') * ysc.
struct AdjDot {
  double2 m1, m2, a1, a2, zeta, isig, ysc;
  int jf, ja;        // queue positions of the forward and adjoint solutions
  int conj;
  int pad;
};

template <typename T>
void launch_pass(const Eng& e, int grid, hipStream_t s);
// Variable-depth (flux form) shifted systems, per pole:
//   K eta = (L_H + gamma C_H - zeta) eta = sc (eta0 + a1 D_H + a2 Z_H),
//   L_H = dx(H dx .) + dy(H dy .),  C_H = dx(H dy .) - dy(H dx .),
//   gamma = t f_c / z,  zeta = (z^2 + t^2 f_c^2) / (t^2 g),  sc = zeta / z,
//   a1 = t m1, a2 = t m2, D_H = div(H (u0, v0)), Z_H = dx(H v0) - dy(H u0),
// solved by BiCGStab (K is not complex-symmetric: C_H is antisymmetric).
// One iteration step: residual round, passes U1 and U2, scalars, pass S,
// scalars.  With ev (7 events) each kernel is bracketed for timing.
template <typename T>
void launch_bcg(const Eng& e, int grid, hipStream_t s, hipEvent_t* ev = nullptr);
void launch_prep_vh(const double* f, const double* H, int nx, int ny, double* D0, double* Z0, int* flags,
                    double* hmax_part, hipStream_t s);
int prep_vh_blocks();
void launch_hmax(const double* H, size_t n, int* flags, double* part, hipStream_t s);
void launch_fill_value(double* p, size_t n, double v, hipStream_t s);
void launch_to_f32(const double* p, float* q, size_t n, hipStream_t s);
int bcg_occupancy(int mixed, int th);

void launch_pass_scalars(const Eng& e, hipStream_t s);
void launch_retire(const Eng& e, hipStream_t s);
void launch_assign(const Eng& e, hipStream_t s);
void launch_count_finished(const Eng& e, hipStream_t s);
int pass_occupancy(int mixed);
void launch_fill_zero(double* p, size_t n, hipStream_t s);
void launch_prep(const double* f, int nx, int ny, double* D0, double* Z0, int* flags, hipStream_t s);
void launch_reconstruct(const double* f, const double* A, int nx, int ny, double S1, double S2,
                        double tg, int has_vel, double* u, hipStream_t s);
void launch_expand(const double2* y, const double* f, int nx, int ny, double2 inv_sigma, double2 m1,
                   double2 m2, double tg, int has_vel, double2* out, hipStream_t s);
void launch_copy(const double* src, double* dst, size_t n, hipStream_t s);
// Partial sums of ||f||_W^2 = g |eta|^2 + H (|u|^2 + |v|^2) for a state f
// [3][n] (H: depth field [n] or nullptr for the constant H0), one per block
// of a fixed grid of wnorm_blocks() blocks, in part[0 .. wnorm_blocks()).
int wnorm_blocks();
void launch_wnorm2(const double* f, const double* H, double H0, double g, size_t n, double* part, hipStream_t s);
void launch_scale3(const double* src, double* dst, size_t n, double s0, double s1, double s2, hipStream_t s);
void launch_scale1(double* p, size_t n, double s, hipStream_t st);
int adj_dot_blocks(size_t n);
void launch_adj_dots(const AdjDot* d, int nd, const double2* yout, int cap, const double* eta0, const double* D0,
                     const double* Z0, int nx, int ny, double tg, int has_vel, double2* part, int nblk,
                     double2* out, hipStream_t s);

}  // namespace rexii

#endif
