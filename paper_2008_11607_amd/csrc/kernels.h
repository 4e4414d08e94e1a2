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
// The solver runs COCG (conjugate orthogonal CG for complex-symmetric
// matrices) on L - zeta_k, all poles of a batch at once ("slots"), with an
// FP64 true-residual / refinement loop around inner iterations in FP64 or
// FP32.  Weighted sums A0 = Re sum c0 y, A1 = Re sum c1 y, A2 = Re sum c2 y
// are accumulated in FP64 and the output is rebuilt from them.
#ifndef REXII_KERNELS_H
#define REXII_KERNELS_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rexii {

// Tile of the stencil kernels: 64 x 16 points, 256 threads (64 x 4), each
// thread handles 4 rows; LDS holds the tile plus a halo of 2.
constexpr int kTX = 64;
constexpr int kTY = 16;
constexpr int kNT = 256;
constexpr int kHalo = 2;

enum SlotStatus : int {
  kIdle = 0,          // slot holds no pole
  kOuterPending = 1,  // needs an FP64 residual (first one: the right-hand side)
  kInner = 2,         // running inner Krylov iterations
  kInnerDone = 3,     // inner solve finished: x64 += d, then a residual
  kDone = 4,          // converged
  kFailMaxIter = 5,   // stopped at max_iter (x64 holds the best iterate)
  kFailBreakdown = 6, // p^T K p vanished or non-finite scalars
};

struct Slot {
  double2 zeta;     // Helmholtz shift of this pole
  double2 a1, a2;   // RHS coefficients of div and curl of the initial velocity
  double2 rr;       // r^T r of the inner iteration (bilinear, no conjugate)
  double2 alpha, beta;
  double bn2;       // ||b||^2
  double rn2;       // latest FP64 true residual ||b - K x||^2
  double in_tol2;   // inner stop: recursive ||r||^2 <= in_tol2
  double tol2;      // done when rn2 <= tol2 * bn2
  double inner_eta2;// relative reduction^2 of one inner solve
  double prev_rn2;  // residual of the previous FP64 round (stagnation test)
  int status;
  int parity;       // which search-direction buffer holds the current p
  int it_total;     // inner iterations over all rounds
  int it_inner;     // iterations of the current inner solve
  int rounds;       // FP64 residual evaluations
  int max_iter;
  int pole;         // index of the pole (or solve) in the problem
  int stagnated;    // 1 if stopped at the FP64 rounding floor above tol
};

struct Geo {
  int nx, ny;
  int tiles_x, tiles_y, nblk;
  double cx, cy;    // (nx/2)^2, (ny/2)^2: coefficients of dx dx and dy dy
};

// Buffers of one batch of B slots.  Vectors are [B][ny][nx].
struct Batch {
  int B;
  Geo geo;
  Slot* slots;           // [B]
  double2* x64;          // FP64 solution
  void* d;               // inner correction (T2)
  void* r;               // inner residual (T2)
  void* p0;              // search directions, ping-pong (T2)
  void* p1;
  double2* part_a;       // [B][nblk] partial sums
  double2* part_b;       // [B][nblk]
  double* part_c;        // [B][nblk]
  int* counter;          // [4] status counts read back by the host
};

// Problem-wide inputs (device)
struct Rhs {
  const double* eta0;    // [ny][nx]
  const double* D0;      // div(u0, v0) or nullptr
  const double* Z0;      // curl(u0, v0) or nullptr
};

// Launchers (kernels.hip).  T is float or double (inner precision).
template <typename T>
void launch_outer_update(const Batch& b, hipStream_t s);
template <typename T>
void launch_outer_residual(const Batch& b, const Rhs& rhs, hipStream_t s);
void launch_scalars_outer(const Batch& b, hipStream_t s);
template <typename T>
void launch_inner_mv(const Batch& b, hipStream_t s);
void launch_scalars_mv(const Batch& b, hipStream_t s);
template <typename T>
void launch_inner_up(const Batch& b, hipStream_t s);
void launch_scalars_up(const Batch& b, hipStream_t s);
void launch_count(const Batch& b, hipStream_t s);
void launch_fill_zero(double* p, size_t n, hipStream_t s);
void launch_prep(const double* f, int nx, int ny, double* D0, double* Z0, int* flags, hipStream_t s);
void launch_accumulate(const Batch& b, const double2* c0, const double2* c1, const double2* c2,
                       int nslots, double* A, hipStream_t s);
void launch_reconstruct(const double* f, const double* A, int nx, int ny, double S1, double S2,
                        double tg, int has_vel, double* u, hipStream_t s);
void launch_expand(const Batch& b, const double* f, int nslots, const double2* inv_sigma,
                   const double2* m1, const double2* m2, double tg, int has_vel,
                   double2* out, hipStream_t s);
void launch_copy(const double* src, double* dst, size_t n, hipStream_t s);

}  // namespace rexii

#endif
