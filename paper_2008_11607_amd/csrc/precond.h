// Launchers of the preconditioned shifted solves (precond.hip): BiCGStab on
// the flux-form height equation K eta = (L_H + gamma C_H - zeta) eta = b,
// right-preconditioned by the constant-depth operator of the mean depth,
// inverted exactly per Fourier mode.  All FP64; vectors are [B][ny][nx]
// complex128 for B slots, one problem (grid, depth) per launch.
#ifndef REXII_PRECOND_H
#define REXII_PRECOND_H

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace rexii {

enum PcState : int {
  kPcIdle = 0,      // no solve
  kPcStart = 1,     // assigned: the next direction kernel sets x = 0, r = b
  kPcIter = 2,      // iterating
  kPcConv = 3,      // recursive residual within the stop test: the host checks the true one
  kPcCap = 4,       // iteration cap reached
  kPcBreak = 5,     // a scalar of the recurrence was zero or not finite
};

struct PcSlot {
  double2 zeta, gamma, sc, a1, a2;   // operator and right-hand side (as the slot engine's SolveDev)
  double2 sigma;                     // shift of the preconditioner
  double2 rho, alpha, omega, beta;
  double tol2, ref2;                 // stop test |b - K x|^2 <= tol2 ref2 (ref2 = 0: relative, ref2 = |b|^2)
  double stop2;                      // tol2 times the reference (set when the solve starts)
  double rn2;                        // |r|^2 of the recurrence, or of the true residual after a check
  double bn2;                        // |b|^2
  int state, it, max_it, pad;
};

// One problem of a call: grid, stencil coefficients, fields.
struct PcProb {
  int nx, ny;
  double cx, cy, cxy;     // nx^2/4, ny^2/4, nx ny/4
  double hbar;            // mean depth (the preconditioner's)
  const double* H;        // depth [ny][nx]
  const double* eta0;     // [ny][nx]
  const double* D0;       // D_H, Z_H of the initial velocity, or nullptr
  const double* Z0;
  const double* sx;       // axis symbols s(k): x wavenumbers 0..nx/2, then y 0..ny-1
};

// Work vectors of B slots (each [B][ny][nx] double2) and block partials
// [B][pc_blocks()][8].
struct PcVec {
  double2 *x, *r, *rh, *p, *v, *ph, *sh, *t;
  double* part;
  PcSlot* slots;
  int B;
};

int pc_blocks();
// p = r + beta (p - omega v), ph = p (kPcIter); start slots: x = 0,
// r = rh = p = ph = b, v = 0 and the partials of <rh, r> = |b|^2.
void launch_pc_dir(const PcVec& w, const PcProb& pb, hipStream_t s);
// vec[b] *= 1 / (n (-hbar S2(k) - sigma_b)) per Fourier mode (after a forward
// transform of vec; the inverse transform follows).
void launch_pc_scale(double2* vec, const PcVec& w, const PcProb& pb, hipStream_t s);
// out = K in for iterating slots; partial dots: which = 0: <rh, out>
// (into part[2..3]); which = 1: <out, s>, <out, out> with s = w.r (into
// part[4..6]).
void launch_pc_matvec(const double2* in, double2* out, int which, const PcVec& w, const PcProb& pb, hipStream_t s);
// s = r - alpha v into r, sh = s
void launch_pc_s(const PcVec& w, const PcProb& pb, hipStream_t s);
// x += alpha ph + omega sh, r = s - omega t; partials <rh, r>, |r|^2
void launch_pc_xr(const PcVec& w, const PcProb& pb, hipStream_t s);
// one block per slot: stage 0 (after the direction kernel): rho of start
// slots; stage 1: alpha; stage 2: omega; stage 3: rho, beta, |r|^2, the stop
// test and the cap
void launch_pc_scalars(const PcVec& w, int stage, hipStream_t s);
// true residual of the slots in state kPcConv or kPcCap: r = rh = p = b - K x,
// v = 0, rho = <rh, r>, rn2 = |r|^2 (a restart if the host continues)
void launch_pc_resid(const PcVec& w, const PcProb& pb, hipStream_t s);
// A_j += Re(c_j x_slot), j = 0, 1, 2 (A: [3][ny][nx])
void launch_pc_accum(const PcVec& w, int slot, double2 c0, double2 c1, double2 c2, double* A, const PcProb& pb,
                     hipStream_t s);
// mean of a depth field: part[pc_blocks()] block sums (the host adds them)
void launch_pc_sum(const double* H, size_t n, double* part, hipStream_t s);

}  // namespace rexii

#endif
