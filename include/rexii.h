/*
 * rexii.h -- C ABI of the REXII shifted-solve library for MI355X (gfx950).
 *
 * The library computes u = exp(tA) f for the linear rotating shallow-water
 * operator A on a doubly periodic grid by the REXII rational approximation
 * of Caliari, Einkemmer, Moriggl and Ostermann (arXiv 2008.11607):
 *
 *     exp(tA) f  ~  Re sum_{k=1}^{P} alpha_k (A - beta_k I)^{-1} f
 *
 * (Sec. 2.2, eqs. REXI_Modified_matrix and modifiedRexiMatrixReducedSum,
 * written as partial fractions).  Every shifted system is solved
 * matrix-free on the GPU, all poles concurrently, and the weighted sum is
 * accumulated in FP64.
 *
 * Operator (Sec. 4, with centred differences, gravity g, depth H and
 * Coriolis parameter f_c; fields f[c][j][i], c in (eta, u, v), j = y index,
 * i = x index, grid spacing 1/nx and 1/ny on the unit square):
 *
 *     A f = ( -dx(H u) - dy(H v),  -g dx eta + f_c v,  -g dy eta - f_c u ),
 *     dx phi[j][i] = (phi[j][i+1] - phi[j][i-1]) * nx / 2   (periodic).
 *
 * Conventions for every entry point
 *   - Return value: REXII_OK (0) or a negative rexii_status.  Nothing throws
 *     or aborts across the ABI; rexii_last_error() gives a message for the
 *     last failing call on the calling thread.
 *   - Device pointers are HIP device memory owned by the caller; the library
 *     never frees or keeps them.  Host pointers are plain host memory.
 *   - Arrays are contiguous, C order, float64, [3][ny][nx] for states.
 *   - GPU work is enqueued on `stream` (NULL = the null stream).  The calls
 *     that solve return only after their result is complete on `stream`
 *     (the host waits for convergence flags it reads back).
 *   - Workspace: pass NULL/0 and the library allocates what it needs on the
 *     device and frees it before returning; or pass a device buffer of at
 *     least rexii_workspace_size() bytes (256-byte aligned).
 *   - Environment: REXII_PROGRESS=<seconds> makes the Krylov slot engine
 *     print a progress line on stderr at that interval (solves started,
 *     slots working); REXII_TUNE_CACHE names the autotuner's cache file.
 */
#ifndef REXII_H
#define REXII_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    REXII_OK = 0,
    REXII_ERR_INVALID_ARG = -1,   /* bad pointer, size, shape or option      */
    REXII_ERR_NONFINITE = -2,     /* NaN or Inf in the input state or depth  */
    REXII_ERR_NOT_CONVERGED = -3, /* a shifted solve hit its iteration cap, or
                                     the achieved error bound (report
                                     err_bound) exceeds tol; u is still
                                     written, from the best iterates        */
    REXII_ERR_BREAKDOWN = -4,     /* Krylov breakdown (p^T K p == 0)         */
    REXII_ERR_OOM = -5,           /* device allocation failed                */
    REXII_ERR_HIP = -6,           /* a HIP runtime call failed               */
    REXII_ERR_WORKSPACE = -7      /* caller workspace too small              */
} rexii_status;

enum { REXII_PREC_FP64 = 0, REXII_PREC_MIXED = 1 };

/* The operator.  H_field == NULL: constant depth H0.  Otherwise H_field is a
 * device array [ny][nx] of positive depths and A is in flux form (the depth
 * sits inside the divergence); H0 is then ignored. */
typedef struct rexii_swe_op {
    int32_t nx, ny;          /* grid points in x and y, each >= 4           */
    double g;                /* gravity, > 0                                */
    double f_cor;            /* Coriolis parameter                          */
    double H0;               /* constant depth, > 0                         */
    const double* H_field;   /* device [ny][nx] or NULL                     */
} rexii_swe_op;

typedef struct rexii_opts {
    double h;               /* Gaussian width of the approximation (Sec. 2.1,
                               best in [0.3, 0.6] per Sec. 3.1); 0 -> 0.5.
                               The approximation's own error floor is about
                               e^{4 pi h - 4 pi^2} (2e-12 at h = 1, 1e-9 at
                               1.5), so a looser tol admits a larger h:
                               fewer poles (P ~ 2 t rho / h), each better
                               separated from the spectrum (512^2,
                               t rho = 1000: h = 1 takes 0.45 x the time of
                               0.5 at tol 1e-6, 0.4 x at 1e-10)           */
    double tol;             /* target relative L2 error of u; 0 -> 1e-10 for
                               FP64, 1e-6 for MIXED.  Sets m0 (Appendix B)
                               and the per-pole residual tolerance          */
    int32_t precision;      /* REXII_PREC_FP64 or REXII_PREC_MIXED (FP32
                               inner Krylov iterations, FP64 residuals,
                               refinement, weights and pole sum)            */
    int32_t max_iter;       /* cap on Krylov iterations of one solve, all
                               refinement rounds together; 0 -> per solve
                               from its Chebyshev iteration estimate c_s:
                               20 c_s + 5000 in FP64, 4 c_s + 2000 for the
                               FP32 inner iterations of MIXED (a solve past
                               it is solved again in FP64).  Shared-Krylov
                               path: cap on m, 0 -> 50000                  */
    int32_t m0;             /* safety term of the M rule; < 0 -> from tol   */
    double rho;             /* bound on the spectral radius of A; <= 0 ->
                               computed (exact for constant depth)          */
    int32_t pole_batch;     /* concurrent solves (slots); 0 -> heuristic;
                               < 0 -> autotuned: candidate slot counts are
                               timed on the problem itself and the best is
                               cached per grid, precision, method and CU
                               count in $REXII_TUNE_CACHE (default
                               $HOME/.cache/rexii_tune.txt)                 */
    int32_t pair_conjugate; /* 1: when div(u0, v0) == 0 the two poles of a
                               term share one Krylov solve (exact identity);
                               0: one solve per pole.  Default 1            */
    double inner_tol;       /* MIXED: relative residual reduction of one FP32
                               inner solve; 0 -> 1e-4                      */
    int32_t method;         /* 0: automatic (COCG on the constant-depth
                               Helmholtz, BiCGStab for a depth field);
                               1: BiCGStab on the flux form also for
                               constant depth;
                               2: BiCGStab on the flux form preconditioned
                               by the exact (FFT) inverse of the mean-depth
                               operator with a damped shift, FP64
                               (precision ignored), pole_batch slots (0 ->
                               up to 32 within 24 GiB; < 0 as 0); not for
                               rexii_shifted_solve.  Its workspace sizing
                               creates rocFFT plans (needs the device)     */
    int32_t profile;        /* 1: launch the inner kernels one by one with
                               HIP events around each (fills the kernel
                               timing fields of the report); 0: replay them
                               from a HIP graph.  Default 0                */
    int32_t tile_rows;      /* BiCGStab path: rows of a 64-column work tile,
                               16 or 32; 0 -> 32 in MIXED, 16 in FP64, or
                               chosen together with the slot count when
                               pole_batch < 0.  The COCG path always uses
                               16.  Other values: REXII_ERR_INVALID_ARG    */
    int32_t scheme;         /* REXII_SCHEME_REXII (0, default) or
                               REXII_SCHEME_REXI (1: the original REXI matrix
                               scheme, eq. originalREXImatrix, as a
                               comparison; rexii_apply_fourier only, other
                               entry points return REXII_ERR_INVALID_ARG)  */
    int32_t reserved_opts;
} rexii_opts;

enum { REXII_SCHEME_REXII = 0, REXII_SCHEME_REXI = 1 };

typedef struct rexii_report {
    int32_t P;               /* number of poles (= 2(N+1))                  */
    int32_t M, N, m0;        /* M rule (eq. matrixAccuracyBound), N = M + L */
    int32_t solves;          /* Krylov systems solved (P, or P/2 paired)    */
    int32_t max_iters;       /* most Krylov iterations of one solve         */
    int32_t max_refine;      /* most FP64 residual/refinement rounds        */
    int32_t not_converged;   /* solves that stopped at max_iter            */
    int64_t total_iters;     /* Krylov iterations summed over solves        */
    double h, t, rho;
    double kappa_sum;        /* sum |alpha_k t| / |h mu|: amplification of
                               per-pole errors in the weighted sum          */
    double pole_tol;         /* tightest relative residual a solve is driven
                               to: solve s gets tol c_s / (a_s sum_j c_j),
                               a_s the sum of its poles' |w_k| / |h mu|,
                               c_s its estimated iterations per e-fold
                               (capped at 1e-2)                             */
    double max_rel_residual; /* largest final FP64 relative residual        */
    double seconds;          /* host wall time of the call (seconds_total)  */
    double alg_bytes;        /* algorithmic HBM bytes of the Krylov kernels */
    int32_t stagnated;       /* FP64 solves stopped at their residual floor
                               above their tolerance (their residuals enter
                               err_bound)                                  */
    int32_t slots;           /* concurrent solves the engine ran with        */
    /* with opts.profile = 1: launches and summed HIP-event time of the COCG
     * pass kernel, and the algorithmic bytes of those launches (a pass reads
     * x, r, p and writes them once: 6 complex values per grid point and
     * live solve; 3 for the first pass after an FP64 residual) */
    int64_t kernel_launches;
    double kernel_ms;
    double kernel_bytes;
    /* BiCGStab path with opts.profile = 1: HIP-event time of each kernel of
     * the kernel_launches iteration steps, summed (ms): residual round,
     * pass U1, pass U2, scalars after U, pass S, scalars after S; and the
     * algorithmic bytes of the pass U1 launches */
    double step_ms[6];
    double u1_bytes;
    int32_t tile_rows;       /* rows of the work tiles the engine ran with   */
    int32_t reserved;
    /* Achieved error bound of the pole sum, relative in the W-norm
     * (W = diag(g, H, H)): by Theorem 1 (eq. teorem, cond(V) = 1 in the W-norm
     * because WA is skew) the error of each pole's resolvent is at most its
     * residual / |h mu|, so
     *     |u - r(tA) f|_W / |f|_W <= err_bound = sum_s wsum_s |r_s|_W / |f|_W,
     * wsum_s = sum of |alpha_k t| / |h mu| over the poles solve s serves and
     * r_s its final FP64 residual (only the height row is non-zero).  The call
     * returns REXII_ERR_NOT_CONVERGED when err_bound > tol.  Explicit shifts
     * (rexii_shifted_solve): the largest relative residual of a shift. */
    double err_bound;
    double seconds_solve;    /* host wall time of the Krylov engine(s): the
                               solves, without set-up and reconstruction    */
    int32_t retried;         /* MIXED: solves whose FP32 inner iterations
                               failed (non-finite, diverged, stalled or past
                               their cap) and that were solved again in FP64 */
    int32_t hist_buckets;    /* 20 */
    int32_t iter_hist[20];   /* solves by Krylov iterations (both attempts of
                               a re-run solve): bucket 0 holds 0..1, bucket
                               k holds [2^k, 2^(k+1)), the last one is open */
} rexii_report;

/* Fill *opts with the defaults described above. */
void rexii_default_opts(rexii_opts* opts);

/* Poles and weights (host, FP64).  Sec. 2.1 eqs. bm and modifiedRexi give
 * c_{1,n}, c_{2,n}; Sec. 2.2 gives C_{1,n}, C_{2,n}; the reduced sum
 * (eq. modifiedRexiMatrixReducedSum) has, for n = 0..N, poles of tA at
 * alpha_{-n} = h(mu - i n) and -alpha_n = -h(mu + i n); M follows
 * eq. matrixAccuracyBound: M = ceil(t rho / h) + m0, N = M + 24.
 *   t > 0, rho > 0, 0 < h < pi; tol in (0, 1) chooses m0 when m0 < 0.
 *   *P receives the pole count 2(N+1).  If beta and alpha are non-NULL they
 *   must hold 2*P doubles each and receive (re, im) pairs of
 *   beta_k = z_k / t and alpha_k = w_k / t, ordered n = 0..N, two per n.
 *   kappa_sum may be NULL.  Errors: REXII_ERR_INVALID_ARG. */
rexii_status rexii_coeffs(double t, double rho, double h, double tol, int32_t m0,
                          int32_t* P, double* beta, double* alpha, double* kappa_sum);

/* Poles and weights of the original REXI matrix scheme (eq. originalREXImatrix,
 * the paper's comparison scheme): exp(tA) f ~ Re sum_k alpha_k (A - beta_k I)^{-1} f
 * with beta_k = -alpha_n / t, alpha_n = h (mu + i n), and weights beta^Re_n / t
 * (eq. originalRexi), n = -N..N ordered 0, 1, -1, 2, -2, ...; *P = 2N + 1,
 * N = M + 24, M from the same rule as rexii_coeffs.  Arguments and errors as
 * rexii_coeffs (no kappa_sum). */
rexii_status rexii_coeffs_rexi(double t, double rho, double h, double tol, int32_t m0,
                               int32_t* P, double* beta, double* alpha);

/* Spectral radius bound of A (eq. matrixAccuracyBound needs an upper bound).
 * Constant depth: exact, sqrt(f_c^2 + g H0 max(s_x^2 + s_y^2)) with
 * s_x = nx sin(2 pi k / nx).  Variable depth: the guaranteed
 * sqrt(g max H) sqrt(nx^2 + ny^2) + |f_c| (reads H_field on `stream`;
 * REXII_ERR_NONFINITE if a depth is not finite and positive). */
rexii_status rexii_rho(const rexii_swe_op* op, hipStream_t stream, double* rho);

/* Device workspace rexii_apply / rexii_apply_adjoint need for these
 * arguments (bytes): an upper bound of both (the adjoint with dJdH keeps
 * every resolvent, so for a plain rexii_apply
 * rexii_batched_workspace_size(1, ...) is the tighter figure).  t is needed
 * because it fixes the pole count.  With opts->pole_batch < 0 the bound
 * covers every slot count and tile height the autotuner may try (it runs its
 * candidates inside the caller's workspace).  A depth field is read on the
 * null stream (its maximum fixes rho). */
rexii_status rexii_workspace_size(const rexii_swe_op* op, const rexii_opts* opts,
                                  double t, size_t* bytes);

/* u = exp(tA) f (REXII approximation): the reduced pole sum of Sec. 2.2
 * (eq. modifiedRexiMatrixReducedSum, as partial fractions) with one Krylov
 * shifted solve per pole (Sec. 4, the per-term systems, solved here through
 * the height equation eq. lswEta and the velocities of eq. lswVelocities),
 * M from eq. matrixAccuracyBound.  The achieved bound of Theorem 1
 * (eq. teorem, with each solve's final residual) is in rep->err_bound; when
 * it exceeds opts->tol the call returns NOT_CONVERGED with u written.
 * f, u: device [3][ny][nx], must not overlap.  t >= 0 (t == 0 copies f).
 * opts may be NULL (defaults); rep may be NULL.  Errors: INVALID_ARG,
 * NONFINITE (f or H_field), NOT_CONVERGED, BREAKDOWN, OOM, HIP, WORKSPACE. */
rexii_status rexii_apply(const rexii_swe_op* op, const double* f, double* u, double t,
                         const rexii_opts* opts, void* workspace, size_t ws_bytes,
                         hipStream_t stream, rexii_report* rep);

/* Reverse mode of rexii_apply for a loss J(u).  The approximant is the real
 * rational function r(tA) of eqs. REXI_Modified_matrix and
 * modifiedRexiMatrixReducedSum; its transpose r(tA)^T = W r(-tA) W^{-1}
 * (A^T = -W A W^{-1}, W = diag(g, H, H)) is the same pole set with the two
 * weights of each term n exchanged and conjugated, so the reverse pass is
 * another rexii_apply-sized set of shifted solves.
 *   gbar = dJ/du (device [3][ny][nx]).  dJdf (device [3][ny][nx], may be
 *   NULL) receives r(tA)^T gbar.  dJdH (host, one double, may be NULL;
 *   constant depth only; needs f) receives dJ/dH0 for the same pole set
 *   (poles do not move with H0): minus the real part of the weighted sum over
 *   poles of the bilinear forms y_k^T (t dA/dH0) x_k, with x_k the forward
 *   resolvents of f and y_k those of gbar under the transposed weights.
 *   Workspace, stream and report as rexii_apply (the report covers both the
 *   forward and the reverse solves).
 * Errors as rexii_apply. */
rexii_status rexii_apply_adjoint(const rexii_swe_op* op, const double* f, const double* gbar,
                                 double* dJdf, double* dJdH, double t, const rexii_opts* opts,
                                 void* workspace, size_t ws_bytes, hipStream_t stream,
                                 rexii_report* rep);

/* Device workspace of rexii_apply_batched for these problems (count = 1:
 * of rexii_apply), bytes; with opts->pole_batch < 0 it covers every job the
 * autotuner may run.  Depth fields are read on the null stream. */
rexii_status rexii_batched_workspace_size(int32_t count, const rexii_swe_op* ops, const double* t,
                                          const rexii_opts* opts, size_t* bytes);

/* count independent problems in one call: ops[i], f[i], u[i], t[i] as in
 * rexii_apply (host arrays of device pointers).  The paper's GPU code splits
 * the terms of the sum into chunks that fit the device (Sec. 4, GPU
 * implementation, algorithm GPUimplementation); here the terms of every
 * instance form one queue of shifted solves (most expensive first) served by
 * one set of solver slots, so a chunk mixes instances and grids, and each
 * instance's weighted sum (eq. modifiedRexiMatrixReducedSum) is accumulated
 * in FP64 as its solves finish.  opts applies to every instance
 * (pole_batch < 0 autotunes the slot count for the batch).  reps may be
 * NULL or hold count reports (one per instance).  Workspace: NULL, or at
 * least rexii_batched_workspace_size() bytes.  Errors as rexii_apply; the
 * first failing instance's status is returned after every instance's u is
 * written. */
rexii_status rexii_apply_batched(int32_t count, const rexii_swe_op* ops, const double* const* f,
                                 double* const* u, const double* t, const rexii_opts* opts,
                                 void* workspace, size_t ws_bytes, hipStream_t stream,
                                 rexii_report* reps);

/* Single-pole resolvents (Sec. 4, per-term systems): x_k = (tA - z_k I)^{-1} f
 * for npoles complex shifts z (host, (re, im) pairs), Re z_k != 0.
 * x: device complex128 [npoles][3][ny][nx] as (re, im) pairs.
 * Errors as rexii_apply. */
rexii_status rexii_shifted_solve(const rexii_swe_op* op, const double* f, double t, int32_t npoles,
                                 const double* z, double* x, const rexii_opts* opts,
                                 void* workspace, size_t ws_bytes, hipStream_t stream,
                                 rexii_report* rep);

/* Fourier-space REXII for a constant depth, the way the paper evaluates its
 * own test problem (Sec. 4: FFT, the pole sum per Fourier mode, inverse FFT).
 * Each mode's 3x3 symbol A_hat(k) has eigenvalues 0 and +-i omega(k), so
 * r(t A_hat) = c0 I + c1 t A_hat + c2 (t A_hat)^2 with c0, c1, c2 the
 * interpolation coefficients of r(x) = sum_k w_k / (x - z_k) on
 * {0, +-i t omega} (Theorem 1, eq. teorem); the real part of the REXII sum
 * (eq. modifiedRexiMatrixReducedSum) is a quadratic with the real parts of
 * those coefficients, applied to the half spectrum of a real FFT.  Same
 * poles, weights and result as rexii_apply with exact shifted solves; no
 * iterations.  All arithmetic FP64 (opts.precision is ignored).
 *   derivative: REXII_DERIV_CENTRED, the operator of rexii_apply, symbol
 *     s = n sin(2 pi k / n); or REXII_DERIV_SPECTRAL, Fourier differentiation
 *     on the unit square, s = 2 pi k for signed k with the Nyquist mode's
 *     derivative 0 (the paper's discretisation).
 *   op->H_field must be NULL.  opts: h, tol, m0 and rho as for rexii_apply
 *     (rho <= 0: the exact maximum of omega over the modes), scheme (REXI
 *     uses the poles of rexii_coeffs_rexi) and profile; other fields
 *     ignored.  f, u: device [3][ny][nx], not overlapping.
 *   Workspace: rexii_fourier_workspace_size() bytes (half spectra
 *     [3][ny][nx/2+1] complex128, coefficient table and split sums,
 *     finiteness words, the FFT work buffer), or NULL to let the library
 *     allocate.  FFT plans are created on first use per device and grid,
 *     and device copies of the term and symbol tables on first use per
 *     device; both are kept until the process ends.
 *   The pole sums depend on a mode only through s_x^2 and s_y^2, which
 *     repeat along each axis: they are formed once per distinct pair
 *     (about 1/8 of the half spectrum on even grids with centred
 *     differences; on square grids the pair is unordered, about 1/16) and
 *     applied to every mode.
 *   Report: P, M, N, m0, h, t, rho, kappa_sum; solves = terms of the sum
 *     (two poles of one n share a denominator); total_iters = distinct
 *     frequencies the sums were formed at; slots = waves per block of the
 *     sum kernel; tile_rows = its term splits; alg_bytes = algorithmic HBM bytes of the path;
 *     kernel_bytes = those of the apply kernel (96 per half-spectrum mode).
 *     With opts.profile = 1: step_ms[0..4] = copy and finiteness check,
 *     forward FFT, pole sums, apply, inverse FFT (HIP events, ms);
 *     kernel_ms = step_ms[2], kernel_launches = 1.
 * Errors: INVALID_ARG (also for a depth field or an unknown derivative),
 * NONFINITE (u is written anyway), OOM, HIP (including rocFFT failures),
 * WORKSPACE. */
enum { REXII_DERIV_CENTRED = 0, REXII_DERIV_SPECTRAL = 1 };

rexii_status rexii_fourier_workspace_size(const rexii_swe_op* op, const rexii_opts* opts, double t,
                                          int32_t derivative, size_t* bytes);

rexii_status rexii_apply_fourier(const rexii_swe_op* op, const double* f, double* u, double t,
                                 int32_t derivative, const rexii_opts* opts, void* workspace,
                                 size_t ws_bytes, hipStream_t stream, rexii_report* rep);

/* For callers that cannot allocate device memory: tight serving loops and
 * harnesses that forbid hipMalloc.  The same computation, kernels and
 * result as rexii_apply_fourier, with every piece of device scratch (half
 * spectra, term table, coefficient table, finiteness words, FFT work
 * buffer) taken
 * from a static array inside the library instead of a workspace:
 * REXII_STATIC_SCRATCH_BYTES bytes per GPU, reserved when the library's
 * code is loaded on that GPU and held until the process ends.
 *   The call allocates no device memory and no pinned host memory.  Its
 *     FFT plans must exist already: creating a plan allocates, so call
 *     rexii_fourier_workspace_size (or rexii_apply_fourier) once for the
 *     grid on that device beforehand (set-up); otherwise the call returns
 *     REXII_ERR_INVALID_ARG.
 *   Arguments, layouts and the report as rexii_apply_fourier;
 *     opts.profile is ignored (no HIP events are created).
 *   Sizes: a problem whose scratch (rexii_fourier_workspace_size bytes)
 *     exceeds REXII_STATIC_SCRATCH_BYTES returns REXII_ERR_WORKSPACE
 *     (covers grids up to 2048 x 2048).
 *   Every call on one GPU uses that GPU's single array and leaves its
 *     contents behind (every word a call reads back is written by a kernel
 *     of that call first): calls
 *     that overlap in time on one GPU, from several host threads or on
 *     several streams, race and give wrong results; serialise them.
 * Errors: as rexii_apply_fourier. */
#define REXII_STATIC_SCRATCH_BYTES ((size_t)256 << 20)

rexii_status rexii_apply_fourier_noalloc(const rexii_swe_op* op, const double* f, double* u, double t,
                                         int32_t derivative, const rexii_opts* opts,
                                         hipStream_t stream, rexii_report* rep);

/* Shared-Krylov (multi-shift) REXII, any depth: all shifted systems
 * (tA - z_k I) x_k = f have one right-hand side, and Krylov spaces are
 * shift invariant, so one Lanczos process per state serves every pole
 * (the systems of the partial-fraction sum, eq. modifiedRexiMatrixReducedSum,
 * solved together instead of one Krylov solve each):
 *     u = ||f||_W V_m Re sum_k w_k (t T_m - z_k I)^{-1} e_1.
 * W = diag(g, H, H) makes A skew-adjoint, so the process is a real
 * two-term recurrence and T_m is skew-tridiagonal.  Pass 1 forms the
 * recurrence coefficients; the host solves the small problems; pass 2
 * repeats the same steps and accumulates u, so the basis is never stored.
 * The poles come from the M rule for the Gershgorin bound of T_m, which is
 * at most rho(A).  m grows until the last 8 coefficients of the small
 * solution hold under tol / 10 of its norm (checked from m = 0.75 t rho on).
 * FP64 throughout (opts.precision ignored).
 *   nrhs states share op and t: f, u device [nrhs][3][ny][nx], not
 *     overlapping.
 *   opts: h, tol, m0 as for rexii_apply; max_iter caps the Krylov dimension
 *     m (default 50000); profile = 1 fills step_ms.
 *   Workspace: rexii_multishift_workspace_size() bytes, or NULL.
 *   Report: solves = max_iters = m, total_iters = sum of m over states,
 *     P, M, N for the largest small problem, rho = its Gershgorin bound,
 *     max_rel_residual = largest tail ratio, alg_bytes = algorithmic HBM
 *     bytes of both passes.  With profile = 1: step_ms[0] pass 1, [1] host
 *     small problems, [2] pass 2 (ms); kernel_ms = step_ms[2] and
 *     kernel_bytes = pass 2's algorithmic bytes.
 * Errors: INVALID_ARG, NONFINITE (f), NOT_CONVERGED (m reached max_iter;
 * u is written from that m), OOM, HIP, WORKSPACE. */
rexii_status rexii_multishift_workspace_size(const rexii_swe_op* op, int32_t nrhs, const rexii_opts* opts,
                                             size_t* bytes);

rexii_status rexii_apply_multishift(const rexii_swe_op* op, int32_t nrhs, const double* f, double* u, double t,
                                    const rexii_opts* opts, void* workspace, size_t ws_bytes,
                                    hipStream_t stream, rexii_report* rep);

/* Message for the last non-OK status returned on this thread ("" if none). */
/* The paper's matrix experiments (Sec. 3.2, Fig. matrixRexiExample) for a
 * circulant matrix A, (A f)_j = sum_q coefs_q f_{(j + offsets_q) mod n}
 * (e.g. the periodic difference matrices A_1 and A_2 of that section), with
 * one of three schemes:
 *   REXII_CIRC_REXII  eq. modifiedRexiMatrixReducedSum (poles of
 *                     rexii_coeffs); A must be real and skew-symmetric;
 *   REXII_CIRC_REXI   the original REXI, eq. originalREXImatrix (poles of
 *                     rexii_coeffs_rexi); same premise on A;
 *   REXII_CIRC_REXIE  eq. REXIE, for A - nu I = i B with B real symmetric
 *                     (real eigenvectors): exp(tA) f = e^{t nu} exp(t(A - nu I)) f,
 *                     the shift nu = i * nu_im (Sec. 2.2's remark on shifts);
 *                     the result is complex.
 * Every resolvent is evaluated exactly, per Fourier mode (the DFT
 * diagonalises A): rocFFT, the pole sum per mode, inverse rocFFT, FP64.
 *   offsets, coefs: host arrays of nstencil (1..64) entries; coefs are (re, im)
 *     pairs.  A premise that does not hold (to 1e-13 of the largest
 *     coefficient): REXII_ERR_INVALID_ARG.  nu_im must be 0 unless REXIE.
 *   f: device float64 [nrhs][n] (real vectors); u: device complex128
 *     [nrhs][n] as (re, im) pairs (imaginary part 0 for REXII and REXI);
 *     not overlapping.  n >= 2, n * nrhs <= 2^31.
 *   M > 0 fixes M (the figure sweeps it); M <= 0 takes eq. matrixAccuracyBound
 *     with rho = max_k |lambda_k - i nu_im| (exact, or opts.rho when > 0) and
 *     m0 from opts (m0 or tol).  opts.h is the Gaussian width; other opts
 *     fields are ignored.  opts may be NULL.
 *   Workspace: rexii_circulant_workspace_size() bytes, 256-byte aligned, or
 *     NULL to let the library allocate.  FFT plans are created on first use
 *     per device, n and nrhs and kept until the process ends.
 *   Report: P (poles), M, N, m0, h, t, rho, kappa_sum (sum over the weights
 *     of |w| / |h mu|, both weight sets for REXIE), total_iters = modes,
 *     slots = waves per block of the pole-sum kernel, seconds.  With
 *     opts.profile = 1: step_ms[0..4] = load and finiteness check, forward
 *     FFT, pole sums, apply, inverse FFT (HIP events, ms), kernel_ms =
 *     step_ms[2].
 *   The call returns when u is complete on `stream`.
 * Errors: INVALID_ARG, NONFINITE (f; u is written anyway), OOM, HIP, WORKSPACE. */
enum { REXII_CIRC_REXII = 0, REXII_CIRC_REXI = 1, REXII_CIRC_REXIE = 2 };
rexii_status rexii_circulant_workspace_size(int32_t n, int32_t nstencil, const int32_t* offsets, const double* coefs,
                                            int32_t nrhs, double t, double nu_im, int32_t scheme, int32_t M,
                                            const rexii_opts* opts, size_t* bytes);
rexii_status rexii_apply_circulant(int32_t n, int32_t nstencil, const int32_t* offsets, const double* coefs,
                                   int32_t nrhs, const double* f, double* u, double t, double nu_im, int32_t scheme,
                                   int32_t M, const rexii_opts* opts, void* workspace, size_t ws_bytes,
                                   hipStream_t stream, rexii_report* rep);

/* A refit of the coefficients of the Gaussian's rational approximation
 * (Sec. 2.1, step 2; Appendix A prints the paper's own fit): R(x) in the
 * symmetric form of eq. A(x,mu) with L terms and shift mu, fitted to
 * psi_1(x) = (4 pi)^{-1/2} e^{-x^2/4} by least squares (eq. minl2approx) on
 * K points chosen Leja fashion from n_candidates equally spaced values of
 * [0, x_max] (x_1 = 0, then the candidate with the largest product of
 * distances to the points chosen so far; psi_1 and R are even).  Householder
 * QR and one refinement step with an extended-precision residual.  Host
 * only, FP64.
 *   a: host, 2(L+1) doubles, receives (Re a_l, Im a_l) for l = 0..L
 *     (a_{-l} = conj(a_l)); points: host, K doubles or NULL (the chosen
 *     points in order); max_err: NULL or receives max |psi_1 - R| over the
 *     candidate grid.  With L = 24, the printed mu, x_max = 60, K = 200 the
 *     fit matches the printed table's accuracy (about 1.5e-14).
 * Errors: INVALID_ARG (1 <= L <= 64, mu != 0, x_max > 0,
 * 2L+1 <= K <= n_candidates <= 2e7, or a rank-deficient system), OOM. */
rexii_status rexii_fit_gaussian(int32_t L, double mu, double x_max, int32_t K, int32_t n_candidates, double* a,
                                double* points, double* max_err);

const char* rexii_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* REXII_H */
