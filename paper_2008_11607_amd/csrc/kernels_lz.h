// Launchers of the shared-Krylov (multi-shift) path (kernels_lz.hip).
// States are [nrhs][3][ny][nx] FP64; beta is [nrhs][ldb] with beta_0 = ||f||_W
// and beta_j = ||w_j||_W; part is [nrhs][lz_blocks()] block partial sums.
#ifndef REXII_KERNELS_LZ_H
#define REXII_KERNELS_LZ_H

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace rexii {

int lz_blocks(int nx, int ny);
// buf = f, beta[r][0] = ||f_r||_W, flag[0] |= 1 on a non-finite value of f.
void launch_lz_start(const double* f, double* buf, const double* H, double H0, double g, int nx, int ny, int nrhs,
                     double* part, int* flag, double* beta, int ldb, hipStream_t s);
// Lanczos step j (1-based) on cur = buf_j, prev = buf_{j-1} (overwritten with
// buf_{j+1}); with part, beta[r][j] = ||w_j||_W is formed; with y and u,
// u += y_j v_j; last: only the accumulation.
void launch_lz_step(const double* cur, double* prev, const double* H, double H0, double g, double fc, int nx, int ny,
                    int nrhs, int j, double* beta, int ldb, double* part, const double* y, int ldy, double* u,
                    int last, hipStream_t s);

}  // namespace rexii

#endif
