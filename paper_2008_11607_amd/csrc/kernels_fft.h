// Launchers of the Fourier-space path (kernels_fft.hip).
#ifndef REXII_KERNELS_FFT_H
#define REXII_KERNELS_FFT_H

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace rexii {

// Fourier-space path (constant depth).  tab holds nterm merged terms
// (a, b^2, A1, B1, A2, B2); deriv 0: centred-difference symbols, 1: Fourier
// differentiation.
// canon_count: number of distinct canonical wavenumbers among k = 0..kmax on
// an axis of n points (modes with the same canonical pair share theta).
int canon_count(int n, int kmax, int deriv);
// coef [cny][cnx] = scale (Re c1, Re c2) per canonical pair; nw waves per
// block, the terms in ns splits (part: ns x entries double2 when ns > 1).
void mode_coef_shape(int entries, int nterm, int* nw, int* ns);
// sxt, syt: the axis symbols s(k) of the x wavenumbers 0..nx/2 and the y
// wavenumbers 0..ny-1 (axis_symbol), device.
double axis_symbol(int k, int n, int deriv);
// sym = 1 (square grids): the table holds the unordered pairs a <= b only,
// cnx (cnx + 1) / 2 entries (mode_entries).
int mode_entries(int cnx, int cny, int sym);
// With ns > 1 the splits go to part; k_mode_coef_sum adds them into coef,
// unless mode_sum_in_apply(entries, ns): then k_mode_apply adds them (pass
// it part and ns).
void launch_mode_coef(double2* coef, double2* part, int cnx, int cny, int sym, const double* sxt, const double* syt,
                      double t, double g, double H, double fc, double scale, const double* tab, int nterm, int nw,
                      int ns, hipStream_t s);
bool mode_sum_in_apply(int entries, int ns);
// F [3][ny][nx/2+1] <- a0 F + C1 t A F + C2 (t A)^2 F with (C1, C2) from
// coef (ns <= 1: scaled entries; ns > 1: ns x ne unscaled split sums, added
// in order and multiplied by scale).
void launch_mode_apply(double2* F, const double2* coef, int ns, int ne, double scale, int cnx, int sym, int nx,
                       int ny, int deriv, const double* sxt, const double* syt, double t, double g, double H,
                       double fc, double a0, hipStream_t s);
// u = f and one finiteness word per block: flags[copy_check_blocks(n)]
// (at most kCopyCheckMaxBlocks), each 0 or 1.
constexpr int kCopyCheckMaxBlocks = 2048;
int copy_check_blocks(size_t n);
void launch_copy_check(const double* f, double* u, size_t n, int* flags, hipStream_t s);

}  // namespace rexii

#endif
