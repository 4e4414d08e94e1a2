// Launchers of the Fourier-space path (kernels_fft.hip).
#ifndef REXII_KERNELS_FFT_H
#define REXII_KERNELS_FFT_H

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace rexii {

// Fourier-space path (constant depth): per-mode filter of the half spectra
// F [3][ny][nx/2+1] by the REXII sum, with tab holding nterm merged terms
// (a, b^2, A1, B1, A2, B2); deriv 0: centred-difference symbols, 1: Fourier
// differentiation.  nw: waves (term slices) per block.
int mode_filter_waves(int nx, int ny, int nterm);
void launch_mode_filter(double2* F, int nx, int ny, int deriv, double t, double g, double H, double fc, double c0,
                        double scale, const double* tab, int nterm, int nw, hipStream_t s);
void launch_copy_check(const double* f, double* u, size_t n, int* flag, hipStream_t s);

}  // namespace rexii

#endif
