// Internal declarations shared by the host-side sources of librexii.
#ifndef REXII_INTERNAL_H
#define REXII_INTERNAL_H

#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/rexii.h"

namespace rexii {

struct cplx {
  double re, im;
};

// error state (thread-local message)
rexii_status set_error(rexii_status st, const std::string& msg);
rexii_status clear_error();

// coefficients (coeffs.cpp)
double mu();
int terms_L();
int m0_from_tol(double tol);
int m_rule(double t, double rho, double h, int m0);
void poles_weights(int M, double h, std::vector<cplx>& z, std::vector<cplx>& w);
void rexi_poles_weights(int M, double h, std::vector<cplx>& z, std::vector<cplx>& w);
void rexie_terms(int M, double h, std::vector<cplx>& z, std::vector<cplx>& wre, std::vector<cplx>& wim);
double kappa_sum(const std::vector<cplx>& w, double h);
double max_s2(int n);
double rho_const(int nx, int ny, double g, double H, double fc);
double rho_bound_var(int nx, int ny, double g, double Hmax, double fc);

// rocFFT plans of the Fourier-space path (kernels_fft.hip): a batch of three
// real 2D transforms [3][ny][nx] <-> [3][ny][nx/2+1], FP64, not in place,
// cached per device and grid; work_bytes receives the larger work buffer.
// With create == false only plans made by an earlier call are returned
// (REXII_ERR_INVALID_ARG when there are none): creating a plan allocates.
rexii_status fft_plans(int nx, int ny, size_t* work_bytes, void** fwd, void** inv, bool create = true);
rexii_status rocfft_ensure_setup();   // once per process, before any rocFFT plan
// batch of complex 2D transforms [batch][ny][nx], in place, FP64
rexii_status fft_plans_c2c(int nx, int ny, int batch, size_t* work_bytes, void** fwd, void** inv);
rexii_status fft_execute(void* plan, void* in, void* out, void* work, size_t work_bytes, hipStream_t s);
// Device address of the library's static scratch array on the current
// device (REXII_STATIC_SCRATCH_BYTES bytes, 256-byte aligned; looked up once
// per device with hipGetSymbolAddress, then kept).
rexii_status static_scratch(void** ptr);

}  // namespace rexii

#endif
