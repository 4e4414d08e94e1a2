// Internal declarations shared by the host-side sources of librexii.
#ifndef REXII_INTERNAL_H
#define REXII_INTERNAL_H

#include <string>
#include <vector>

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
double kappa_sum(const std::vector<cplx>& w, double h);
double max_s2(int n);
double rho_const(int nx, int ny, double g, double H, double fc);
double rho_bound_var(int nx, int ny, double g, double Hmax, double fc);

}  // namespace rexii

#endif
