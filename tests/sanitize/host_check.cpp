// Host-only exercise of librexii's planning code, built with the host-side
// address and undefined-behaviour sanitizers (tests/test_host_sanitizers.py).
// Nothing here needs a GPU: every call either returns before touching the
// device (argument checks) or is pure host work (coefficients, the M rule,
// pole plans, slot and workspace sizing, the circulant premises).  A
// sanitizer report aborts the program; the checks below fail it with
// exit status 1.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rexii.h"

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static void coefficients() {
  const double trhos[] = {1e-3, 1.0, 37.5, 100.0, 1000.0, 5000.0};
  const double hs[] = {0.1, 0.5, 1.0, 1.5};
  const double tols[] = {1e-16, 1e-10, 1e-6};
  for (double trho : trhos)
    for (double h : hs)
      for (double tol : tols)
        for (int m0 : {-1, 0, 11}) {
          int P = 0;
          CHECK(rexii_coeffs(1.0, trho, h, tol, m0, &P, nullptr, nullptr, nullptr) == REXII_OK);
          std::vector<double> b(2 * size_t(P)), a(2 * size_t(P));
          double kap = 0.0;
          CHECK(rexii_coeffs(1.0, trho, h, tol, m0, &P, b.data(), a.data(), &kap) == REXII_OK);
          CHECK(P % 2 == 0 && kap > 0.0 && std::isfinite(kap));
          for (int k = 0; k < P; ++k) CHECK(std::isfinite(b[2 * k]) && std::isfinite(a[2 * k + 1]));
          // the two poles of a term: beta_2 = -conj(beta_1)
          for (int k = 0; k + 1 < P; k += 2) {
            CHECK(b[2 * k] == -b[2 * k + 2]);
            CHECK(b[2 * k + 1] == b[2 * k + 3]);
          }
          int Pr = 0;
          CHECK(rexii_coeffs_rexi(1.0, trho, h, tol, m0, &Pr, nullptr, nullptr) == REXII_OK);
          std::vector<double> br(2 * size_t(Pr)), ar(2 * size_t(Pr));
          CHECK(rexii_coeffs_rexi(1.0, trho, h, tol, m0, &Pr, br.data(), ar.data()) == REXII_OK);
          CHECK(Pr == P - 1);
        }
  int P = 0;
  CHECK(rexii_coeffs(0.0, 1.0, 0.5, 1e-10, -1, &P, nullptr, nullptr, nullptr) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_coeffs(1.0, 1.0, 4.0, 1e-10, -1, &P, nullptr, nullptr, nullptr) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_coeffs(1.0, 1.0, 0.5, 2.0, -1, &P, nullptr, nullptr, nullptr) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_coeffs(1.0, 1e300, 0.5, 1e-10, -1, &P, nullptr, nullptr, nullptr) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_coeffs(1.0, 1.0, 0.5, 1e-10, -1, nullptr, nullptr, nullptr, nullptr) == REXII_ERR_INVALID_ARG);
  CHECK(std::strlen(rexii_last_error()) > 0);
}

static rexii_swe_op lrsw(int nx, int ny, double fc) {
  rexii_swe_op op;
  op.nx = nx;
  op.ny = ny;
  op.g = 1.0;
  op.f_cor = fc;
  op.H0 = 1.0;
  op.H_field = nullptr;
  return op;
}

static void plans_and_sizes() {
  // constant-depth plans and slot-engine sizes: one problem, with and
  // without the autotuner's bound, both precisions, and the adjoint sizing
  const int grids[][2] = {{4, 4}, {64, 64}, {96, 80}, {512, 512}, {1024, 1024}, {2048, 2048}, {37, 129}};
  for (auto& gsz : grids)
    for (int prec : {REXII_PREC_FP64, REXII_PREC_MIXED})
      for (int pb : {0, -1, 8, 1024})
        for (double trho : {10.0, 500.0, 2000.0}) {
          rexii_opts o;
          rexii_default_opts(&o);
          o.precision = prec;
          o.pole_batch = pb;
          o.tol = prec == REXII_PREC_MIXED ? 1e-6 : 1e-10;
          rexii_swe_op op = lrsw(gsz[0], gsz[1], 10.0);
          o.rho = 0.0;
          // t such that t rho ~ trho with rho <= sqrt(f^2 + 2 n^2)
          const double rho = std::sqrt(100.0 + 4.0 * (double(gsz[0]) * gsz[0] + double(gsz[1]) * gsz[1]));
          const double t = trho / rho;
          size_t b1 = 0, b2 = 0;
          CHECK(rexii_workspace_size(&op, &o, t, &b1) == REXII_OK);
          CHECK(rexii_batched_workspace_size(1, &op, &t, &o, &b2) == REXII_OK);
          CHECK(b1 > 0 && b2 > 0 && b2 <= b1);
        }
  // a heterogeneous batch of the batched configuration's shapes
  std::vector<rexii_swe_op> ops;
  std::vector<double> ts;
  const int sizes[] = {128, 256, 512, 1024};
  for (int i = 0; i < 64; ++i) {
    const int D = sizes[(i * 7) % 4];
    ops.push_back(lrsw(D, D, 10.0));
    ts.push_back((50.0 + 30.0 * i) / (1.5 * D));
  }
  ts[5] = 0.0;   // t = 0 states take no solves
  for (int pb : {0, -1, 64}) {
    rexii_opts o;
    rexii_default_opts(&o);
    o.precision = REXII_PREC_MIXED;
    o.tol = 1e-6;
    o.pole_batch = pb;
    size_t b = 0;
    CHECK(rexii_batched_workspace_size(int(ops.size()), ops.data(), ts.data(), &o, &b) == REXII_OK);
    CHECK(b > 0);
  }
  // invalid operators and options are refused on the host
  rexii_opts o;
  rexii_default_opts(&o);
  size_t b = 0;
  rexii_swe_op bad = lrsw(2, 8, 10.0);
  CHECK(rexii_workspace_size(&bad, &o, 1.0, &b) == REXII_ERR_INVALID_ARG);
  bad = lrsw(8, 8, 10.0);
  bad.g = -1.0;
  CHECK(rexii_workspace_size(&bad, &o, 1.0, &b) == REXII_ERR_INVALID_ARG);
  rexii_swe_op ok = lrsw(8, 8, 10.0);
  o.tile_rows = 7;
  o.method = 1;
  CHECK(rexii_workspace_size(&ok, &o, 1.0, &b) == REXII_ERR_INVALID_ARG);
  double t0 = -1.0;
  rexii_default_opts(&o);
  CHECK(rexii_batched_workspace_size(1, &ok, &t0, &o, &b) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_batched_workspace_size(0, &ok, &t0, &o, &b) == REXII_ERR_INVALID_ARG);
}

static void entry_point_checks() {
  // argument checks that return before any device work (pointers are never
  // dereferenced)
  const double* dummy = reinterpret_cast<const double*>(16);
  double* far = reinterpret_cast<double*>(size_t(1) << 30);
  rexii_swe_op op = lrsw(8, 8, 10.0);
  rexii_report rep;
  CHECK(rexii_apply(&op, dummy, const_cast<double*>(dummy), 1.0, nullptr, nullptr, 0, nullptr, &rep) ==
        REXII_ERR_INVALID_ARG);
  CHECK(rexii_apply(&op, nullptr, far, 1.0, nullptr, nullptr, 0, nullptr, &rep) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_apply_fourier(&op, dummy, far, 1.0, 5, nullptr, nullptr, 0, nullptr, &rep) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_apply_multishift(&op, 0, dummy, far, 1.0, nullptr, nullptr, 0, nullptr, &rep) ==
        REXII_ERR_INVALID_ARG);
  CHECK(rexii_apply_adjoint(&op, nullptr, dummy, nullptr, nullptr, 1.0, nullptr, nullptr, 0, nullptr, &rep) ==
        REXII_ERR_INVALID_ARG);
  // circulant: the premises, the exact rho and the term tables are host work;
  // an overlapping output is refused only after them
  const int n = 70;
  const int32_t off1[2] = {1, -1};
  const double c1[4] = {0.5 * n, 0.0, -0.5 * n, 0.0};
  const int32_t off2[3] = {-1, 0, 1};
  const double c2[6] = {0.0, 1225.0, 0.0, -2450.0, 0.0, 1225.0};
  const double* f = reinterpret_cast<const double*>(size_t(1) << 20);
  double* u_overlap = reinterpret_cast<double*>((size_t(1) << 20) + 8 * 35);
  for (int scheme : {REXII_CIRC_REXII, REXII_CIRC_REXI})
    for (int M : {0, 20, 151, 400})
      CHECK(rexii_apply_circulant(n, 2, off1, c1, 1, f, u_overlap, 1.0, 0.0, scheme, M, nullptr, nullptr, 0, nullptr,
                                  &rep) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_apply_circulant(n, 3, off2, c2, 1, f, u_overlap, 1.0, -2450.0, REXII_CIRC_REXIE, 0, nullptr, nullptr, 0,
                              nullptr, &rep) == REXII_ERR_INVALID_ARG);
  CHECK(rexii_apply_circulant(n, 3, off2, c2, 1, f, u_overlap, 1.0, 0.0, REXII_CIRC_REXII, 0, nullptr, nullptr, 0,
                              nullptr, &rep) == REXII_ERR_INVALID_ARG);   // A_2 is not real
}

int main() {
  coefficients();
  plans_and_sizes();
  entry_point_checks();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
