"""Pins of the oracle's refit of the Gaussian's rational approximation
(Sec. 2.1, step 2: eqs. ratapproxgaush1, A(x,mu), minl2approx; Appendix A),
and parity of the library's rexii_fit_gaussian (host code, through the C
ABI) with it.  No GPU needed."""
import math
import os

import numpy as np
import pytest

from oracle import refit as rf
from oracle.table_a import L, MU, a as a_printed

XF = np.linspace(-60.0, 60.0, 120001)


@pytest.fixture(scope="module")
def oracle_fit():
    return rf.refit()


def test_symmetric_form_is_the_complex_sum():
    # eq. A(x,mu) restates Re sum_{l=-L}^{L} a_l / (i x + mu + i l) with
    # a_{-l} = conj(a_l) (eq. ratapproxgaush1): checked for random coefficients
    rng = np.random.default_rng(3)
    a = rng.standard_normal(L + 1) + 1j * rng.standard_normal(L + 1)
    a[0] = a[0].real
    x = np.linspace(-40.0, 40.0, 801)
    direct = np.zeros_like(x)
    for l in range(-L, L + 1):
        al = a[l] if l >= 0 else np.conj(a[-l])
        direct += (al / (1j * x + MU + 1j * l)).real
    assert np.max(np.abs(rf.R_of(a, x) - direct)) <= 1e-13 * np.max(np.abs(direct))


def test_leja_order():
    # x_1 = 0; x_2 maximises |x| on [0, X]; x_3 maximises x (X - x); x_4 is
    # the smaller of the mirror pair maximising x (X - x) |x - X/2|
    c = 60.0 * np.arange(6001) / 6000
    p = rf.leja_points(c, 4)
    assert p[0] == 0.0 and p[1] == 60.0 and p[2] == 30.0
    r = 30.0 - 30.0 / math.sqrt(3.0)       # roots of the derivative of x (60 - x) (x - 30)
    assert abs(p[3] - r) <= 0.01 + 1e-12
    assert len(np.unique(rf.leja_points(c, 200))) == 200


def test_refit_reaches_the_printed_accuracy(oracle_fit):
    # the paper's fit is within 8e-15 of psi_1 (Sec. 2.1); evaluated here the
    # printed table is within 1.4e-14 on [-60, 60], and the refit within
    # 2e-14 (reading: the paper's K, interval and mu are not given)
    a, _ = oracle_fit
    pr = np.array([a_printed(l) for l in range(L + 1)])
    e_printed = np.max(np.abs(rf.R_of(pr, XF) - rf.psi1(XF)))
    e_refit = np.max(np.abs(rf.R_of(a, XF) - rf.psi1(XF)))
    assert e_printed <= 1.5e-14
    assert e_refit <= 2e-14
    # the two fits are the same function to within their errors
    assert np.max(np.abs(rf.R_of(a, XF) - rf.R_of(pr, XF))) <= 3e-14
    # and the same coefficients to the conditioning of the problem
    assert np.max(np.abs(a - pr)) <= 1e-3 * np.max(np.abs(pr))


def test_refit_is_a_least_squares_solution(oracle_fit):
    # the normal equations hold at the chosen points: G^T (b - G y) ~ 0
    a, pts = oracle_fit
    G = rf.design_matrix(pts)
    y = np.concatenate([[a[0].real], a[1:].real, a[1:].imag])
    r = rf.psi1(pts) - G @ y
    assert np.max(np.abs(G.T @ r)) <= 1e-13 * np.linalg.norm(G) * np.linalg.norm(rf.psi1(pts))


def test_refit_fails_without_the_refinement():
    # the plain orthogonal solve stops near 5e-14: the refinement step is what
    # reaches the printed accuracy (so a dropped refinement fails the pin above)
    cand = 60.0 * np.arange(200001) / 200000
    pts = rf.leja_points(cand, 200)
    y, *_ = np.linalg.lstsq(rf.design_matrix(pts), rf.psi1(pts), rcond=None)
    e = np.max(np.abs(rf.design_matrix(XF) @ y - rf.psi1(XF)))
    assert e >= 2e-14


def test_library_refit_matches_oracle(oracle_fit):
    from paper_2008_11607_amd import rexii
    if not os.path.exists(rexii.LIB_PATH):
        from paper_2008_11607_amd import build
        build.build()
    a_lib, pts_lib, err = rexii.fit_gaussian()
    a_or, pts_or = oracle_fit
    assert np.array_equal(pts_lib, pts_or)              # the same Leja points, bit for bit
    assert np.max(np.abs(rf.R_of(a_lib, XF) - rf.psi1(XF))) <= 2e-14
    assert np.max(np.abs(rf.R_of(a_lib, XF) - rf.R_of(a_or, XF))) <= 3e-14
    assert np.max(np.abs(a_lib - a_or)) <= 1e-8 * np.max(np.abs(a_or))
    assert 0.0 < err <= 2e-14
    # a smaller problem: L = 8 on [0, 30] (a coarser fit, same method)
    a8, p8, e8 = rexii.fit_gaussian(L=8, x_max=30.0, K=60, n_candidates=30001)
    o8, q8 = rf.refit(K=60, x_max=30.0, n_candidates=30001, L=8)
    assert np.array_equal(p8, q8)
    x = np.linspace(-30.0, 30.0, 6001)
    assert np.max(np.abs(rf.R_of(a8, x) - rf.R_of(o8, x))) <= 1e-12
    assert abs(e8 - np.max(np.abs(rf.R_of(o8, x) - rf.psi1(x)))) <= 0.1 * e8 + 1e-15


def test_library_refit_rejects_bad_arguments():
    import ctypes
    from paper_2008_11607_amd import rexii
    lib = rexii.load()
    a = np.zeros(2 * 25)
    ptr = a.ctypes.data_as(ctypes.c_void_p)
    assert lib.rexii_fit_gaussian(24, MU, 60.0, 40, 1000, ptr, None, None) == -1     # K < 2L + 1
    assert lib.rexii_fit_gaussian(0, MU, 60.0, 200, 1000, ptr, None, None) == -1
    assert lib.rexii_fit_gaussian(24, 0.0, 60.0, 200, 1000, ptr, None, None) == -1
    assert lib.rexii_fit_gaussian(24, MU, -1.0, 200, 1000, ptr, None, None) == -1
    assert lib.rexii_fit_gaussian(24, MU, 60.0, 200, 100, ptr, None, None) == -1     # fewer candidates than K
    assert lib.rexii_fit_gaussian(24, MU, 60.0, 200, 1000, None, None, None) == -1
