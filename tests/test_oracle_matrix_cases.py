"""Pins of the oracle's matrix test cases and comparison schemes (Sec. 3.2,
Fig. matrixRexiExample; eqs. modifiedRexiMatrixReducedSum, originalREXImatrix,
REXIE; the remark on shifted matrices in Sec. 2.2)."""
import math

import numpy as np
import pytest

from oracle import coeffs as oc
from oracle import matrix_cases as mc

N_PTS = 70


@pytest.fixture(scope="module")
def case1():
    st = mc.stencil_A1(N_PTS)
    A = mc.circulant_dense(N_PTS, st)
    f = mc.f0(mc.grid_A1(N_PTS))
    return st, A, f, mc.expm_dense(A, f).real


@pytest.fixture(scope="module")
def case2():
    st = mc.stencil_A2(N_PTS)
    A = mc.circulant_dense(N_PTS, st)
    f = mc.f0(mc.grid_A2(N_PTS))
    return st, A, f, mc.expm_dense(A, f)


def test_spectra_as_stated(case1, case2):
    # A_1: real skew-symmetric, eigenvalues in i[-70, 70]; A_2: i times a real
    # symmetric matrix, eigenvalues in i[-4900, 0] (Sec. 3.2)
    _, A1, _, _ = case1
    _, A2, _, _ = case2
    assert np.all(A1.imag == 0) and np.array_equal(A1.real, -A1.real.T)
    e1 = np.linalg.eigvals(A1.real)
    assert np.max(np.abs(e1.real)) < 1e-12 and 69.9 < np.max(np.abs(e1.imag)) <= 70.0
    B2 = (A2 / 1j)
    assert np.max(np.abs(B2.imag)) == 0 and np.array_equal(B2.real, B2.real.T)
    e2 = np.linalg.eigvalsh(B2.real)
    assert -4900.0 - 1e-9 <= e2.min() < -4899.9 and abs(e2.max()) < 1e-9


def test_circulant_exponential_is_the_dense_one(case1, case2):
    # the DFT diagonalises a circulant matrix: exp by eigenvalues = Pade expm
    for st, _, f, ref in (case1, case2):
        assert mc.rel_l2(mc.expm_circulant(N_PTS, st, f), ref) <= 1e-12


@pytest.mark.parametrize("h", [0.2, 0.5])
def test_rexii_error_follows_the_bound(case1, h):
    # Fig. matrixRexiExample (a): REXII is accurate once (M - 11) h >= rho(A)
    # (eq. matrixAccuracyBound) and not before
    st, A, f, ref = case1
    rho = float(np.max(np.abs(mc.circulant_symbol(N_PTS, st))))
    M = oc.M_rule(1.0, rho, h, 11)
    assert mc.rel_l2(mc.rexii_dense(A.real, f, M, h), ref) <= 1e-13
    M_short = oc.M_rule(1.0, 50.0, h, 11)
    assert mc.rel_l2(mc.rexii_dense(A.real, f, M_short, h), ref) >= 1e-7


def test_rexii_floor_at_h1(case1):
    # at h = 1 the error stops at the aliasing floor e^{4 pi h - 4 pi^2}
    st, A, f, ref = case1
    floor = math.exp(4.0 * math.pi - 4.0 * math.pi ** 2)
    for M in (81, 151):
        e = mc.rel_l2(mc.rexii_dense(A.real, f, M, 1.0), ref)
        assert 0.5 * floor <= e <= 2.0 * floor


def test_rexi_has_no_such_bound(case1):
    # Fig. matrixRexiExample (b): the original REXI (eq. originalREXImatrix)
    # stays far above REXII's accuracy for the same M, even with M several
    # times the bound's value (A_1 has complex eigenvectors)
    st, A, f, ref = case1
    h = 0.5
    for reach in (70.0, 140.0, 400.0):
        M = oc.M_rule(1.0, reach, h, 11)
        e_rexi = mc.rel_l2(mc.rexi_dense(A.real, f, M, h), ref)
        e_rexii = mc.rel_l2(mc.rexii_dense(A.real, f, M, h), ref)
        assert e_rexi >= 1e-7 and e_rexi >= 1e6 * e_rexii


def test_rexie_on_shifted_schroedinger(case2):
    # Fig. matrixRexiExample (c): REXIE (eq. REXIE) on A_2 with the shift
    # nu = -2450 i (rho(A - nu I) = 2450) is accurate at the M of the bound
    # for 2450 and not below it
    st, A, f, ref = case2
    h, nu = 0.5, -2450j
    M = oc.M_rule(1.0, 2450.0, h, 11)
    assert mc.rel_l2(mc.rexie_dense(A, f, M, h, nu=nu), ref) <= 1e-12
    assert mc.rel_l2(mc.rexie_dense(A, f, oc.M_rule(1.0, 2300.0, h, 11), h, nu=nu), ref) >= 0.1


def test_rexie_shift_halves_the_terms(case2):
    # without the shift rho = 4900: the M for 2450 misses the modes with
    # |lambda| > 2450 (f_0 is smooth, so little of its energy sits there, but
    # far more than the tolerance), the M for 4900 is enough (remark on
    # shifted matrices, Sec. 2.2)
    st, A, f, ref = case2
    h = 0.5
    assert mc.rel_l2(mc.rexie_circulant(N_PTS, st, f, oc.M_rule(1.0, 2450.0, h, 11), h), ref) >= 1e-8
    assert mc.rel_l2(mc.rexie_circulant(N_PTS, st, f, oc.M_rule(1.0, 4900.0, h, 11), h), ref) <= 1e-12


def test_rexie_needs_real_eigenvectors(case1):
    # A_1 = i B with B = -i A_1 Hermitian but not real: its eigenvectors are
    # complex, and REXIE does not converge to exp(A_1) f
    st, A, f, ref = case1
    M = oc.M_rule(1.0, 400.0, 0.5, 11)
    assert mc.rel_l2(mc.rexie_circulant(N_PTS, st, f, M, 0.5), ref) >= 1e-6


@pytest.mark.parametrize("scheme", ["rexii", "rexi", "rexie"])
def test_per_mode_forms_equal_dense_solves(case1, case2, scheme):
    # the per-Fourier-mode evaluation of each scheme (used for circulant
    # matrices of any size) equals the dense-solve form up to rounding
    h = 0.5
    if scheme == "rexie":
        st, A, f, _ = case2
        M = oc.M_rule(1.0, 2450.0, h, 11)
        d = mc.rexie_dense(A, f, M, h, nu=-2450j)
        c = mc.rexie_circulant(N_PTS, st, f, M, h, nu=-2450j)
    else:
        st, A, f, _ = case1
        M = oc.M_rule(1.0, 70.0, h, 11)
        d = (mc.rexii_dense if scheme == "rexii" else mc.rexi_dense)(A.real, f, M, h)
        c = (mc.rexii_circulant if scheme == "rexii" else mc.rexi_circulant)(N_PTS, st, f, M, h)
    assert mc.rel_l2(c, d) <= 1e-12
