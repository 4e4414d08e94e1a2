"""Pins of the oracle's scalar REXII coefficients against closed forms and the
paper's printed values (Sec. 2, Appendices A and B)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import coeffs
from oracle.table_a import A_COEFFS, L, MU

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def test_table_a_fit_error():
    # Sec. 2.1 step 2: R approximates psi_1 with max error below 8e-15.
    x = np.linspace(-60.0, 60.0, 120001)
    err = np.max(np.abs(coeffs.R_complex(x) - coeffs.psi(x, 1.0)))
    # printed claim 8e-15; the 16-digit table leaves a little slack
    assert err < 1.5 * GOLDEN["table_A_fit_error_claim"]["max_error"]


def test_table_a_closed_form_matches_complex_form():
    # eq. A(x,mu) is the real closed form of eq. ratapproxgaush1 when
    # a_{-l} = conj(a_l).
    x = np.linspace(-80.0, 80.0, 4001)
    assert np.max(np.abs(coeffs.R_closed(x) - coeffs.R_complex(x))) < 1e-14


def test_table_a_sign_reading():
    # The other reading of the sign column (sign applies to both parts) does
    # not approximate the Gaussian at all.
    x = np.linspace(-60.0, 60.0, 6001)
    s = np.zeros_like(x, dtype=complex)
    # signs as printed: the entries whose real part is negative
    for l in range(-L, L + 1):
        re, im = A_COEFFS[abs(l)]
        if re < 0:
            im = -im
        al = complex(re, im if l >= 0 else -im)
        s += al / (1j * x + MU + 1j * l)
    assert np.max(np.abs(s.real - coeffs.psi(x, 1.0))) > 0.1


def test_gaussian_sum_reproduces_exponential():
    # eq. eixsumM with b_m from eq. bm: accurate for |x| <= (M - 11) h.
    h, M = 0.5, 60
    x = np.linspace(-(M - 11) * h, (M - 11) * h, 501)
    err = np.abs(coeffs.gaussian_sum(x, M, h) - np.exp(1j * x))
    assert err.max() < 1e-14


@pytest.mark.parametrize("h,bound", [(0.1, 1.5e-13), (0.5, 1e-13)])
def test_scalar_rexii_accuracy(h, bound):
    # eq. modifiedRexi with M from eq. Mformula is accurate to ~1e-13.
    xmax = 30.0
    M = coeffs.M_rule(1.0, xmax, h, 11)
    x = np.linspace(-xmax, xmax, 1201)
    err = np.abs(coeffs.rexii_scalar(x, M, h) - np.exp(1j * x))
    assert err.max() < bound


def test_scalar_rexii_h1_aliasing_floor():
    # At h = 1 the error floor is the aliasing term e^{4 pi h - 4 pi^2}
    # ~ 2.05e-12 of the Poisson-summation argument (Appendix B), matching the
    # ~2.8e-12 the paper prints for h = 1 (Table w11).
    h = 1.0
    M = coeffs.M_rule(1.0, 30.0, h, 11)
    x = np.linspace(-30.0, 30.0, 1201)
    err = np.abs(coeffs.rexii_scalar(x, M, h) - np.exp(1j * x)).max()
    floor = math.exp(4 * math.pi * h - 4 * math.pi ** 2)
    assert 0.5 * floor < err < 3.0 * floor


def test_sharp_drop_in_M():
    # Fig. exLB: the error drops to machine precision at M ~ |x|/h + 11.
    x, h = 30.0, 0.5
    good = coeffs.M_rule(1.0, x, h, 11)
    e_good = abs(coeffs.rexii_scalar(np.array([x]), good, h)[0] - np.exp(1j * x))
    e_bad = abs(coeffs.rexii_scalar(np.array([x]), good - 10, h)[0] - np.exp(1j * x))
    assert e_good < 1e-13
    assert e_bad > 1e-6


def test_rexi_and_rexii_agree_for_real_x():
    # Sec. 2.1: eqs. originalRexi and modifiedRexi are equivalent for real x.
    h, M = 0.5, 40
    x = np.linspace(-14.0, 14.0, 301)
    assert np.max(np.abs(coeffs.rexi_scalar(x, M, h) - coeffs.rexii_scalar(x, M, h))) < 1e-13


def test_m0_of_tol():
    # Appendix B: c ~ 12 at tol 1e-16, m0 = c - 1 ~ 11.
    assert coeffs.m0_of_tol(GOLDEN["m0"]["tol"]) == GOLDEN["m0"]["m0"]
    assert coeffs.m0_of_tol(1e-10) == 9
    assert coeffs.m0_of_tol(1e-6) == 7


@pytest.mark.parametrize("table", ["w11", "w150"])
def test_M_rule_wave1(table):
    # Sec. 4, wave scenario 1: M = ceil(sqrt(2) pi 6 tau / h) + 11.
    tab = GOLDEN[table]
    for row in tab["rows"]:
        M = coeffs.M_rule(tab["tau"], math.sqrt(2) * math.pi * tab["D_eff"], row["h"], 11)
        assert M == row["M"], (table, row)


def test_M_rule_gaussian():
    # Table G1001 with rho from eq. lswRoh at D = 128.
    tab = GOLDEN["G1001"]
    rho = math.sqrt(2 * math.pi ** 2 * tab["D"] ** 2 + 1)
    for row in tab["rows"]:
        assert coeffs.M_rule(tab["tau"], rho, row["h"], 11) == row["M"]


def test_c_coefficient_symmetry():
    # Sec. 2.2 remark: conj(c_{1,n}) = c_{1,-n}, conj(c_{2,n}) = -c_{2,-n}.
    ns, c1, c2 = coeffs.c_coefs(30, 0.5)
    scale = np.max(np.abs(c1))
    assert np.max(np.abs(np.conj(c1) - c1[::-1])) < 1e-15 * scale
    assert np.max(np.abs(np.conj(c2) + c2[::-1])) < 1e-15 * scale


@pytest.mark.parametrize("theta", [0.3, 30.0, 300.0, 1000.0])
def test_partial_fractions_on_rotation_generator(theta):
    # exp of [[0, theta], [-theta, 0]] is the rotation by theta (textbook).
    h = 0.5
    M = coeffs.M_rule(1.0, theta, h, 11)
    z, w = coeffs.poles_weights(M, h)
    A = np.array([[0.0, theta], [-theta, 0.0]])
    f = np.array([0.7, -1.3])
    u = np.zeros(2, dtype=complex)
    for zk, wk in zip(z, w):
        u += wk * np.linalg.solve(A - zk * np.eye(2), f)
    ex = np.array([[math.cos(theta), math.sin(theta)], [-math.sin(theta), math.cos(theta)]]) @ f
    # rounding in the pole sum grows mildly with theta (about P terms)
    assert np.max(np.abs(u.real - ex)) < 1e-13 * max(1.0, theta / 500.0)


def test_partial_fractions_equal_nested_two_solve_form():
    # The pole/weight split equals the paper's two-solve term (Sec. 4).
    from oracle import lrsw
    op = lrsw.LRSW(6, 6, g=1.0, H=1.0, fc=3.0)
    rng = np.random.default_rng(0)
    f = rng.standard_normal(op.n)
    tA = 0.4 * lrsw.dense_A(op)
    M, h = 25, 0.5
    z, w = coeffs.poles_weights(M, h)
    u = np.zeros(op.n, dtype=complex)
    for zk, wk in zip(z, w):
        u += wk * np.linalg.solve(tA - zk * np.eye(op.n), f)
    nested = coeffs.nested_matrix_apply(tA, f, M, h)
    assert np.max(np.abs(u.real - nested)) < 1e-13 * np.max(np.abs(nested))


def test_pole_structure_and_counts():
    h = 0.5
    c = coeffs.api_coeffs(100.0 / 91.06041950265768, 91.06041950265768, h=h, tol=1e-10)
    assert c["m0"] == 9 and c["P"] == 468
    z = c["z"]
    assert np.allclose(z[0::2].real, h * MU) and np.allclose(z[1::2].real, -h * MU)
    assert np.allclose(z[1::2], -np.conj(z[0::2]))
    # kappa_sum grows with t rho (about 2.3e2 at t rho = 100).
    assert 200.0 < c["kappa_sum"] < 260.0
