"""Pins of the oracle's operator and exact exponential: dense assembly vs
Fourier symbol, three independent exponentials, invariants."""
import numpy as np
import pytest

from oracle import expm_modes as em
from oracle import lrsw, varh
from paper_2008_11607_amd import inputs


def _f(nx, ny, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, ny, nx))


@pytest.mark.parametrize("nx,ny,g,H,fc", [(8, 8, 1.0, 1.0, 10.0), (10, 6, 2.0, 0.5, 3.0),
                                          (7, 9, 1.0, 1.0, 0.0)])
def test_symbol_matches_stencil(nx, ny, g, H, fc):
    # The FFT symbol applied per mode equals the centred-difference stencil.
    op = lrsw.LRSW(nx, ny, g=g, H=H, fc=fc)
    f = _f(nx, ny, 1)
    Af = lrsw.from_modes(lrsw.modes_matvec(lrsw.symbol(op), lrsw.to_modes(f))).real
    assert np.max(np.abs(Af - lrsw.apply_A(op, f))) < 1e-12 * np.max(np.abs(Af))


@pytest.mark.parametrize("nx,ny,g,H,fc,t", [(8, 8, 1.0, 1.0, 10.0, 0.7), (10, 6, 2.0, 0.5, 3.0, 1.3),
                                            (12, 12, 1.0, 1.0, 10.0, 5.0)])
def test_three_exponentials_agree(nx, ny, g, H, fc, t):
    # Cayley-Hamilton closed form == Hermitian eigendecomposition == dense expm.
    op = lrsw.LRSW(nx, ny, g=g, H=H, fc=fc)
    f = _f(nx, ny, 2)
    ref = em.expm_dense(op, f, t)
    u1 = em.expm_closed(op, f, t)
    assert np.max(np.abs(u1.imag)) < 1e-13
    assert em.rel_l2(u1.real, ref) < 1e-12
    assert em.rel_l2(em.expm_eigh(op, f, t), ref) < 1e-12


def test_zero_frequency_mode_series():
    # f_c = 0 has omega = 0 at the zero mode; the sinc form stays exact.
    op = lrsw.LRSW(8, 8, fc=0.0)
    f = _f(8, 8, 3)
    assert em.rel_l2(em.expm_closed_real(op, f, 0.9), em.expm_dense(op, f, 0.9)) < 1e-12


def test_energy_and_group_property():
    op = lrsw.LRSW(32, 32, g=1.0, H=1.0, fc=10.0)
    f = inputs.gaussian_bumps(32, nbumps=4, seed=7, velocity=True)
    t = 3.3
    u = em.expm_closed_real(op, f, t)
    # W A skew => ||exp(tA) f||_W = ||f||_W
    assert abs(em.energy(op, u) / em.energy(op, f) - 1.0) < 1e-13
    # exp(2tA) f = exp(tA) exp(tA) f
    assert em.rel_l2(em.expm_closed_real(op, u, t), em.expm_closed_real(op, f, 2 * t)) < 1e-13
    # exp(-tA) exp(tA) f = f
    assert em.rel_l2(em.expm_closed_real(op, u, -t), f) < 1e-13


def test_energy_in_W_norm_when_g_ne_H():
    op = lrsw.LRSW(16, 16, g=2.0, H=0.5, fc=4.0)
    f = _f(16, 16, 4)
    u = em.expm_closed_real(op, f, 2.0)
    assert abs(em.energy(op, u) / em.energy(op, f) - 1.0) < 1e-13
    # the plain norm is not conserved here
    assert abs(np.sum(u ** 2) / np.sum(f ** 2) - 1.0) > 1e-6


@pytest.mark.parametrize("nx,ny,fc", [(8, 8, 10.0), (16, 16, 20.0), (12, 8, 1.0), (6, 10, 0.0)])
def test_rho_exact_constant_depth(nx, ny, fc):
    op = lrsw.LRSW(nx, ny, fc=fc)
    lam = np.linalg.eigvals(lrsw.dense_A(op))
    assert abs(lrsw.rho(op) - np.max(np.abs(lam))) < 1e-9 * lrsw.rho(op)
    assert np.max(np.abs(lam.real)) < 1e-9 * lrsw.rho(op)


def test_rho_closed_form_when_four_divides_D():
    # max(s_x^2 + s_y^2) = 2 D^2 when 4 | D: rho = sqrt(f_c^2 + 2 g H D^2).
    op = lrsw.LRSW(64, 64, fc=10.0)
    assert abs(lrsw.rho(op) - 91.06041950265768) < 1e-10


@pytest.mark.parametrize("n", [8, 12])
def test_rho_bound_variable_depth(n):
    op = lrsw.LRSW(n, n, fc=5.0, Hfield=inputs.variable_depth(n))
    lam = np.linalg.eigvals(lrsw.dense_A(op))
    assert np.max(np.abs(lam.real)) < 1e-9 * np.max(np.abs(lam))
    assert lrsw.rho(op) >= np.max(np.abs(lam))


def test_variable_depth_is_W_skew():
    op = lrsw.LRSW(8, 8, g=1.5, fc=7.0, Hfield=inputs.variable_depth(8))
    A = lrsw.dense_A(op)
    W = np.diag(np.concatenate([np.full(64, 1.5), op.Hfield.ravel(), op.Hfield.ravel()]))
    assert np.max(np.abs(W @ A + (W @ A).T)) < 1e-12 * np.max(np.abs(A))


def test_chebyshev_matches_dense_variable_depth():
    op = lrsw.LRSW(8, 8, fc=10.0, Hfield=inputs.variable_depth(8))
    f = inputs.gaussian_bumps(8, nbumps=3, seed=9, velocity=True)
    t = 40.0 / lrsw.rho(op)
    ref = em.expm_dense(op, f, t)
    u = varh.chebyshev_expm(op, f, t)
    assert em.rel_l2(u, ref) < 1e-12
    assert abs(varh.w_energy(op, u) / varh.w_energy(op, f) - 1.0) < 1e-12
