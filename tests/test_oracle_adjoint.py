"""Pins of the oracle's gradients: dot tests against dense transposes,
central finite differences, and the 6x6 block-exponential Frechet derivative."""
import numpy as np
import scipy.linalg

from oracle import adjoint as adj
from oracle import coeffs, lrsw
from oracle import expm_modes as em
from oracle import rexii_modes as rm
from paper_2008_11607_amd import inputs


def _setup(n=12, trho=30.0, seed=11):
    op = lrsw.LRSW(n, n, fc=10.0)
    rho = lrsw.rho(op)
    t = trho / rho
    c = coeffs.api_coeffs(t, rho, h=0.5, tol=1e-10)
    f = inputs.gaussian_bumps(n, nbumps=2, seed=seed, velocity=True)
    idx = inputs.sample_indices(n, n, 20, seed + 1)
    y = np.random.default_rng(seed + 2).standard_normal(20)
    return op, t, c, f, idx, y


def test_transposes_against_dense():
    op, t, c, f, idx, y = _setup(8)
    g = np.random.default_rng(5).standard_normal(f.shape)
    A = lrsw.dense_A(op)
    eT = (scipy.linalg.expm(t * A).T @ g.ravel()).reshape(g.shape)
    assert em.rel_l2(adj.expm_T_apply(op, g, t), eT) < 1e-12
    I = np.eye(A.shape[0])
    rT = np.zeros(A.shape[0], dtype=complex)
    for zk, wk in zip(c["z"], c["w"]):
        rT += wk * np.linalg.solve(t * A.T - zk * I, g.ravel())
    rT = rT.real.reshape(g.shape)
    assert em.rel_l2(adj.rexii_T_apply(op, g, t, c["z"], c["w"]), rT) < 1e-12
    assert em.rel_l2(adj.rexii_T_spectral(op, g, t, c["z"], c["w"]), rT) < 1e-12


def test_rexii_dot_test():
    op, t, c, f, idx, y = _setup(16)
    g = np.random.default_rng(6).standard_normal(f.shape)
    lhs = np.sum(rm.rexii_spectral(op, f, t, c["z"], c["w"]) * g)
    rhs = np.sum(f * adj.rexii_T_spectral(op, g, t, c["z"], c["w"]))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_dJdf_central_differences():
    # J is quadratic in f, so central differences are exact up to rounding.
    op, t, c, f, idx, y = _setup(12)
    J0, dJdf, _ = adj.grad_rexii(op, f, t, c["z"], c["w"], idx, y)
    rng = np.random.default_rng(9)
    eps = 1e-6
    for _ in range(3):
        d = rng.standard_normal(f.shape)
        Jp = adj.loss(rm.rexii_spectral(op, f + eps * d, t, c["z"], c["w"]), idx, y)
        Jm = adj.loss(rm.rexii_spectral(op, f - eps * d, t, c["z"], c["w"]), idx, y)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - np.sum(dJdf * d)) < 1e-7 * max(1.0, abs(fd))


def test_dJdH_central_differences():
    op, t, c, f, idx, y = _setup(12)
    _, _, dJdH = adj.grad_rexii(op, f, t, c["z"], c["w"], idx, y)
    _, _, dJdH_ex = adj.grad_exact(op, f, t, idx, y)
    eps = 1e-5
    opp = lrsw.LRSW(op.nx, op.ny, g=op.g, H=op.H + eps, fc=op.fc)
    opm = lrsw.LRSW(op.nx, op.ny, g=op.g, H=op.H - eps, fc=op.fc)
    Jp = adj.loss(rm.rexii_spectral(opp, f, t, c["z"], c["w"]), idx, y)
    Jm = adj.loss(rm.rexii_spectral(opm, f, t, c["z"], c["w"]), idx, y)
    fd = (Jp - Jm) / (2 * eps)
    assert abs(fd - dJdH) < 1e-7 * max(1.0, abs(fd))
    # exact exponential vs approximant: equal to the approximation error
    assert abs(dJdH - dJdH_ex) < 1e-9 * max(1.0, abs(dJdH_ex))
    Jpe = adj.loss(em.expm_closed_real(opp, f, t), idx, y)
    Jme = adj.loss(em.expm_closed_real(opm, f, t), idx, y)
    assert abs((Jpe - Jme) / (2 * eps) - dJdH_ex) < 1e-7 * max(1.0, abs(dJdH_ex))


def test_frechet_eigenbasis_vs_block_expm():
    op, t, c, f, idx, y = _setup(10)
    modes = [(0, 1), (3, 2), (5, 5), (7, 9), (0, 0)]
    blk = adj.frechet_exp_block(op, f, t, modes)
    # frechet_exp_apply returns the real physical field; compare its modes to
    # the block result symmetrised the same way (real part in physical space)
    full = np.zeros((3, op.ny, op.nx), dtype=complex)
    X = t * lrsw.symbol(op)
    Ef = adj._E_hat(op) * t
    F = lrsw.to_modes(f)
    for ky in range(op.ny):
        for kx in range(op.nx):
            Blk = np.zeros((6, 6), dtype=complex)
            Blk[:3, :3] = X[ky, kx]
            Blk[:3, 3:] = Ef[ky, kx]
            Blk[3:, 3:] = X[ky, kx]
            full[:, ky, kx] = scipy.linalg.expm(Blk)[:3, 3:] @ F[:, ky, kx]
    ref = lrsw.from_modes(full).real
    assert em.rel_l2(adj.frechet_exp_apply(op, f, t), ref) < 1e-11
    for (ky, kx), b in zip(modes, blk):
        assert np.allclose(b, full[:, ky, kx])
