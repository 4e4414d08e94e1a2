"""Exact u = exp(tA) f for the centred-difference LRSW operator.

Test infrastructure only (see the oracle package docstring).

For constant depth the operator is diagonalised by the 2-D FFT into 3x3
blocks A_hat(k) (Sec. 2.1, eqs. AisVEV and REXI_VEV_DECOMP: matrix functions
via the eigendecomposition).  Each block has characteristic polynomial
lambda^3 + omega^2 lambda, so by Cayley-Hamilton
    exp(t A_hat) = I + (sin(omega t)/omega) A_hat + ((1 - cos(omega t))/omega^2) A_hat^2.
The same result is also computed from a Hermitian eigendecomposition
(cross-check) and, on small grids, from a dense matrix exponential.
"""
import numpy as np
import scipy.linalg

from . import lrsw


def expm_closed(op, f, t):
    """exp(tA) f via the per-mode Cayley-Hamilton closed form.
    sin(wt)/w = t sinc(wt/pi) and (1-cos wt)/w^2 = (t^2/2) sinc(wt/(2 pi))^2
    (numpy's sinc(x) = sin(pi x)/(pi x)) stay exact as w t -> 0."""
    Ah = lrsw.symbol(op)
    w = lrsw.omega(op)
    F = lrsw.to_modes(f)
    AF = lrsw.modes_matvec(Ah, F)
    AAF = lrsw.modes_matvec(Ah, AF)
    s1 = t * np.sinc(w * t / np.pi)
    s2 = 0.5 * t * t * np.sinc(w * t / (2.0 * np.pi)) ** 2
    U = F + s1[None] * AF + s2[None] * AAF
    return lrsw.from_modes(U)


def expm_closed_real(op, f, t):
    """Real part of expm_closed; the discarded imaginary part is rounding."""
    return expm_closed(op, f, t).real


def expm_eigh(op, f, t):
    """exp(tA) f from the eigendecomposition of the Hermitian matrix
    i W^{1/2} A_hat W^{-1/2} (W = diag(g, H, H)), independent of the closed
    form.  Returns the real part."""
    Ah = lrsw.symbol(op)
    s = np.sqrt(np.array([op.g, op.H, op.H]))
    S = s[None, None, :, None] * Ah / s[None, None, None, :]
    lam, V = np.linalg.eigh(1j * S)                 # S = -i V diag(lam) V^H
    F = lrsw.to_modes(f)
    G = (s[:, None, None] * F).transpose(1, 2, 0)[..., None]      # [y][x][3][1]
    VhG = np.conj(np.swapaxes(V, -1, -2)) @ G
    E = np.exp(-1j * t * lam)[..., None] * VhG
    U = (V @ E)[..., 0].transpose(2, 0, 1) / s[:, None, None]
    return lrsw.from_modes(U).real


def expm_dense(op, f, t):
    """exp(tA) f with scipy's dense matrix exponential of the assembled
    operator (small grids; works for variable depth too)."""
    A = lrsw.dense_A(op)
    return (scipy.linalg.expm(t * A) @ np.asarray(f).ravel()).reshape(3, op.ny, op.nx)


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 over all components."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def energy(op, f):
    """Discrete energy ||f||_W^2 = g|eta|^2 + sum H (u^2 + v^2); conserved by
    exp(tA) because W A is skew-symmetric."""
    Hd = op.depth()
    return float(op.g * np.sum(f[0] ** 2) + np.sum(Hd * (f[1] ** 2 + f[2] ** 2)))
