"""The exact REXII approximant r(tA) f = Re sum_k w_k (tA - z_k I)^{-1} f for the
constant-depth centred-difference LRSW operator, solved per Fourier mode
(no Krylov iterations), and single-pole resolvents.

Test infrastructure only (see the oracle package docstring).

Theorem 1 of the paper (eq. teorem) evaluates the rational function on the
spectrum: with A = V E V^{-1}, r(tA) = V r(tE) V^{-1}.  Per mode the block
t A_hat has eigenvalues 0 and +-i omega t, so r(t A_hat) is the quadratic in
t A_hat that interpolates r at those three points.  With Newton divided
differences on the nodes (0, i theta, -i theta), theta = omega t,
    r(X) = r(0) I + r[0, i theta] X + r[0, i theta, -i theta] X (X - i theta I).
For one pole 1/(x - z) the divided differences are exact products:
1/(x1-z)(x2-z) (with a minus sign) and 1/(x1-z)(x2-z)(x3-z), so the formula
stays exact at theta = 0 and needs no division by theta.

The real part is taken in physical space, after the inverse FFT
(eq. modifiedRexiMatrixReducedSum is a statement about a real operator and a
real vector).
"""
import numpy as np

from . import lrsw


def resolvent_modes(op, f, t, z):
    """x = (tA - z I)^{-1} f (complex, [3][ny][nx]) by a 3x3 solve per mode."""
    Ah = lrsw.symbol(op)
    F = lrsw.to_modes(f).transpose(1, 2, 0)[..., None]
    K = t * Ah - z * np.eye(3)[None, None]
    X = np.linalg.solve(K, F)[..., 0].transpose(2, 0, 1)
    return lrsw.from_modes(X)


def rexii_direct(op, f, t, z, w):
    """Re sum_k w_k (tA - z_k)^{-1} f with one batched 3x3 solve per pole and
    mode (the plain definition; small grids and pole counts)."""
    Ah = lrsw.symbol(op)
    F = lrsw.to_modes(f).transpose(1, 2, 0)[..., None]
    I3 = np.eye(3)[None, None]
    acc = np.zeros(F.shape, dtype=np.complex128)
    for zk, wk in zip(z, w):
        acc += wk * np.linalg.solve(t * Ah - zk * I3, F)
    return lrsw.from_modes(acc[..., 0].transpose(2, 0, 1)).real


def divided_differences(theta, z, w):
    """(r(0), r[0, i theta], r[0, i theta, -i theta]) for r(x) = sum_k w_k/(x - z_k),
    for every value in the array theta."""
    th = np.asarray(theta, dtype=np.float64).ravel()
    d0 = np.zeros(th.shape, dtype=np.complex128)
    d1 = np.zeros(th.shape, dtype=np.complex128)
    d2 = np.zeros(th.shape, dtype=np.complex128)
    # chunk over poles to bound memory
    for s in range(0, len(z), 256):
        zk = z[s:s + 256][None, :]
        wk = w[s:s + 256][None, :]
        a0 = 1.0 / (0.0 - zk)
        ap = 1.0 / (1j * th[:, None] - zk)
        am = 1.0 / (-1j * th[:, None] - zk)
        d0 += np.sum(wk * a0, axis=1)
        d1 += -np.sum(wk * a0 * ap, axis=1)
        d2 += np.sum(wk * a0 * ap * am, axis=1)
    return d0, d1, d2


def rexii_symbol(Ah, om, F, t, z, w):
    """r(t A_hat) F per mode for any symbol with eigenvalues 0, +-i om
    (module docstring); returns the complex modal result."""
    theta = om * t
    uniq, inv = np.unique(theta, return_inverse=True)
    d0, d1, d2 = divided_differences(uniq, np.asarray(z), np.asarray(w))
    inv = inv.reshape(theta.shape)
    D0, D1, D2 = d0[inv], d1[inv], d2[inv]
    XF = t * lrsw.modes_matvec(Ah, F)
    XXF = t * lrsw.modes_matvec(Ah, XF)
    # r(X) F = d0 F + d1 X F + d2 (X^2 F - i theta X F)
    return D0[None] * F + D1[None] * XF + D2[None] * (XXF - 1j * theta[None] * XF)


def rexii_spectral(op, f, t, z, w, return_complex=False):
    """Re sum_k w_k (tA - z_k)^{-1} f through the spectral interpolation
    described in the module docstring (cost O(P * distinct omega + D^2))."""
    S = rexii_symbol(lrsw.symbol(op), lrsw.omega(op), lrsw.to_modes(f), t, z, w)
    u = lrsw.from_modes(S)
    return u if return_complex else u.real


def rexii_dense(op, f, t, z, w):
    """Re sum_k w_k (tA - z_k I)^{-1} f with dense solves on the assembled
    operator (any depth; small grids only)."""
    A = lrsw.dense_A(op)
    I = np.eye(A.shape[0])
    b = np.asarray(f, dtype=np.float64).ravel()
    acc = np.zeros(A.shape[0], dtype=np.complex128)
    for zk, wk in zip(z, w):
        acc += wk * np.linalg.solve(t * A - zk * I, b)
    return acc.real.reshape(3, op.ny, op.nx)
