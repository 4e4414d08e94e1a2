"""Gradients of J = |P u - y|^2 with u = exp(tA) f (exact) or u = r(tA) f (the
REXII approximant), with respect to the initial state f and the constant
depth H.  P samples eta at given flat indices.

Test infrastructure only (see the oracle package docstring).

Per Fourier mode (constant depth) the transpose of the real operator A is the
conjugate transpose of its block: A^T <-> A_hat(k)^H.  The depth enters A
linearly, dA/dH = E with E f = (-dx u - dy v, 0, 0), E_hat =
[[0, -i s_x, -i s_y], 0, 0].  The derivative of a matrix function in a
direction (its Frechet derivative) is computed in the eigenbasis:
L_phi(X, Y) = V (Delta o (V^{-1} Y V)) V^{-1} with Delta_ij the divided
difference phi[lambda_i, lambda_j] (Sec. 2.1: matrix functions through
A = V E V^{-1}).

The pole set (M and hence every z_k, w_k) is held fixed when H varies; the
spectral radius used to choose it depends on H.
"""
import numpy as np
import scipy.linalg

from . import lrsw


def sample(u, idx):
    """P u: eta values at flat indices idx."""
    return np.asarray(u[0]).ravel()[idx]


def sample_T(v, idx, shape):
    """P^T v: scatter into an eta field, zero velocities."""
    out = np.zeros(shape)
    eta = out[0].reshape(-1)          # a view: out is C-contiguous
    eta[idx] = v
    return out


def loss(u, idx, y):
    r = sample(u, idx) - y
    return float(r @ r)


def grad_u(u, idx, y):
    """dJ/du = 2 P^T (P u - y)."""
    return sample_T(2.0 * (sample(u, idx) - y), idx, u.shape)


def _eig_blocks(M):
    lam, V = np.linalg.eig(M)
    Vi = np.linalg.inv(V)
    return lam, V, Vi


def _apply_blocks(B, F):
    return np.einsum("yxab,byx->ayx", B, F)


def expm_T_apply(op, g, t):
    """exp(tA)^T g per mode with t A_hat^H (exact exponential)."""
    AhH = np.conj(np.swapaxes(lrsw.symbol(op), -1, -2))
    lam, V, Vi = _eig_blocks(t * AhH)
    B = V @ (np.exp(lam)[..., None] * Vi)
    return lrsw.from_modes(_apply_blocks(B, lrsw.to_modes(g))).real


def rexii_T_apply(op, g, t, z, w):
    """r(tA)^T g = Re sum_k w_k (tA^T - z_k)^{-1} g, per mode with A_hat^H
    (direct 3x3 solves, small sizes) -- the exact adjoint of the approximant."""
    AhH = np.conj(np.swapaxes(lrsw.symbol(op), -1, -2))
    G = lrsw.to_modes(g).transpose(1, 2, 0)[..., None]
    I3 = np.eye(3)[None, None]
    acc = np.zeros(G.shape, dtype=np.complex128)
    for zk, wk in zip(z, w):
        acc += wk * np.linalg.solve(t * AhH - zk * I3, G)
    return lrsw.from_modes(acc[..., 0].transpose(2, 0, 1)).real


def rexii_T_spectral(op, g, t, z, w):
    """Same as rexii_T_apply via the eigendecomposition of t A_hat^H:
    r(X) = V diag(sum_k w_k / (lambda - z_k)) V^{-1}."""
    AhH = np.conj(np.swapaxes(lrsw.symbol(op), -1, -2))
    lam, V, Vi = _eig_blocks(t * AhH)
    rl = np.zeros(lam.shape, dtype=np.complex128)
    for zk, wk in zip(z, w):
        rl += wk / (lam - zk)
    B = V @ (rl[..., None] * Vi)
    return lrsw.from_modes(_apply_blocks(B, lrsw.to_modes(g))).real


def _E_hat(op):
    SX, SY = lrsw.wavenumbers(op)
    E = np.zeros((op.ny, op.nx, 3, 3), dtype=np.complex128)
    E[..., 0, 1] = -1j * SX
    E[..., 0, 2] = -1j * SY
    return E


def frechet_exp_apply(op, f, t):
    """(d/dH) exp(tA) f = L_exp(tA, tE) f per mode via divided differences
    in the eigenbasis of t A_hat (eigenvalues 0, +-i omega t, distinct when
    omega > 0)."""
    X = t * lrsw.symbol(op)
    Y = t * _E_hat(op)
    lam, V, Vi = _eig_blocks(X)
    e = np.exp(lam)
    li = lam[..., :, None]
    lj = lam[..., None, :]
    diff = li - lj
    same = np.abs(diff) < 1e-12 * (1.0 + np.abs(li))
    Dl = np.where(same, e[..., :, None], (e[..., :, None] - e[..., None, :]) / np.where(same, 1.0, diff))
    B = V @ (Dl * (Vi @ Y @ V)) @ Vi
    return lrsw.from_modes(_apply_blocks(B, lrsw.to_modes(f))).real


def frechet_exp_block(op, f, t, modes):
    """Cross-check of frechet_exp_apply at selected modes: the top-right block of
    expm([[tA_hat, tE_hat], [0, tA_hat]]) (6x6 per mode).  Returns the per-mode
    vectors L F_hat at the listed (ky, kx) modes."""
    X = t * lrsw.symbol(op)
    Y = t * _E_hat(op)
    F = lrsw.to_modes(f)
    out = []
    for ky, kx in modes:
        Blk = np.zeros((6, 6), dtype=np.complex128)
        Blk[:3, :3] = X[ky, kx]
        Blk[:3, 3:] = Y[ky, kx]
        Blk[3:, 3:] = X[ky, kx]
        Lm = scipy.linalg.expm(Blk)[:3, 3:]
        out.append(Lm @ F[:, ky, kx])
    return np.array(out)


def frechet_rexii_apply(op, f, t, z, w):
    """(d/dH) r(tA) f = -Re sum_k w_k (tA - z_k)^{-1} tE (tA - z_k)^{-1} f
    per mode, as a divided-difference Frechet derivative of r in the
    eigenbasis: r[l_i, l_j] = -sum_k w_k / ((l_i - z_k)(l_j - z_k))."""
    X = t * lrsw.symbol(op)
    Y = t * _E_hat(op)
    lam, V, Vi = _eig_blocks(X)
    Dl = np.zeros(lam.shape + (3,), dtype=np.complex128)
    for zk, wk in zip(z, w):
        a = 1.0 / (lam - zk)
        Dl += -wk * a[..., :, None] * a[..., None, :]
    B = V @ (Dl * (Vi @ Y @ V)) @ Vi
    return lrsw.from_modes(_apply_blocks(B, lrsw.to_modes(f))).real


def grad_exact(op, f, t, idx, y):
    """(J, dJ/df, dJ/dH) for u = exp(tA) f (exact exponential)."""
    from .expm_modes import expm_closed_real
    u = expm_closed_real(op, f, t)
    gu = grad_u(u, idx, y)
    dJdf = expm_T_apply(op, gu, t)
    dJdH = float(np.sum(gu * frechet_exp_apply(op, f, t)))
    return loss(u, idx, y), dJdf, dJdH


def grad_rexii(op, f, t, z, w, idx, y):
    """(J, dJ/df, dJ/dH) for u = r(tA) f (the REXII approximant with a frozen
    pole set)."""
    from .rexii_modes import rexii_spectral
    u = rexii_spectral(op, f, t, z, w)
    gu = grad_u(u, idx, y)
    dJdf = rexii_T_spectral(op, gu, t, z, w)
    dJdH = float(np.sum(gu * frechet_rexii_apply(op, f, t, z, w)))
    return loss(u, idx, y), dJdf, dJdH
