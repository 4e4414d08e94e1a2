"""References for the variable-depth (flux form) operator, which the FFT does
not diagonalise.

Test infrastructure only (see the oracle package docstring).

* ``expm_dense`` (in expm_modes) on small grids.
* ``chebyshev_expm``: the Chebyshev series of the exponential (Tal-Ezer and
  Kosloff, 1984).  With the spectrum of A inside i[-rho, rho] and
  X = A / (i rho) (spectrum in [-1, 1]),
      exp(tA) = J_0(t rho) I + 2 sum_{k>=1} i^k J_k(t rho) T_k(X).
  Writing Q_k = i^k T_k(X) f, the Chebyshev recurrence becomes the real
  recurrence Q_0 = f, Q_1 = (A/rho) f, Q_{k+1} = 2 (A/rho) Q_k + Q_{k-1}.
  It is a polynomial method, independent of the rational approximation and
  of any linear solve.  Parity unpinned beyond its agreement with the dense
  exponential on small grids (checked in tests).
* ``rexii_dense``/``resolvent_dense``: dense shifted solves (small grids).
"""
import math

import numpy as np
import scipy.special

from . import lrsw


def chebyshev_expm(op, f, t, rho=None, tol=1e-17):
    """exp(tA) f by the Chebyshev-Bessel series; rho must bound the spectral
    radius of A (defaults to the guaranteed bound lrsw.rho)."""
    rho = lrsw.rho(op) if rho is None else float(rho)
    x = t * rho
    kmax = int(x + 20.0 * max(1.0, x) ** (1.0 / 3.0) + 60)
    J = scipy.special.jv(np.arange(kmax + 1), x)
    q_prev = np.asarray(f, dtype=np.float64).copy()
    q = lrsw.apply_A(op, q_prev) / rho
    u = J[0] * q_prev + 2.0 * J[1] * q
    small = 0
    for k in range(1, kmax):
        q_next = 2.0 * lrsw.apply_A(op, q) / rho + q_prev
        q_prev, q = q, q_next
        u += 2.0 * J[k + 1] * q
        if k > x and abs(J[k + 1]) < tol:
            small += 1
            if small >= 4:
                break
        else:
            small = 0
    return u


def resolvent_dense(op, f, t, z):
    """(tA - z I)^{-1} f by a dense solve (small grids, any depth)."""
    A = lrsw.dense_A(op)
    x = np.linalg.solve(t * A - z * np.eye(A.shape[0]), np.asarray(f).ravel().astype(complex))
    return x.reshape(3, op.ny, op.nx)


def w_energy(op, f):
    """||f||_W^2 with W = diag(g, H, H): conserved by exp(tA) for any depth."""
    Hd = op.depth()
    return float(op.g * np.sum(f[0] ** 2) + np.sum(Hd * (f[1] ** 2 + f[2] ** 2)))
