"""The linear rotating shallow-water operator on a doubly periodic grid,
discretised with second-order centred differences.

Test infrastructure only (see the oracle package docstring).

The paper's operator (Sec. 4) acts on f = (eta, u, v) as
    A f = (-d_x u - d_y v,  -d_x eta + v,  -d_y eta - u)
with spectral derivatives and unit Coriolis parameter.  This module keeps the
same sign pattern, with gravity g, depth H (constant, or a field in flux
form) and Coriolis parameter f_c:
    A f = (-dx(H u) - dy(H v),  -g dx eta + f_c v,  -g dy eta - f_c u),
where dx phi[j][i] = (phi[j][i+1] - phi[j][i-1]) / (2 Dx), periodic, Dx = 1/nx
(and dy likewise, Dy = 1/ny).  Fields are stored f[c][j][i] with c in
(eta, u, v), j the y index, i the x index.

With W = diag(g, H, H) the product W A is skew-symmetric, so the spectrum of
A is imaginary (the property sigma(A) in iR the paper assumes, Sec. 1).
"""
import math
from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class LRSW:
    nx: int
    ny: int
    g: float = 1.0
    H: float = 1.0                       # constant depth (used if Hfield is None)
    fc: float = 10.0                     # Coriolis parameter
    Hfield: Optional[np.ndarray] = None  # variable depth [ny][nx], flux form

    @property
    def n(self):
        return 3 * self.nx * self.ny

    def depth(self):
        if self.Hfield is None:
            return np.full((self.ny, self.nx), float(self.H))
        return np.asarray(self.Hfield, dtype=np.float64)


def dx(phi, nx):
    """Centred difference in x (last axis), periodic, spacing 1/nx."""
    return (np.roll(phi, -1, axis=-1) - np.roll(phi, 1, axis=-1)) * (nx / 2.0)


def dy(phi, ny):
    """Centred difference in y (second-to-last axis), periodic, spacing 1/ny."""
    return (np.roll(phi, -1, axis=-2) - np.roll(phi, 1, axis=-2)) * (ny / 2.0)


def apply_A(op, f):
    """A f for f of shape [3][ny][nx] (flux form for variable depth)."""
    eta, u, v = f[0], f[1], f[2]
    Hd = op.depth()
    out = np.empty_like(f, dtype=np.float64)
    out[0] = -dx(Hd * u, op.nx) - dy(Hd * v, op.ny)
    out[1] = -op.g * dx(eta, op.nx) + op.fc * v
    out[2] = -op.g * dy(eta, op.ny) - op.fc * u
    return out


def dense_A(op):
    """Dense matrix of A, assembled column by column from apply_A on unit
    vectors (no Fourier analysis involved).  Small grids only."""
    n = op.n
    A = np.zeros((n, n))
    e = np.zeros(n)
    for c in range(n):
        e[c] = 1.0
        A[:, c] = apply_A(op, e.reshape(3, op.ny, op.nx)).ravel()
        e[c] = 0.0
    return A


# ----------------------------------------------------------------------------
# Fourier symbol (constant depth)
# ----------------------------------------------------------------------------
def wavenumbers(op):
    """s_x[i] = nx sin(2 pi i / nx) on the x axis and s_y likewise: dx acting on
    exp(2 pi i (kx x + ky y)) multiplies it by i s_x."""
    kx = np.arange(op.nx)
    ky = np.arange(op.ny)
    sx = op.nx * np.sin(2.0 * np.pi * kx / op.nx)
    sy = op.ny * np.sin(2.0 * np.pi * ky / op.ny)
    return sx[None, :] * np.ones((op.ny, 1)), sy[:, None] * np.ones((1, op.nx))


def symbol(op):
    """A_hat[ky][kx] (3x3 complex per mode) for constant depth:
    [[0, -i H s_x, -i H s_y], [-i g s_x, 0, f_c], [-i g s_y, -f_c, 0]]."""
    if op.Hfield is not None:
        raise ValueError("the Fourier symbol needs constant depth")
    SX, SY = wavenumbers(op)
    Ah = np.zeros((op.ny, op.nx, 3, 3), dtype=np.complex128)
    Ah[..., 0, 1] = -1j * op.H * SX
    Ah[..., 0, 2] = -1j * op.H * SY
    Ah[..., 1, 0] = -1j * op.g * SX
    Ah[..., 2, 0] = -1j * op.g * SY
    Ah[..., 1, 2] = op.fc
    Ah[..., 2, 1] = -op.fc
    return Ah


def s2_axis(n):
    """s(k)^2 = (n sin(2 pi k / n))^2 for k = 0..n-1, evaluated at a canonical
    representative of k (sin^2 has period n/2 for even n and is symmetric
    about n/4; for odd n it is symmetric about n/2), so that modes with the
    same frequency get bit-identical values."""
    k = np.arange(n)
    if n % 2 == 0:
        kc = k % (n // 2)
        kc = np.minimum(kc, n // 2 - kc)
    else:
        kc = np.minimum(k, n - k)
    return (n * np.sin(2.0 * np.pi * kc / n)) ** 2


def omega(op):
    """Per-mode frequency omega = sqrt(f_c^2 + g H (s_x^2 + s_y^2)); the
    eigenvalues of A_hat are 0 and +-i omega (characteristic polynomial
    lambda^3 + omega^2 lambda)."""
    sx2 = s2_axis(op.nx)[None, :]
    sy2 = s2_axis(op.ny)[:, None]
    return np.sqrt(op.fc ** 2 + op.g * op.H * (sx2 + sy2))


def rho(op):
    """Spectral radius of A (eq. matrixAccuracyBound needs an upper bound).

    Constant depth: the exact discrete maximum of omega over all modes.
    Variable depth: the guaranteed bound sqrt(g max H) * sqrt(nx^2 + ny^2) + |f_c|
    (W^{1/2} A W^{-1/2} is skew; its gravity part has norm
    <= sqrt(g max H) |grad| with |grad|^2 <= nx^2 + ny^2, its Coriolis part
    has norm |f_c|)."""
    if op.Hfield is None:
        return float(omega(op).max())
    Hmax = float(np.max(op.Hfield))
    return math.sqrt(op.g * Hmax) * math.sqrt(op.nx ** 2 + op.ny ** 2) + abs(op.fc)


def to_modes(f):
    """FFT of each of the three fields: F[c][ky][kx]."""
    return np.fft.fft2(np.asarray(f, dtype=np.float64), axes=(-2, -1))


def from_modes(F):
    """Inverse FFT of each field (complex result; callers take Re)."""
    return np.fft.ifft2(F, axes=(-2, -1))


def modes_matvec(Ah, F):
    """(A_hat F) per mode, for F[c][ky][kx] and Ah[ky][kx][3][3]."""
    return np.einsum("yxab,byx->ayx", Ah, F)
