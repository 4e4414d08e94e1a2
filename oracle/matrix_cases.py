"""The paper's matrix test cases (Sec. 3.2) and the comparison schemes applied
to matrices: REXII (eq. modifiedRexiMatrixReducedSum), the original REXI
(eq. originalREXImatrix) and REXIE (eq. REXIE), all by dense solves.

Test infrastructure only (see the oracle package docstring).  Plain FP64
NumPy/SciPy.

Test matrices (Sec. 3.2):
  A_1  second-order centred difference of d/dx, periodic on [0, 1] with step
       1/70 (70 unknowns: the end point of the closed grid is the first
       point again); real skew-symmetric, eigenvalues in i[-70, 70], complex
       eigenvectors.
  A_2  i times the second-order difference of d^2/dx^2, periodic on [-1, 1]
       with step 1/35 (70 unknowns); purely imaginary and Hermitian times i
       (skew-Hermitian), eigenvalues in i[-4900, 0], real eigenvectors; the
       paper shifts it by nu = -2450 i.
  f_0  (2 + cos(2 pi x))^{-1} at the grid points.

A circulant matrix is given here by its stencil: (A f)_j = sum_d c_d f_{j+d}
(indices mod n), d = -s..s.
"""
import numpy as np
import scipy.linalg

from .coeffs import L, MU, b_coef, poles_weights, rexi_poles_weights
from .table_a import a


# ----------------------------------------------------------------------------
# circulant matrices
# ----------------------------------------------------------------------------
def circulant_dense(n, stencil):
    """Dense n x n matrix of (A f)_j = sum_d c_d f_{(j+d) mod n}; stencil is a
    dict {d: c_d}."""
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        for d, c in stencil.items():
            A[j, (j + d) % n] += c
    return A


def circulant_symbol(n, stencil):
    """Eigenvalue of the circulant matrix on the Fourier mode e^{2 pi i j k / n}:
    lambda(k) = sum_d c_d e^{2 pi i d k / n}, k = 0..n-1 (numpy FFT order)."""
    k = np.arange(n)
    lam = np.zeros(n, dtype=np.complex128)
    for d, c in stencil.items():
        lam += c * np.exp(2j * np.pi * d * k / n)
    return lam


def stencil_A1(n=70):
    """d/dx by centred differences, periodic on [0, 1], step 1/n."""
    return {1: 0.5 * n, -1: -0.5 * n}


def stencil_A2(n=70, length=2.0):
    """i d^2/dx^2 by second differences, periodic on an interval of the given
    length, step length / n."""
    dx = length / n
    c = 1.0 / (dx * dx)
    return {-1: 1j * c, 0: -2j * c, 1: 1j * c}


def grid_A1(n=70):
    return np.arange(n) / n


def grid_A2(n=70):
    return -1.0 + 2.0 * np.arange(n) / n


def f0(x):
    """The paper's vector f_0 = (2 + cos(2 pi x))^{-1} (Sec. 3.2)."""
    return 1.0 / (2.0 + np.cos(2.0 * np.pi * x))


# ----------------------------------------------------------------------------
# reference exponentials
# ----------------------------------------------------------------------------
def expm_dense(A, f, t=1.0):
    """exp(tA) f by scipy's dense matrix exponential (Pade)."""
    return scipy.linalg.expm(t * A) @ f


def expm_circulant(n, stencil, f, t=1.0):
    """exp(tA) f for a circulant A through its eigen-decomposition: the DFT
    diagonalises every circulant matrix, with eigenvalues circulant_symbol."""
    lam = circulant_symbol(n, stencil)
    return np.fft.ifft(np.exp(t * lam) * np.fft.fft(f))


# ----------------------------------------------------------------------------
# the three schemes applied to a dense matrix (one dense solve per pole)
# ----------------------------------------------------------------------------
def rexii_dense(A, f, M, h, t=1.0):
    """REXII for real A and real f: Re sum_k w_k (tA - z_k I)^{-1} f with the
    partial fractions of the reduced sum (eq. modifiedRexiMatrixReducedSum)."""
    z, w = poles_weights(M, h)
    tA = t * A
    I = np.eye(A.shape[0])
    acc = np.zeros(A.shape[0], dtype=np.complex128)
    for zk, wk in zip(z, w):
        acc += wk * np.linalg.solve(tA - zk * I, f)
    return acc.real


def rexi_dense(A, f, M, h, t=1.0):
    """The original REXI for real A and real f (eq. originalREXImatrix):
    sum_{n=-N}^{N} Re(beta^Re_n (tA + alpha_n I)^{-1} f), alpha_n = h(mu + i n)."""
    z, w = rexi_poles_weights(M, h)
    tA = t * A
    I = np.eye(A.shape[0])
    acc = np.zeros(A.shape[0], dtype=np.complex128)
    for zk, wk in zip(z, w):
        acc += wk * np.linalg.solve(tA - zk * I, f)
    return acc.real


def rexi_betas(M, h):
    """(n, alpha_n, beta^Re_n, beta^Im_n) for n = -N..N: beta^Re_n =
    h sum_k a_k Re(b_{n-k}) and beta^Im_n = h sum_k a_k Im(b_{n-k}) over
    k = -L..L with |n - k| <= M (eq. originalRexi with the Table A
    coefficients)."""
    N = M + L
    ns = np.arange(-N, N + 1)
    bre = np.zeros(len(ns), dtype=np.complex128)
    bim = np.zeros(len(ns), dtype=np.complex128)
    for k in range(-L, L + 1):
        inside = np.abs(ns - k) <= M
        bk = b_coef(ns[inside] - k, h)
        bre[inside] += a(k) * bk.real
        bim[inside] += a(k) * bk.imag
    return ns, h * (MU + 1j * ns), h * bre, h * bim


def rexie_dense(A, f, M, h, t=1.0, nu=0.0):
    """REXIE (eq. REXIE) for A - nu I = i B with B real diagonalisable (real
    eigenvectors) and real f:
        exp(tA) f = e^{t nu} exp(t(A - nu I)) f,
        exp(tA') f ~ sum_n Re(beta^Re_n (tA' + alpha_n I)^{-1} f)
                     + i Re(beta^Im_n (tA' + alpha_n I)^{-1} f).
    One dense solve per n; the shift nu follows the remark on shifted
    matrices in Sec. 2.2."""
    _, al, bre, bim = rexi_betas(M, h)
    tA = t * (A - nu * np.eye(A.shape[0]))
    I = np.eye(A.shape[0])
    re = np.zeros(A.shape[0])
    im = np.zeros(A.shape[0])
    for a_n, br, bi in zip(al, bre, bim):
        y = np.linalg.solve(tA + a_n * I, f)
        re += (br * y).real
        im += (bi * y).real
    return np.exp(t * nu) * (re + 1j * im)


# ----------------------------------------------------------------------------
# the same schemes per Fourier mode of a circulant matrix (exact up to
# rounding: the DFT diagonalises the matrix, so each resolvent is a scalar
# division per mode)
# ----------------------------------------------------------------------------
def _real_part_in_space(g, fh):
    """Fourier coefficients of Re(ifft(g * fh)) for real data f (fh its DFT):
    (g(k) fh(k) + conj(g(-k) fh(-k))) / 2."""
    gm = np.roll(g[::-1], 1)           # g(-k)
    fm = np.roll(fh[::-1], 1)
    return 0.5 * (g * fh + np.conj(gm * fm))


def rexii_circulant(n, stencil, f, M, h, t=1.0):
    """REXII for a real circulant A and real f, per Fourier mode."""
    z, w = poles_weights(M, h)
    lam = t * circulant_symbol(n, stencil)
    g = np.zeros(n, dtype=np.complex128)
    for zk, wk in zip(z, w):
        g += wk / (lam - zk)
    return np.fft.ifft(_real_part_in_space(g, np.fft.fft(f))).real


def rexi_circulant(n, stencil, f, M, h, t=1.0):
    """The original REXI for a real circulant A and real f, per Fourier mode."""
    z, w = rexi_poles_weights(M, h)
    lam = t * circulant_symbol(n, stencil)
    g = np.zeros(n, dtype=np.complex128)
    for zk, wk in zip(z, w):
        g += wk / (lam - zk)
    return np.fft.ifft(_real_part_in_space(g, np.fft.fft(f))).real


def rexie_circulant(n, stencil, f, M, h, t=1.0, nu=0.0):
    """REXIE for a circulant A with A - nu I = i B (B real) and real f, per
    Fourier mode: the real parts are taken in physical space."""
    _, al, bre, bim = rexi_betas(M, h)
    lam = t * (circulant_symbol(n, stencil) - nu)
    gre = np.zeros(n, dtype=np.complex128)
    gim = np.zeros(n, dtype=np.complex128)
    for a_n, br, bi in zip(al, bre, bim):
        gre += br / (lam + a_n)
        gim += bi / (lam + a_n)
    fh = np.fft.fft(f)
    re = np.fft.ifft(_real_part_in_space(gre, fh)).real
    im = np.fft.ifft(_real_part_in_space(gim, fh)).real
    return np.exp(t * nu) * (re + 1j * im)


def rel_l2(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
