"""Scalar REXII coefficients, the accuracy rule and the pole/weight form.

Test infrastructure only (see the oracle package docstring).  Plain FP64
NumPy, written from Sec. 2 and Appendices A and B of the paper.

Notation follows the paper: h (Gaussian width), M (truncation of the
Gaussian sum), L = 24, mu, a_l (Appendix A), b_m (eq. bm), n = m + l,
N = M + L, alpha_n = h (mu + i n), c_{1,n}, c_{2,n} (eq. modifiedRexi),
C_{1,n} = c_{1,n} h mu + c_{2,n} h n and C_{2,n} = i c_{2,n} (Sec. 2.2),
Gamma_0 = 1, Gamma_n = 2 (eq. modifiedRexiMatrixReducedSum).

The API's poles beta_k and weights alpha_k (u ~ Re sum_k alpha_k
(A - beta_k I)^{-1} f) are the partial fractions of the reduced sum:
term n has poles at tau A = alpha_{-n} and tau A = -alpha_n.  Because the
paper's alpha_n is a pole parameter while the API's alpha_k is a weight,
this module uses z_k (poles of tau A) and w_k (weights) internally.
"""
import math

import numpy as np

from .table_a import L, MU, a


# ----------------------------------------------------------------------------
# Step 1 (Sec. 2.1): e^{ix} as a sum of shifted Gaussians
# ----------------------------------------------------------------------------
def psi(x, h):
    """psi_h(x) = (4 pi)^{-1/2} exp(-x^2 / (4 h^2))  (eq. psi)."""
    x = np.asarray(x, dtype=np.float64)
    return np.exp(-x * x / (4.0 * h * h)) / math.sqrt(4.0 * math.pi)


def b_coef(m, h):
    """b_m = e^{-i m h} e^{h^2}  (eq. bm)."""
    m = np.asarray(m, dtype=np.float64)
    return np.exp(-1j * m * h) * math.exp(h * h)


def gaussian_sum(x, M, h):
    """sum_{m=-M}^{M} b_m psi_h(x + m h)  (eq. eixsumM), an approximation of
    e^{ix} for |x| <= (M - 11) h  (eq. Mformula)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.complex128)
    for m in range(-M, M + 1):
        out += b_coef(m, h) * psi(x + m * h, h)
    return out


# ----------------------------------------------------------------------------
# Step 2 (Sec. 2.1): the Gaussian psi_1 as a sum of rational functions
# ----------------------------------------------------------------------------
def R_complex(x):
    """R(x) = Re sum_{l=-L}^{L} a_l / (i x + mu + i l)  (eq. ratapproxgaush1)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.zeros(x.shape, dtype=np.complex128)
    for l in range(-L, L + 1):
        s += a(l) / (1j * x + MU + 1j * l)
    return s.real


def R_closed(x):
    """The real closed form of R (eq. A(x,mu)), valid when a_{-l} = conj(a_l)."""
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    out = a(0).real * MU / (x2 + MU * MU)
    for l in range(1, L + 1):
        al = a(l)
        num = (2.0 * MU * al.real * (MU * MU + l * l + x2)
               + 2.0 * l * al.imag * (MU * MU + l * l - x2))
        den = x2 * x2 + 2.0 * (MU * MU - l * l) * x2 + (MU * MU + l * l) ** 2
        out = out + num / den
    return out


# ----------------------------------------------------------------------------
# Step 3 (Sec. 2.1): REXII coefficients c_{1,n}, c_{2,n}
# ----------------------------------------------------------------------------
def c_coefs(M, h):
    """c_{1,n} and c_{2,n} for n = -N..N (eq. modifiedRexi definitions):
        c_{1,n} = h sum_{k=L1(n)}^{L2(n)} Re(a_k) b_{n-k}
        c_{2,n} = h sum_{k=L1(n)}^{L2(n)} Im(a_k) b_{n-k}
    with L1(n) = max(-L, n - M), L2(n) = min(L, n + M).
    Returns (n, c1, c2) arrays of length 2N+1."""
    N = M + L
    ns = np.arange(-N, N + 1)
    c1 = np.zeros(len(ns), dtype=np.complex128)
    c2 = np.zeros(len(ns), dtype=np.complex128)
    # The range L1(n) <= k <= L2(n) is exactly -L <= k <= L together with
    # |n - k| <= M (the index m = n - k of b_m stays within -M..M); the loop
    # runs over k and adds the k-th term to every n it belongs to.
    for k in range(-L, L + 1):
        inside = np.abs(ns - k) <= M
        bk = b_coef(ns[inside] - k, h)
        c1[inside] += a(k).real * bk
        c2[inside] += a(k).imag * bk
    return ns, h * c1, h * c2


def rexii_scalar(x, M, h):
    """REXII(ix) = sum_{n=-N}^{N} (c_{1,n} h mu + c_{2,n}(x + h n)) /
    ((alpha_{-n} - i x)(alpha_n + i x))  (eq. modifiedRexi)."""
    x = np.asarray(x, dtype=np.float64)
    ns, c1, c2 = c_coefs(M, h)
    out = np.zeros(x.shape, dtype=np.complex128)
    for n, a1, a2 in zip(ns, c1, c2):
        al_n = h * (MU + 1j * n)
        al_mn = h * (MU - 1j * n)
        out += (a1 * h * MU + a2 * (x + h * n)) / ((al_mn - 1j * x) * (al_n + 1j * x))
    return out


def rexi_scalar(x, M, h):
    """The original REXI(ix) (eq. originalRexi) with the symmetric Table A
    coefficients:  beta^Re_n = h sum a_k Re(b_{n-k}),
    beta^Im_n = h sum a_k Im(b_{n-k}),
    REXI(ix) = sum_n Re(beta^Re_n / (ix + alpha_n)) + i Re(beta^Im_n / (ix + alpha_n)).
    Comparison scheme; used only by the oracle tests."""
    x = np.asarray(x, dtype=np.float64)
    N = M + L
    ns = np.arange(-N, N + 1)
    bre = np.zeros(len(ns), dtype=np.complex128)
    bim = np.zeros(len(ns), dtype=np.complex128)
    for k in range(-L, L + 1):          # same index set as in c_coefs
        inside = np.abs(ns - k) <= M
        bk = b_coef(ns[inside] - k, h)
        bre[inside] += a(k) * bk.real
        bim[inside] += a(k) * bk.imag
    bre *= h
    bim *= h
    out = np.zeros(x.shape, dtype=np.complex128)
    for n, br, bi in zip(ns, bre, bim):
        al_n = h * (MU + 1j * n)
        out += (br / (1j * x + al_n)).real + 1j * (bi / (1j * x + al_n)).real
    return out


def rexi_poles_weights(M, h):
    """The original REXI matrix scheme (eq. originalREXImatrix),
    REXI(tau A) = sum_{n=-N}^{N} Re(beta^Re_n (tau A + alpha_n I)^{-1}),
    alpha_n = h (mu + i n), beta^Re_n = h sum_k a_k Re(b_{n-k}), written as
    Re sum_k w_k (tau A - z_k I)^{-1} with z = -alpha_n and w = beta^Re_n,
    n = -N..N (2N + 1 poles, N = M + L).  Comparison scheme."""
    N = M + L
    ns = np.arange(-N, N + 1)
    bre = np.zeros(len(ns), dtype=np.complex128)   # a_k is complex
    for k in range(-L, L + 1):
        inside = np.abs(ns - k) <= M
        bre[inside] += a(k) * b_coef(ns[inside] - k, h).real
    bre *= h
    z = -h * (MU + 1j * ns)
    return z, bre


# ----------------------------------------------------------------------------
# Accuracy rule (eqs. Mformula, matrixAccuracyBound; Appendix B)
# ----------------------------------------------------------------------------
def m0_of_tol(tol):
    """m_0 = c - 1 with c = 2 sqrt(-log(sqrt(4 pi) tol)) (Appendix B): psi_h(z)
    <= tol once |z| >= c h.  Rounded up to an integer, so the M rule stays an
    upper bound.  tol = 1e-16 gives 11 (the paper's value), 1e-10 gives 9,
    1e-6 gives 7."""
    c = 2.0 * math.sqrt(-math.log(math.sqrt(4.0 * math.pi) * tol))
    return int(math.ceil(c - 1.0))


def M_rule(t, rho, h, m0=11):
    """Smallest M with t rho <= (M - m0) h  (eq. matrixAccuracyBound)."""
    return int(math.ceil(t * rho / h)) + int(m0)


# ----------------------------------------------------------------------------
# Matrix form (Sec. 2.2) and the reduced sum over n >= 0
# ----------------------------------------------------------------------------
def C_coefs(M, h):
    """(n, C1, C2, Gamma) for n = 0..N with C_{1,n} = c_{1,n} h mu + c_{2,n} h n,
    C_{2,n} = i c_{2,n} (Sec. 2.2) and Gamma_0 = 1, Gamma_n = 2
    (eq. modifiedRexiMatrixReducedSum)."""
    ns, c1, c2 = c_coefs(M, h)
    keep = ns >= 0
    n = ns[keep]
    C1 = c1[keep] * h * MU + c2[keep] * h * n
    C2 = 1j * c2[keep]
    G = np.where(n == 0, 1.0, 2.0)
    return n, C1, C2, G


def poles_weights(M, h):
    """Partial-fraction form of the reduced sum.

    Term n of eq. modifiedRexiMatrixReducedSum is, as a rational function of
    X = tau A,  Gamma_n (C_{1,n} - C_{2,n} X) (alpha_{-n} - X)^{-1} (alpha_n + X)^{-1}.
    Its poles are z_{n,1} = alpha_{-n} and z_{n,2} = -alpha_n, which differ by
    2 h mu, so the term equals w_{n,1}/(X - z_{n,1}) + w_{n,2}/(X - z_{n,2})
    with residues
        w_{n,1} = -Gamma_n (C_{1,n} - C_{2,n} z_{n,1}) / (2 h mu)
        w_{n,2} = +Gamma_n (C_{1,n} - C_{2,n} z_{n,2}) / (2 h mu).
    Returns complex arrays z, w of length P = 2(N+1), ordered
    [z_{0,1}, z_{0,2}, z_{1,1}, z_{1,2}, ...].  Then
    exp(tau A) f ~ Re sum_k w_k (tau A - z_k I)^{-1} f."""
    n, C1, C2, G = C_coefs(M, h)
    z1 = h * (MU - 1j * n)
    z2 = -h * (MU + 1j * n)
    w1 = -G * (C1 - C2 * z1) / (2.0 * h * MU)
    w2 = G * (C1 - C2 * z2) / (2.0 * h * MU)
    z = np.empty(2 * len(n), dtype=np.complex128)
    w = np.empty(2 * len(n), dtype=np.complex128)
    z[0::2], z[1::2] = z1, z2
    w[0::2], w[1::2] = w1, w2
    return z, w


def kappa_sum(w, h):
    """Amplification of per-pole relative errors in the weighted sum:
    sum_k |w_k| / |h mu| (each resolvent has norm <= 1/|h mu| for a
    skew-symmetric A, because every pole is at distance |h mu| from the
    imaginary axis)."""
    return float(np.sum(np.abs(w)) / abs(h * MU))


def api_coeffs(t, rho, h=0.5, tol=1e-10, m0=None):
    """The coefficients exported at the API: poles beta_k = z_k / t and
    weights alpha_k = w_k / t, so exp(tA) f ~ Re sum_k alpha_k (A - beta_k I)^{-1} f.
    Returns dict(P, M, N, beta, alpha, z, w, kappa_sum, m0)."""
    if m0 is None:
        m0 = m0_of_tol(tol)
    M = M_rule(t, rho, h, m0)
    z, w = poles_weights(M, h)
    return dict(P=len(z), M=M, N=M + L, m0=m0, z=z, w=w, beta=z / t,
                alpha=w / t, kappa_sum=kappa_sum(w, h))


def nested_matrix_apply(tA, f, M, h):
    """The paper's per-term algorithm (Sec. 4): for n = 0..N solve
    (tau A + alpha_n I) g1 = f, (alpha_{-n} I - tau A) g2 = g1, then
    g3 = Gamma_n (C_{2,n} g1 + (C_{1,n} - C_{2,n} alpha_{-n}) g2) and return
    Re sum_n g3.  (The product C_{2,n}(C_{1,n}/C_{2,n} - alpha_{-n}) is formed
    without the division, since c_{2,n} can be ~1e-9.)  Dense, small only."""
    n, C1, C2, G = C_coefs(M, h)
    I = np.eye(tA.shape[0])
    acc = np.zeros(tA.shape[0], dtype=np.complex128)
    for nn, a1, a2, g in zip(n, C1, C2, G):
        al_n = h * (MU + 1j * nn)
        al_mn = h * (MU - 1j * nn)
        g1 = np.linalg.solve(tA + al_n * I, f)
        g2 = np.linalg.solve(al_mn * I - tA, g1)
        acc += g * (a2 * g1 + (a1 - a2 * al_mn) * g2)
    return acc.real
