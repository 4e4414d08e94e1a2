"""A refit of the coefficients a_l of the rational approximation of the unit
Gaussian (Sec. 2.1, step 2): the symmetric form R(x) of eq. A(x,mu), least
squares on points chosen one at a time like Leja points (eq. minl2approx).

Test infrastructure only (see the oracle package docstring).  Plain FP64
NumPy, with the least-squares residual of one refinement step taken in
extended precision (np.longdouble).

The paper fixes the form and the method but not the number of points K, the
interval, or how mu is chosen ("such that a high accuracy is obtained").
Readings used here:
  * mu is the printed value (Appendix A); L = 24.
  * Both psi_1 and R are even, so points are taken on [0, x_max] with
    x_max = 60 (the interval on which the printed table is checked); the
    candidates are n_candidates equally spaced values there.
  * Leja order: x_1 = 0, then x_{k+1} is the candidate with the largest
    product of distances to x_1..x_k; K = 200.  Mirror-image candidates tie
    exactly; values within 1e-12 (relative, of the log-product) of the
    largest count as ties, and ties go to the smallest x.
  * The least-squares problem G y = psi_1(x) is solved by an orthogonal
    factorisation (numpy's lstsq), then refined once: r = b - G y in
    extended precision, y += lstsq(G, r).  G is ill-conditioned (~1e12), so
    the refinement is what brings the fit to the printed table's accuracy.
"""
import math

import numpy as np

from .table_a import L as L_PRINTED
from .table_a import MU as MU_PRINTED


def psi1(x):
    """psi_1(x) = (4 pi)^{-1/2} exp(-x^2 / 4)  (eq. psi with h = 1)."""
    x = np.asarray(x, dtype=np.float64)
    return np.exp(-x * x / 4.0) / math.sqrt(4.0 * math.pi)


def design_matrix(x, mu=MU_PRINTED, L=L_PRINTED):
    """Rows G(x_k, mu, L) of eq. A(x,mu): R(x) = G(x) y with
    y = [a_0, Re a_1..Re a_L, Im a_1..Im a_L]."""
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    cols = [mu / (x2 + mu * mu)]
    dens = [x2 * x2 + 2.0 * (mu * mu - l * l) * x2 + (mu * mu + l * l) ** 2 for l in range(1, L + 1)]
    for l in range(1, L + 1):
        cols.append(2.0 * mu * (mu * mu + l * l + x2) / dens[l - 1])
    for l in range(1, L + 1):
        cols.append(2.0 * l * (mu * mu + l * l - x2) / dens[l - 1])
    return np.stack(cols, axis=-1)


def leja_points(candidates, K):
    """x_1 = 0 (must be a candidate), then greedily the candidate maximising
    the product of distances to the points chosen so far (as a sum of logs)."""
    c = np.asarray(candidates, dtype=np.float64)
    j0 = int(np.argmin(np.abs(c)))
    pts = [c[j0]]
    logp = np.full(c.shape, 0.0)
    for k in range(1, K):
        with np.errstate(divide="ignore"):
            logp += np.log(np.abs(c - pts[-1]))
        m = np.max(logp)
        # the grid is symmetric, so the product has exact ties (mirror
        # images); those within 1e-12 of the largest go to the smallest x
        j = int(np.argmax(logp >= m - 1e-12 * max(1.0, abs(m))))
        pts.append(c[j])
    return np.array(pts)


def refit(K=200, x_max=60.0, n_candidates=200001, mu=MU_PRINTED, L=L_PRINTED):
    """(a, points): a[l] for l = 0..L (complex, a_{-l} = conj(a_l)) and the
    chosen points."""
    cand = x_max * np.arange(n_candidates, dtype=np.float64) / (n_candidates - 1)
    pts = leja_points(cand, K)
    G = design_matrix(pts, mu, L)
    b = psi1(pts)
    y, *_ = np.linalg.lstsq(G, b, rcond=None)
    r = (b.astype(np.longdouble) - G.astype(np.longdouble) @ y.astype(np.longdouble)).astype(np.float64)
    dy, *_ = np.linalg.lstsq(G, r, rcond=None)
    y = y + dy
    a = np.zeros(L + 1, dtype=np.complex128)
    a[0] = y[0]
    a[1:] = y[1:L + 1] + 1j * y[L + 1:]
    return a, pts


def R_of(a, x, mu=MU_PRINTED):
    """R(x) of eq. A(x,mu) for coefficients a[0..L]."""
    L = len(a) - 1
    y = np.concatenate([[a[0].real], a[1:].real, a[1:].imag])
    return design_matrix(x, mu, L) @ y
