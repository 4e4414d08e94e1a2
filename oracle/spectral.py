"""The paper's own LRSW test problem (Sec. 4): spectral derivatives, unit
Coriolis parameter, g = H = 1, on a D x D grid of the unit square, with the
three initial conditions of the paper (wave scenarios 1 and 2, eqs.
WAVESCENARIO1 / WAVESCENARIO2, and the Gaussian scenario, eq.
GAUSSIANSCENARIO).  Used only to check the oracle's coefficients and
per-mode REXII against the errors and term counts the paper prints.

Test infrastructure only (see the oracle package docstring).
"""
import math

import numpy as np

from . import lrsw
from .rexii_modes import rexii_symbol


def symbol(D):
    """A_hat = [[0, -i kx, -i ky], [-i kx, 0, 1], [-i ky, -1, 0]] with
    kx = 2 pi * (signed integer wavenumber), and omega = sqrt(1 + kx^2 + ky^2)."""
    k = 2.0 * np.pi * np.fft.fftfreq(D, 1.0 / D)
    KX = np.broadcast_to(k[None, :], (D, D))
    KY = np.broadcast_to(k[:, None], (D, D))
    Ah = np.zeros((D, D, 3, 3), dtype=np.complex128)
    Ah[..., 0, 1] = -1j * KX
    Ah[..., 0, 2] = -1j * KY
    Ah[..., 1, 0] = -1j * KX
    Ah[..., 2, 0] = -1j * KY
    Ah[..., 1, 2] = 1.0
    Ah[..., 2, 1] = -1.0
    om = np.sqrt(1.0 + KX ** 2 + KY ** 2)
    return Ah, om


def rho_spectral(D):
    """rho(A) = sqrt(2 pi^2 D^2 + 1)  (eq. lswRoh)."""
    return math.sqrt(2.0 * math.pi ** 2 * D * D + 1.0)


def scenario(name, D=128):
    x = np.arange(D) / D
    X = x[None, :]
    Y = x[:, None]
    pi = np.pi
    f = np.zeros((3, D, D))
    if name == "wave1":
        f[0] = np.sin(4 * pi * X) * np.cos(2 * pi * Y) - 0.2 * np.cos(4 * pi * X) * np.sin(4 * pi * Y)
        f[1] = np.cos(8 * pi * X) * np.cos(2 * pi * Y)
        f[2] = np.cos(4 * pi * X) * np.cos(4 * pi * Y)
    elif name == "wave2":
        f[0] = np.sin(32 * pi * X) * np.cos(16 * pi * Y) - 0.2 * np.cos(32 * pi * X) * np.sin(32 * pi * Y)
        f[1] = np.cos(64 * pi * X) * np.cos(16 * pi * Y)
        f[2] = np.cos(32 * pi * X) * np.cos(32 * pi * Y)
    elif name == "gaussian":
        f[0] = np.exp(-100.0 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))
        f[1] = 0.1 * np.sin(64 * pi * X) * np.sin(16 * pi * Y)
        f[2] = 0.1 * np.sin(32 * pi * X) * np.sin(32 * pi * Y)
    else:
        raise ValueError(name)
    return f


def exact(f, tau):
    """exp(tau A) f by the per-mode Cayley-Hamilton closed form."""
    D = f.shape[-1]
    Ah, om = symbol(D)
    F = lrsw.to_modes(f)
    AF = lrsw.modes_matvec(Ah, F)
    AAF = lrsw.modes_matvec(Ah, AF)
    s1 = tau * np.sinc(om * tau / np.pi)
    s2 = 0.5 * tau * tau * np.sinc(om * tau / (2.0 * np.pi)) ** 2
    return lrsw.from_modes(F + s1[None] * AF + s2[None] * AAF).real


def rexii(f, tau, z, w):
    """Re sum_k w_k (tau A - z_k)^{-1} f per mode."""
    D = f.shape[-1]
    Ah, om = symbol(D)
    return lrsw.from_modes(rexii_symbol(Ah, om, lrsw.to_modes(f), tau, z, w)).real


def max_err(a, b):
    """The paper's error measure: max over grid points (and fields) of |a - b|."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
