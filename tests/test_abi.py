"""The C-ABI library loads, exports every symbol its header declares, and its
host-only logic (coefficients, argument checks) is right.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import coeffs as oc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rx():
    from paper_2008_11607_amd import rexii
    if not os.path.exists(rexii.LIB_PATH):
        from paper_2008_11607_amd import build
        build.build()
    rexii.load()
    return rexii


def _declared_symbols():
    out = set()
    for name in os.listdir(os.path.join(ROOT, "include")):
        if name.endswith(".h"):
            text = open(os.path.join(ROOT, "include", name)).read()
            out |= set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(rexii_\w+)\s*\(", text, flags=re.M))
    return out


def test_exports_every_declared_symbol(rx):
    syms = _declared_symbols()
    assert {"rexii_apply", "rexii_apply_adjoint", "rexii_coeffs"} <= syms
    lib = rx.load()
    for s in syms:
        assert hasattr(lib, s), s
    assert set(rx.EXPORTS) == syms


@pytest.mark.parametrize("trho,h,tol", [(100.0, 0.5, 1e-10), (1000.0, 0.5, 1e-6), (37.5, 1.0, 1e-10),
                                        (500.0, 0.3, 1e-12)])
def test_coeffs_match_oracle(rx, trho, h, tol):
    rho = 91.06041950265768
    t = trho / rho
    beta, alpha, kap = rx.coeffs(t, rho, h=h, tol=tol)
    ref = oc.api_coeffs(t, rho, h=h, tol=tol)
    assert len(beta) == ref["P"]
    assert np.max(np.abs(beta - ref["beta"])) <= 1e-14 * np.max(np.abs(ref["beta"]))
    assert np.max(np.abs(alpha - ref["alpha"])) <= 1e-13 * np.max(np.abs(ref["alpha"]))
    assert abs(kap - ref["kappa_sum"]) <= 1e-12 * ref["kappa_sum"]


@pytest.mark.parametrize("M,h", [(150, 0.2), (40, 0.5)])
def test_coeffs_rexi_match_oracle(rx, M, h):
    # rho chosen so that the M rule gives M exactly (m0 = 0, t = 1)
    beta, alpha = rx.coeffs_rexi(1.0, M * h, h=h, m0=0)
    z, w = oc.rexi_poles_weights(M, h)
    assert len(beta) == len(z)
    # same pole set (ordered 0, 1, -1, 2, -2, ... here, -N..N in the oracle)
    ob = np.argsort(beta.imag, kind="stable")
    oz = np.argsort(z.imag, kind="stable")
    assert np.max(np.abs(beta[ob] - z[oz])) <= 1e-14 * np.max(np.abs(z))
    assert np.max(np.abs(alpha[ob] - w[oz])) <= 1e-13 * np.max(np.abs(w))


def test_coeffs_explicit_m0(rx):
    beta, _, _ = rx.coeffs(1.0, 30.0, h=0.5, m0=11)
    # M = ceil(30/0.5) + 11 = 71, N = 95, P = 192
    assert len(beta) == 2 * (71 + 24 + 1)


def test_coeffs_query_only(rx):
    lib = rx.load()
    P = ctypes.c_int32(-1)
    assert lib.rexii_coeffs(1.0, 10.0, 0.5, 1e-10, -1, ctypes.byref(P), None, None, None) == 0
    assert P.value == 2 * (20 + 9 + 24 + 1)


@pytest.mark.parametrize("args", [(0.0, 10.0, 0.5, 1e-10), (1.0, -1.0, 0.5, 1e-10), (1.0, 10.0, 4.0, 1e-10),
                                  (1.0, 10.0, 0.5, 2.0), (float("nan"), 10.0, 0.5, 1e-10)])
def test_coeffs_invalid(rx, args):
    lib = rx.load()
    P = ctypes.c_int32()
    st = lib.rexii_coeffs(*args, -1, ctypes.byref(P), None, None, None)
    assert st == -1
    assert "rexii_coeffs" in rx.last_error()


def test_apply_rejects_bad_arguments_before_touching_the_device(rx):
    lib = rx.load()
    dummy = ctypes.c_void_p(16)       # never dereferenced: validation fails first
    rep = rx.Report()
    o = rx.make_opts()
    for nx, ny, g, H in [(2, 8, 1.0, 1.0), (8, 3, 1.0, 1.0), (8, 8, 0.0, 1.0), (8, 8, 1.0, -1.0)]:
        op = rx.make_op(nx, ny, g=g, H=H)
        st = lib.rexii_apply(ctypes.byref(op), dummy, ctypes.c_void_p(1 << 20), 1.0, ctypes.byref(o),
                             None, 0, None, ctypes.byref(rep))
        assert st == -1, (nx, ny, g, H)
    op = rx.make_op(8, 8)
    assert lib.rexii_apply(None, dummy, dummy, 1.0, None, None, 0, None, None) == -1
    assert lib.rexii_apply(ctypes.byref(op), None, dummy, 1.0, None, None, 0, None, None) == -1
    assert lib.rexii_apply(ctypes.byref(op), dummy, ctypes.c_void_p(1 << 20), -1.0, None, None, 0, None, None) == -1


def test_apply_fourier_rejects_bad_arguments_before_touching_the_device(rx):
    lib = rx.load()
    dummy = ctypes.c_void_p(16)       # never dereferenced: validation fails first
    far = ctypes.c_void_p(1 << 20)
    op = rx.make_op(8, 8)
    for deriv in (-1, 2):
        assert lib.rexii_apply_fourier(ctypes.byref(op), dummy, far, 1.0, deriv, None, None, 0, None, None) == -1
    assert "derivative" in rx.last_error()
    opv = rx.make_op(8, 8)
    opv.H_field = dummy               # a depth field is not supported by the Fourier path
    assert lib.rexii_apply_fourier(ctypes.byref(opv), dummy, far, 1.0, 0, None, None, 0, None, None) == -1
    assert lib.rexii_apply_fourier(ctypes.byref(op), dummy, dummy, 1.0, 0, None, None, 0, None, None) == -1
    assert lib.rexii_apply_fourier(ctypes.byref(op), None, far, 1.0, 0, None, None, 0, None, None) == -1
    assert lib.rexii_apply_fourier(ctypes.byref(op), dummy, far, -1.0, 0, None, None, 0, None, None) == -1
    nb = ctypes.c_size_t(7)
    assert lib.rexii_fourier_workspace_size(ctypes.byref(op), None, 0.0, 0, ctypes.byref(nb)) == 0
    assert nb.value == 0
    assert lib.rexii_fourier_workspace_size(ctypes.byref(op), None, 1.0, 5, ctypes.byref(nb)) == -1


def test_apply_multishift_rejects_bad_arguments_before_touching_the_device(rx):
    lib = rx.load()
    dummy = ctypes.c_void_p(16)       # never dereferenced: validation fails first
    far = ctypes.c_void_p(1 << 30)
    op = rx.make_op(8, 8)
    for nrhs in (0, -1, 70000):
        assert lib.rexii_apply_multishift(ctypes.byref(op), nrhs, dummy, far, 1.0, None, None, 0, None, None) == -1
    assert lib.rexii_apply_multishift(ctypes.byref(op), 2, dummy, ctypes.c_void_p(16 + 8 * 192), 1.0, None, None, 0,
                                      None, None) == -1   # u overlaps the second state of f
    assert lib.rexii_apply_multishift(ctypes.byref(op), 1, None, far, 1.0, None, None, 0, None, None) == -1
    assert lib.rexii_apply_multishift(ctypes.byref(op), 1, dummy, far, float("inf"), None, None, 0, None, None) == -1
    nb = ctypes.c_size_t(0)
    assert lib.rexii_multishift_workspace_size(ctypes.byref(op), 2, None, ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 2 * 3 * 64 * 8
    assert lib.rexii_multishift_workspace_size(ctypes.byref(op), 0, None, ctypes.byref(nb)) == -1


def test_default_opts(rx):
    o = rx.make_opts()
    assert o.h == 0.5 and o.m0 == -1 and o.pair_conjugate == 1 and o.precision == 0


def test_apply_circulant_rejects_bad_arguments_before_touching_the_device(rx):
    # the schemes' premises (Sec. 2.2 and the remark on REXIE) are checked on
    # the host: REXII / REXI need a real skew-symmetric circulant matrix,
    # REXIE needs A - nu I = i B with B real symmetric
    from oracle import matrix_cases as mc
    lib = rx.load()
    dummy = ctypes.c_void_p(16)       # never dereferenced: validation fails first
    far = ctypes.c_void_p(1 << 30)
    rep = rx.Report()

    def call(n, stencil, scheme, nu=0.0, nrhs=1, f=dummy, u=far, t=1.0):
        off, cc = rx._stencil_arrays(stencil)
        return lib.rexii_apply_circulant(n, len(off), off.ctypes.data_as(ctypes.c_void_p),
                                         cc.ctypes.data_as(ctypes.c_void_p), nrhs, f, u, t, nu, scheme, 0, None,
                                         None, 0, None, ctypes.byref(rep))

    A1, A2 = mc.stencil_A1(70), mc.stencil_A2(70)
    assert call(70, A1, 2) == -1                   # A_1 = i B with B Hermitian, not real: no REXIE
    assert "REXIE" in rx.last_error()
    assert call(70, A2, 0) == -1 and call(70, A2, 1) == -1   # A_2 is not real
    assert call(70, A1, 0, nu=-2450.0) == -1       # the shift is a REXIE option
    assert call(70, {1: 1.0, -1: -0.5}, 0) == -1   # not skew-symmetric
    assert call(70, {1: 1j, -1: 2j}, 2) == -1      # i B with B not symmetric
    assert call(70, {0: 1.0 + 1j}, 2) == -1        # real part on the diagonal
    assert call(1, A1, 0) == -1                    # n >= 2
    assert call(70, A1, 0, nrhs=0) == -1
    assert call(70, A1, 3) == -1                   # unknown scheme
    assert call(70, A1, 0, f=None) == -1
    assert call(70, A1, 0, t=-1.0) == -1
    assert call(70, A1, 0, u=ctypes.c_void_p(16 + 8 * 35)) == -1   # u overlaps f
    off = np.zeros(65, dtype=np.int32)
    cc = np.zeros(130)
    assert lib.rexii_apply_circulant(70, 65, off.ctypes.data_as(ctypes.c_void_p), cc.ctypes.data_as(ctypes.c_void_p),
                                     1, dummy, far, 1.0, 0.0, 0, 0, None, None, 0, None, None) == -1
