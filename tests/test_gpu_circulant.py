"""Parity of the circulant-matrix path (rexii_apply_circulant, through the C
ABI) with the FP64 CPU oracle: the paper's matrix experiments (Sec. 3.2,
Fig. matrixRexiExample) with REXII (eq. modifiedRexiMatrixReducedSum), the
original REXI (eq. originalREXImatrix) and REXIE (eq. REXIE).

Every resolvent is exact per Fourier mode on both sides, so the GPU result is
held to the oracle's per-mode evaluation of the same scheme (itself pinned to
dense solves and dense expm) at round-off level, and the figure's claims are
checked on the GPU's own results against dense expm."""
import numpy as np
import pytest

from oracle import coeffs as oc
from oracle import matrix_cases as mc

pytestmark = pytest.mark.gpu

N_PTS = 70
BAR = 1e-11     # GPU vs the oracle's per-mode form of the same scheme


@pytest.fixture(scope="module")
def rx():
    import torch
    assert torch.cuda.is_available()
    from paper_2008_11607_amd import rexii
    rexii.load()
    return rexii


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def cases():
    st1, st2 = mc.stencil_A1(N_PTS), mc.stencil_A2(N_PTS)
    f1, f2 = mc.f0(mc.grid_A1(N_PTS)), mc.f0(mc.grid_A2(N_PTS))
    ref1 = mc.expm_dense(mc.circulant_dense(N_PTS, st1), f1)
    ref2 = mc.expm_dense(mc.circulant_dense(N_PTS, st2), f2)
    return dict(st1=st1, st2=st2, f1=f1, f2=f2, ref1=ref1, ref2=ref2)


@pytest.mark.parametrize("h", [0.2, 0.5])
@pytest.mark.parametrize("reach", [30.0, 50.0, 70.0, 140.0])
def test_rexii_and_rexi_on_A1_match_oracle(rx, cases, h, reach):
    # one point of Fig. matrixRexiExample (a) and (b) each: M from the bound
    # for the given reach
    M = oc.M_rule(1.0, reach, h, 11)
    f = cases["f1"]
    for scheme, orc in (("rexii", mc.rexii_circulant), ("rexi", mc.rexi_circulant)):
        u, rep = rx.apply_circulant(_dev(f), 1.0, cases["st1"], scheme=scheme, M=M, h=h)
        ref = orc(N_PTS, cases["st1"], f, M, h)
        got = _host(u)
        assert np.max(np.abs(got.imag)) == 0.0
        e = mc.rel_l2(got.real, ref)
        print(f"A1 {scheme} h={h} M={M}: GPU vs oracle {e:.2e}", flush=True)
        assert e <= BAR
        assert rep["M"] == M and rep["P"] == (2 * (M + 25) if scheme == "rexii" else 2 * (M + 24) + 1)
        rho1 = float(np.max(np.abs(mc.circulant_symbol(N_PTS, cases["st1"]))))
        assert abs(rep["rho"] - rho1) <= 1e-12 * rho1


def test_figure_matrix_example_on_gpu(rx, cases):
    """Fig. matrixRexiExample on the GPU's own results (h = 0.5): REXII's error
    drops to round-off once (M - 11) h reaches rho(A_1) (eq. matrixAccuracyBound)
    and not before; the original REXI stays far above it for the same M;
    REXIE on the shifted A_2 is accurate at the M of the bound for 2450."""
    h = 0.5
    f, ref = cases["f1"], cases["ref1"].real
    rho1 = float(np.max(np.abs(mc.circulant_symbol(N_PTS, cases["st1"]))))
    errs = {}
    for M in (60, 100, 140, oc.M_rule(1.0, rho1, h, 11), 200, 400):
        ur, rr = rx.apply_circulant(_dev(f), 1.0, cases["st1"], scheme="rexii", M=M, h=h)
        ui, _ = rx.apply_circulant(_dev(f), 1.0, cases["st1"], scheme="rexi", M=M, h=h)
        errs[M] = (mc.rel_l2(_host(ur).real, ref), mc.rel_l2(_host(ui).real, ref))
        print(f"M={M}: REXII {errs[M][0]:.2e}  REXI {errs[M][1]:.2e}", flush=True)
    Mb = oc.M_rule(1.0, rho1, h, 11)
    assert abs(rr["rho"] - rho1) <= 1e-12 * rho1
    for M, (e_rexii, e_rexi) in errs.items():
        if M >= Mb:
            assert e_rexii <= 1e-13
            assert e_rexi >= 1e-7 and e_rexi >= 1e6 * e_rexii
        elif (M - 11) * h < 0.75 * rho1:
            assert e_rexii >= 1e-7
    # REXIE on A_2 - nu I, nu = -2450 i
    f2, ref2 = cases["f2"], cases["ref2"]
    ue, re_ = rx.apply_circulant(_dev(f2), 1.0, cases["st2"], scheme="rexie", nu=-2450j,
                                 M=oc.M_rule(1.0, 2450.0, h, 11), h=h)
    assert abs(re_["rho"] - 2450.0) <= 1e-9 * 2450.0
    assert mc.rel_l2(_host(ue), ref2) <= 1e-12
    ue_short, _ = rx.apply_circulant(_dev(f2), 1.0, cases["st2"], scheme="rexie", nu=-2450j,
                                     M=oc.M_rule(1.0, 2300.0, h, 11), h=h)
    assert mc.rel_l2(_host(ue_short), ref2) >= 0.1


@pytest.mark.parametrize("reach", [2300.0, 2450.0, 4900.0])
def test_rexie_on_A2_matches_oracle(rx, cases, reach):
    h = 0.5
    M = oc.M_rule(1.0, reach, h, 11)
    u, rep = rx.apply_circulant(_dev(cases["f2"]), 1.0, cases["st2"], scheme="rexie", nu=-2450j, M=M, h=h)
    ref = mc.rexie_circulant(N_PTS, cases["st2"], cases["f2"], M, h, nu=-2450j)
    e = mc.rel_l2(_host(u), ref)
    print(f"A2 REXIE M={M}: GPU vs oracle {e:.2e}", flush=True)
    assert e <= BAR
    assert rep["P"] == 2 * (M + 24) + 1


def test_m_from_the_rule_and_tolerance(rx, cases):
    # M <= 0: eq. matrixAccuracyBound with the exact rho and m0 from tol
    u, rep = rx.apply_circulant(_dev(cases["f1"]), 1.0, cases["st1"], scheme="rexii", tol=1e-10)
    rho1 = float(np.max(np.abs(mc.circulant_symbol(N_PTS, cases["st1"]))))
    assert rep["M"] == oc.M_rule(1.0, rho1, 0.5, oc.m0_of_tol(1e-10))
    assert mc.rel_l2(_host(u).real, cases["ref1"].real) <= 1e-10


@pytest.mark.parametrize("n,nrhs", [(4096, 3), (1001, 2), (2, 1), (65536, 1)])
def test_larger_and_ragged_sizes_match_oracle(rx, n, nrhs):
    """Grids beyond the paper's 70 points (several blocks of the pole-sum
    kernel, odd and tiny lengths, several vectors per call): a fourth-order
    centred difference (skew-symmetric) with REXII and REXI, and i times a
    wide symmetric stencil with REXIE."""
    rng = np.random.default_rng(n)
    f = rng.standard_normal((nrhs, n))
    t = 150.0 / n          # t rho of a few hundred: the oracle's per-mode sums stay quick
    skew = {1: 2.0 / 3.0 * n, -1: -2.0 / 3.0 * n, 2: -1.0 / 12.0 * n, -2: 1.0 / 12.0 * n}
    sym = {0: -2.5j * n, 1: 1.2j * n, -1: 1.2j * n, 3: 0.05j * n, -3: 0.05j * n}
    for scheme, st, nu in (("rexii", skew, 0.0), ("rexi", skew, 0.0), ("rexie", sym, -1.3j * n)):
        u, rep = rx.apply_circulant(_dev(f), t, st, scheme=scheme, nu=nu, h=0.5, tol=1e-10)
        M = rep["M"]
        got = _host(u)
        for r in range(nrhs):
            if scheme == "rexii":
                ref = mc.rexii_circulant(n, st, f[r], M, 0.5, t=t)
            elif scheme == "rexi":
                ref = mc.rexi_circulant(n, st, f[r], M, 0.5, t=t)
            else:
                ref = mc.rexie_circulant(n, st, f[r], M, 0.5, t=t, nu=nu)
            e = mc.rel_l2(got[r] if scheme == "rexie" else got[r].real, ref)
            assert e <= BAR, (scheme, r, e)
        if scheme == "rexii":
            # and the exact exponential
            ex = mc.expm_circulant(n, st, f[0], t=t).real
            assert mc.rel_l2(got[0].real, ex) <= 1e-9


def test_edge_cases(rx, cases):
    import torch
    f = cases["f1"]
    # t = 0: u = f
    u, _ = rx.apply_circulant(_dev(f), 0.0, cases["st1"], scheme="rexii")
    assert np.array_equal(_host(u).real, f) and np.all(_host(u).imag == 0)
    # a non-finite input is reported (u is written anyway)
    fb = f.copy()
    fb[5] = np.nan
    with pytest.raises(rx.RexiiError) as e:
        rx.apply_circulant(_dev(fb), 1.0, cases["st1"], scheme="rexii", M=100)
    assert e.value.status == -2
    # a caller workspace gives the same result bit for bit
    ws_bytes = rx.circulant_workspace_size(N_PTS, 1.0, cases["st1"], scheme="rexii", M=120)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    lib = rx.load()
    import ctypes
    off, cc = rx._stencil_arrays(cases["st1"])
    fd = _dev(f)
    u1 = torch.empty(N_PTS, dtype=torch.complex128, device="cuda")
    u2, _ = rx.apply_circulant(fd, 1.0, cases["st1"], scheme="rexii", M=120)
    st = lib.rexii_apply_circulant(N_PTS, len(off), off.ctypes.data_as(ctypes.c_void_p),
                                   cc.ctypes.data_as(ctypes.c_void_p), 1, ctypes.c_void_p(fd.data_ptr()),
                                   ctypes.c_void_p(u1.data_ptr()), 1.0, 0.0, 0, 120, None,
                                   ctypes.c_void_p(ws.data_ptr()), ws_bytes, rx._stream(), None)
    assert st == 0
    assert torch.equal(u1, u2)
    st = lib.rexii_apply_circulant(N_PTS, len(off), off.ctypes.data_as(ctypes.c_void_p),
                                   cc.ctypes.data_as(ctypes.c_void_p), 1, ctypes.c_void_p(fd.data_ptr()),
                                   ctypes.c_void_p(u1.data_ptr()), 1.0, 0.0, 0, 120, None,
                                   ctypes.c_void_p(ws.data_ptr()), ws_bytes - 256, rx._stream(), None)
    assert st == -7
