"""Adjoint of the HIP path (rexii_apply_adjoint and the autograd Function)
against the oracle's exact adjoints and central finite differences."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import coeffs as oc
from oracle import expm_modes as em
from oracle import lrsw
from oracle import rexii_modes as rm
from paper_2008_11607_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rx():
    import torch
    assert torch.cuda.is_available()
    from paper_2008_11607_amd import rexii
    rexii.load()
    return rexii


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _setup(nx, ny, trho, g=1.0, H=1.0, fc=10.0, velocity=False, nsamp=64, seed=41):
    op = lrsw.LRSW(nx, ny, g=g, H=H, fc=fc)
    rho = lrsw.rho(op)
    t = trho / rho
    fstar = inputs.gaussian_bumps(nx, ny, nbumps=4, seed=seed)
    f = inputs.gaussian_bumps(nx, ny, nbumps=4, seed=seed + 1, velocity=velocity)
    idx = inputs.sample_indices(nx, ny, nsamp, seed + 2)
    y = adj.sample(em.expm_closed_real(op, fstar, t), idx)
    return op, rho, t, f, idx, y


@pytest.mark.parametrize("nx,ny,g,H,velocity", [(64, 64, 1.0, 1.0, False), (72, 40, 1.3, 0.8, True)])
def test_adjoint_matches_oracle(rx, nx, ny, g, H, velocity):
    op, rho, t, f, idx, y = _setup(nx, ny, 80.0, g=g, H=H, velocity=velocity)
    c = oc.api_coeffs(t, rho, h=0.5, tol=1e-10)
    u = rm.rexii_spectral(op, f, t, c["z"], c["w"])
    gbar = adj.grad_u(u, idx, y)
    dJdf, dJdH, rep = rx.apply_adjoint(_dev(f), _dev(gbar), t, g=g, fc=op.fc, H=H)
    ref_f = adj.rexii_T_spectral(op, gbar, t, c["z"], c["w"])
    assert em.rel_l2(dJdf.cpu().numpy(), ref_f) <= 1e-10
    ref_H = float(np.sum(gbar * adj.frechet_rexii_apply(op, f, t, c["z"], c["w"])))
    assert abs(dJdH - ref_H) <= 1e-9 * max(1.0, abs(ref_H))


def test_adjoint_dot_test(rx):
    op, rho, t, f, idx, y = _setup(64, 48, 60.0, g=1.5, H=0.7, velocity=True)
    rng = np.random.default_rng(3)
    gbar = rng.standard_normal(f.shape)
    u, _ = rx.apply(_dev(f), t, g=op.g, fc=op.fc, H=op.H)
    dJdf, _, _ = rx.apply_adjoint(None, _dev(gbar), t, g=op.g, fc=op.fc, H=op.H, want_dJdH=False)
    lhs = float(np.sum(u.cpu().numpy() * gbar))
    rhs = float(np.sum(f * dJdf.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0)


def test_autograd_against_finite_differences(rx):
    import torch
    op, rho, t, f, idx, y = _setup(48, 48, 50.0)
    fd = _dev(f).requires_grad_(True)
    Ht = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    idx_t = torch.from_numpy(idx).cuda()
    y_t = _dev(y)

    def J(ff, HH):
        u = rx.rexii_exp(ff, HH, t, fc=op.fc, rho=rho)
        r = u[0].reshape(-1)[idx_t] - y_t
        return (r * r).sum()

    loss = J(fd, Ht)
    loss.backward()
    gf = fd.grad.detach().cpu().numpy()
    gH = float(Ht.grad)
    eps = 1e-6
    rng = np.random.default_rng(8)
    with torch.no_grad():
        for _ in range(3):
            d = _dev(rng.standard_normal(f.shape))
            fdv = (float(J(fd + eps * d, Ht)) - float(J(fd - eps * d, Ht))) / (2 * eps)
            assert abs(fdv - float(np.sum(gf * d.cpu().numpy()))) <= 1e-6 * max(1.0, abs(fdv))
        epsH = 1e-5
        Hp = torch.tensor(1.0 + epsH, dtype=torch.float64, device="cuda")
        Hm = torch.tensor(1.0 - epsH, dtype=torch.float64, device="cuda")
        fdH = (float(J(fd, Hp)) - float(J(fd, Hm))) / (2 * epsH)
    assert abs(fdH - gH) <= 1e-6 * max(1.0, abs(fdH))


@pytest.fixture(scope="module")
def case256():
    # the adjoint workload: 256^2, t rho = 500, 1024 sampled eta points, y
    # from a hidden state (seed 41), f from seed 42; the pole set of tol 1e-10
    op, rho, t, f, idx, y = _setup(256, 256, 500.0, nsamp=1024)
    c = oc.api_coeffs(t, rho, h=0.5, tol=1e-10)
    J, dJdf, dJdH = adj.grad_rexii(op, f, t, c["z"], c["w"], idx, y)
    u = rm.rexii_spectral(op, f, t, c["z"], c["w"])
    return dict(op=op, rho=rho, t=t, f=f, idx=idx, y=y, c=c, J=J, dJdf=dJdf, dJdH=dJdH,
                gbar=adj.grad_u(u, idx, y))


def test_adjoint_256_vs_oracle_approximant(rx, case256):
    """rexii_apply_adjoint at 256^2 against the oracle's gradients of the same
    approximant (the transposed pole sum and its Frechet derivative in H)."""
    k = case256
    print("adjoint 256^2 t rho 500", flush=True)
    dJdf, dJdH, rep = rx.apply_adjoint(_dev(k["f"]), _dev(k["gbar"]), k["t"], fc=k["op"].fc)
    assert rep["P"] == len(k["c"]["z"]) == 2068 and rep["not_converged"] == 0
    assert rep["err_bound"] <= 1e-10
    ef = em.rel_l2(dJdf.cpu().numpy(), k["dJdf"])
    eh = abs(dJdH - k["dJdH"]) / abs(k["dJdH"])
    print(f"  dJ/df rel {ef:.3e}  dJ/dH rel {eh:.3e}", flush=True)
    assert ef <= 1e-10
    assert eh <= 1e-10


def test_adjoint_256_vs_exact_gradient(rx, case256):
    """The same gradients against the exact exponential's (the approximation
    error of the pole set is ~1e-13 at h = 0.5)."""
    k = case256
    J_ex, dJdf_ex, dJdH_ex = adj.grad_exact(k["op"], k["f"], k["t"], k["idx"], k["y"])
    dJdf, dJdH, _ = rx.apply_adjoint(_dev(k["f"]), _dev(k["gbar"]), k["t"], fc=k["op"].fc)
    assert em.rel_l2(dJdf.cpu().numpy(), dJdf_ex) <= 1e-9
    assert abs(dJdH - dJdH_ex) <= 1e-9 * abs(dJdH_ex)


def test_autograd_256_vs_central_differences(rx, case256):
    """torch.autograd through RexiiExp at 256^2 against central differences
    (eps = 1e-6, FP64) of J in 8 random directions of f and in H.  J is
    evaluated with the GPU's Fourier-space REXII for the same frozen pole set
    (rho and m0 fixed): the same approximant as the Krylov forward, evaluated
    without iterations, so J is linear in f up to rounding and its
    differences are not swamped by solver tolerances."""
    import torch
    k = case256
    op, t, rho = k["op"], k["t"], k["rho"]
    m0 = k["c"]["m0"]
    idx_t = torch.from_numpy(k["idx"]).cuda()
    y_t = _dev(k["y"])
    fd = _dev(k["f"]).requires_grad_(True)
    Ht = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    u = rx.rexii_exp(fd, Ht, t, fc=op.fc, rho=rho)
    r = u[0].reshape(-1)[idx_t] - y_t
    (r * r).sum().backward()
    gf = fd.grad.detach()
    gH = float(Ht.grad)

    def J(ff, HH):
        uu, _ = rx.apply_fourier(ff, t, fc=op.fc, H=HH, rho=rho, m0=m0, tol=1e-10)
        rr = uu[0].reshape(-1)[idx_t] - y_t
        return float((rr * rr).sum())

    eps = 1e-6
    rng = np.random.default_rng(44)
    with torch.no_grad():
        f0 = fd.detach()
        for j in range(8):
            d = _dev(rng.standard_normal(k["f"].shape))
            fdv = (J(f0 + eps * d, 1.0) - J(f0 - eps * d, 1.0)) / (2 * eps)
            an = float((gf * d).sum())
            print(f"  direction {j}: FD {fdv:.12e} autograd {an:.12e} rel {abs(fdv - an) / abs(fdv):.2e}",
                  flush=True)
            assert abs(fdv - an) <= 1e-8 * abs(fdv)
        fdH = (J(f0, 1.0 + eps) - J(f0, 1.0 - eps)) / (2 * eps)
    print(f"  H: FD {fdH:.12e} autograd {gH:.12e}", flush=True)
    assert abs(fdH - gH) <= 1e-8 * abs(fdH)
