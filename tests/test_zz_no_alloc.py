"""rexii_apply_fourier_noalloc, the entry point for callers that cannot
allocate device memory, through the C ABI: the same result as
rexii_apply_fourier on two calls in a row (the second on a smaller grid,
after the first has left its data in the static scratch), both within the
oracle's bar for the Fourier path; sizes beyond the static scratch and grids
without FFT plans are refused with an error, and the non-finite check still
works without pinned memory."""
import numpy as np
import pytest

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


def test_noalloc_matches_apply_fourier_two_calls(rx):
    import torch
    # a larger grid first, then a smaller one: the second call must not
    # depend on what the first left in the shared scratch
    cases = [(160, 144, 400.0, 10.0, 71), (64, 48, 100.0, 20.0, 72)]
    for nx, ny, trho, fc, seed in cases:
        print(f"noalloc fourier {nx}x{ny} t rho {trho}", flush=True)
        op = lrsw.LRSW(nx, ny, fc=fc)
        rho = lrsw.rho(op)
        t = trho / rho
        f = inputs.gaussian_bumps(nx, ny, nbumps=6, seed=seed, velocity=True)
        fd = _dev(f)
        rx.fourier_workspace_size(nx, ny, t, fc=fc)  # set-up: creates the grid's FFT plans
        ref, rref = rx.apply_fourier(fd, t, fc=fc)
        u = torch.full_like(fd, float("nan"))
        got, rep = rx.apply_fourier_noalloc(fd, t, fc=fc, out=u)
        torch.cuda.synchronize()
        assert got.data_ptr() == u.data_ptr()
        # same kernels, plans and arithmetic order: bitwise the same result
        assert torch.equal(got, ref)
        for k in ("P", "M", "N", "solves", "total_iters"):
            assert rep[k] == rref[k], k
        c = oc.api_coeffs(t, rho, h=0.5, tol=1e-10)
        assert rep["P"] == len(c["z"])
        oracle = rm.rexii_spectral(op, f, t, c["z"], c["w"])
        assert em.rel_l2(got.cpu().numpy(), oracle) <= 1e-12


def test_noalloc_refuses_what_it_cannot_do(rx):
    import torch
    # no FFT plan for this grid yet: creating one would allocate
    f = _dev(inputs.gaussian_bumps(53, 47, nbumps=2, seed=3))
    with pytest.raises(rx.RexiiError) as e:
        rx.apply_fourier_noalloc(f, 0.01, fc=10.0)
    assert e.value.status == -1 and "plan" in str(e.value)
    # half spectra alone beyond the static scratch (4096^2: 403 MB)
    big = torch.zeros((3, 4096, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(rx.RexiiError) as e:
        rx.apply_fourier_noalloc(big, 0.001, fc=10.0)
    assert e.value.status == -7
    del big
    # non-finite input: reported, as by the allocating entry point
    nx = 64
    rx.fourier_workspace_size(nx, nx, 0.01, fc=10.0)
    g = inputs.gaussian_bumps(nx, nbumps=2, seed=4)
    g[1, 3, 5] = np.inf
    with pytest.raises(rx.RexiiError) as e:
        rx.apply_fourier_noalloc(_dev(g), 0.01, fc=10.0)
    assert e.value.status == -2
    # and a finite call right after it starts from a cleared flag
    h = inputs.gaussian_bumps(nx, nbumps=2, seed=5)
    u, _ = rx.apply_fourier_noalloc(_dev(h), 0.01, fc=10.0)
    ref, _ = rx.apply_fourier(_dev(h), 0.01, fc=10.0)
    assert torch.equal(u, ref)
