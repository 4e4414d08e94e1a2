"""Consistency of the stored oracle samples of the 2048^2 variable-depth
(t rho = 100 and 5000) and the 512^2 and 2048^2 constant-depth benchmark
workloads (written by the scripts in tests/golden from the oracle)."""
import json
import os

import numpy as np
import pytest

from oracle import lrsw
from paper_2008_11607_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("name", ["varh2048_trho100.json", "varh2048_trho5000.json"])
def test_varh2048_golden_metadata(name):
    with open(os.path.join(HERE, "golden", name)) as fh:
        g = json.load(fh)
    D = g["D"]
    op = lrsw.LRSW(D, D, g=g["g"], fc=g["f_c"], Hfield=inputs.variable_depth(D))
    rho = lrsw.rho(op)
    assert abs(rho - g["rho"]) <= 1e-12 * rho
    assert abs(g["t"] * rho - g["t_rho"]) <= 1e-12 * g["t_rho"]
    idx = np.asarray(g["index"])
    assert len(idx) == len(g["value"]) == len(np.unique(idx))
    assert idx.min() >= 0 and idx.max() < 3 * D * D
    # exp(tA) conserves the W-energy: the stored reference does to 1e-13 per
    # 100 of t rho (the rounding of the Chebyshev-Bessel recurrence grows
    # with its ~t rho terms)
    assert abs(g["w_energy_u"] / g["w_energy_f"] - 1.0) <= 1e-13 * max(1.0, g["t_rho"] / 100.0)
    # the input energy matches the seeded generator
    f = inputs.gaussian_bumps(D, nbumps=g["nbumps"], seed=g["seed"])
    from oracle import varh
    assert abs(varh.w_energy(op, f) / g["w_energy_f"] - 1.0) <= 1e-14


@pytest.mark.parametrize("name", ["lrsw512_trho1000.json", "lrsw2048_trho5000.json"])
def test_lrsw_golden_metadata(name):
    """The stored samples of the constant-depth workloads (written by
    tests/golden/make_lrsw512.py and make_lrsw2048.py from the oracle's
    closed form)."""
    with open(os.path.join(HERE, "golden", name)) as fh:
        g = json.load(fh)
    D = g["D"]
    op = lrsw.LRSW(D, D, g=g["g"], H=g["H"], fc=g["f_c"])
    rho = lrsw.rho(op)
    assert abs(rho - g["rho"]) <= 1e-12 * rho
    assert abs(g["t"] * rho - g["t_rho"]) <= 1e-12 * g["t_rho"]
    idx = np.asarray(g["index"])
    assert len(idx) == len(g["value"]) == len(np.unique(idx))
    assert idx.min() >= 0 and idx.max() < 3 * D * D
    # g = H: the plain norm is conserved by exp(tA)
    assert abs(g["norm_u"] / g["norm_f"] - 1.0) <= 1e-13
    f = inputs.gaussian_bumps(D, nbumps=g["nbumps"], seed=g["seed"])
    assert abs(np.linalg.norm(f) / g["norm_f"] - 1.0) <= 1e-14


def test_adjoint_golden_metadata():
    """The stored gradients of the adjoint workload (tests/golden/
    make_adjoint256.py): the seeded inputs and y are reproduced, and the
    loss and depth gradient of the approximant agree with those of the
    exact exponential to the approximation's accuracy."""
    from oracle import adjoint as adj
    from oracle import expm_modes as em
    with open(os.path.join(HERE, "golden", "adjoint256_trho500.json")) as fh:
        g = json.load(fh)
    D = g["D"]
    op = lrsw.LRSW(D, D, g=g["g"], H=g["H"], fc=g["f_c"])
    rho = lrsw.rho(op)
    assert abs(rho - g["rho"]) <= 1e-12 * rho
    assert abs(g["t"] * rho - g["t_rho"]) <= 1e-12 * g["t_rho"]
    idx = np.asarray(g["sample_index"])
    assert np.array_equal(idx, inputs.sample_indices(D, D, len(idx), 43))
    # y = P exp(tA) f* for the hidden state
    fstar = inputs.gaussian_bumps(D, nbumps=g["nbumps"], seed=g["seed_fstar"])
    y = adj.sample(em.expm_closed_real(op, fstar, g["t"]), idx)
    assert np.max(np.abs(y - np.asarray(g["y"]))) <= 1e-14 * np.max(np.abs(y))
    # approximant vs exact: h = 0.5, tol 1e-10 poles
    assert abs(g["J"] - g["J_exact"]) <= 1e-10 * g["J_exact"]
    assert abs(g["dJdH"] - g["dJdH_exact"]) <= 1e-10 * abs(g["dJdH_exact"])
    assert g["P"] == 2068
    out = np.asarray(g["index"])
    assert len(out) == len(g["dJdf"]) == len(np.unique(out)) and out.max() < 3 * D * D


def test_matrix_cases_golden():
    """The stored exponentials of the paper's matrix test cases and of the
    large circulant workloads (tests/golden/make_matrix_cases.py): the input
    generators' stencils are the oracle's A_1 and A_2, the 70-point values
    are the oracle's dense expm, and exp(tA) of a skew-Hermitian A conserves
    the norm of the (real, unit-free) inputs."""
    from oracle import matrix_cases as mc
    with open(os.path.join(HERE, "golden", "matrix_cases.json")) as fh:
        g = json.load(fh)
    n = g["A1"]["n"]
    assert inputs.advection_stencil(n) == mc.stencil_A1(n)
    s_in, s_or = inputs.schroedinger_stencil(n), mc.stencil_A2(n)
    assert s_in.keys() == s_or.keys() and all(abs(s_in[d] - s_or[d]) <= 1e-12 * abs(s_or[d]) for d in s_or)
    assert np.array_equal(inputs.matrix_case_vector(n), mc.f0(mc.grid_A1(n)))
    assert np.array_equal(inputs.matrix_case_vector(n, start=-1.0, length=2.0), mc.f0(mc.grid_A2(n)))
    e1 = mc.expm_circulant(n, mc.stencil_A1(n), mc.f0(mc.grid_A1(n)))
    assert np.max(np.abs(e1.real - np.asarray(g["A1"]["re"]))) <= 1e-13
    e2 = mc.expm_circulant(n, mc.stencil_A2(n), mc.f0(mc.grid_A2(n)))
    assert np.max(np.abs(e2 - (np.asarray(g["A2"]["re"]) + 1j * np.asarray(g["A2"]["im"])))) <= 1e-12
    for name in ("advection", "schroedinger"):
        c = g[name]
        assert abs(c["t"] * c["rho"] - c["t_rho"]) <= 1e-12 * c["t_rho"]
        f = inputs.random_vectors(c["n"], c["nrhs"], c["seed"])
        assert abs(c["norm"] / np.linalg.norm(f) - 1.0) <= 1e-12
        idx = np.asarray(c["index"])
        assert len(idx) == len(c["re"]) == len(np.unique(idx)) and idx.max() < c["n"] * c["nrhs"]
