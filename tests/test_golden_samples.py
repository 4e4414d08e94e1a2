"""Consistency of the stored oracle samples of the 2048^2 variable-depth and
512^2 benchmark workloads (written by the scripts in tests/golden from the oracle)."""
import json
import os

import numpy as np

from oracle import lrsw
from paper_2008_11607_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def test_varh2048_golden_metadata():
    with open(os.path.join(HERE, "golden", "varh2048_trho100.json")) as fh:
        g = json.load(fh)
    D = g["D"]
    op = lrsw.LRSW(D, D, g=g["g"], fc=g["f_c"], Hfield=inputs.variable_depth(D))
    rho = lrsw.rho(op)
    assert abs(rho - g["rho"]) <= 1e-12 * rho
    assert abs(g["t"] * rho - g["t_rho"]) <= 1e-12 * g["t_rho"]
    idx = np.asarray(g["index"])
    assert len(idx) == len(g["value"]) == len(np.unique(idx))
    assert idx.min() >= 0 and idx.max() < 3 * D * D
    # exp(tA) conserves the W-energy: the stored reference does to 1e-13
    assert abs(g["w_energy_u"] / g["w_energy_f"] - 1.0) <= 1e-13
    # the input energy matches the seeded generator
    f = inputs.gaussian_bumps(D, nbumps=g["nbumps"], seed=g["seed"])
    from oracle import varh
    assert abs(varh.w_energy(op, f) / g["w_energy_f"] - 1.0) <= 1e-14


def test_lrsw512_golden_metadata():
    """The stored samples of the 512^2 benchmark workload (written by
    tests/golden/make_lrsw512.py from the oracle's closed form)."""
    with open(os.path.join(HERE, "golden", "lrsw512_trho1000.json")) as fh:
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
