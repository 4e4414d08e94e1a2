"""Writes lrsw2048_trho5000.json: sampled values of the exact exp(tA) f for a
2048^2 constant-depth workload (g = H = 1, f_c = 20, t rho = 5000 with rho the
exact discrete spectral radius, initial height 16 seeded bumps, seed 5),
from the oracle's per-mode closed form.  Calls only the oracle and the
input generators.

    python tests/golden/make_lrsw2048.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import expm_modes as em  # noqa: E402
from oracle import lrsw  # noqa: E402
from paper_2008_11607_amd import inputs  # noqa: E402

D, FC, TRHO, SEED, NSAMP, SAMPLE_SEED = 2048, 20.0, 5000.0, 5, 4096, 2048


def main():
    op = lrsw.LRSW(D, D, g=1.0, fc=FC)
    rho = lrsw.rho(op)
    t = TRHO / rho
    f = inputs.gaussian_bumps(D, nbumps=16, seed=SEED)
    u = em.expm_closed_real(op, f, t)
    idx = inputs.sample_indices(3 * D, D, NSAMP, SAMPLE_SEED)   # flat over [3][D][D]
    out = dict(D=D, g=1.0, H=1.0, f_c=FC, t_rho=TRHO, rho=rho, t=t, seed=SEED, nbumps=16,
               reference="oracle per-mode closed form (expm_modes.expm_closed_real)",
               norm_u=float(np.linalg.norm(u)), norm_f=float(np.linalg.norm(f)),
               index=[int(i) for i in idx], value=[float(v) for v in u.reshape(-1)[idx]])
    with open(os.path.join(HERE, "lrsw2048_trho5000.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
