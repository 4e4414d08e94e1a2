"""Writes varh2048_trho<T>.json: sampled values of exp(tA) f for the 2048^2
variable-depth workload (flux form, H = 1 + 0.3 sin(2 pi x) cos(2 pi y),
g = 1, f_c = 20, t rho = T with rho the guaranteed spectral bound, initial
height 16 seeded bumps, seed 50), computed by the oracle's Chebyshev-Bessel
series.  Calls only the oracle and the input generators.

    python tests/golden/make_varh2048.py          (t rho = 100: about two minutes on one core)
    python tests/golden/make_varh2048.py 5000     (t rho = 5000: about an hour)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lrsw, varh  # noqa: E402
from paper_2008_11607_amd import inputs  # noqa: E402

D, FC, SEED, NSAMP, SAMPLE_SEED = 2048, 20.0, 50, 4096, 501


def main(TRHO=100.0):
    Hf = inputs.variable_depth(D)
    op = lrsw.LRSW(D, D, g=1.0, fc=FC, Hfield=Hf)
    rho = lrsw.rho(op)
    t = TRHO / rho
    f = inputs.gaussian_bumps(D, nbumps=16, seed=SEED)
    u = varh.chebyshev_expm(op, f, t)
    idx = inputs.sample_indices(3 * D, D, NSAMP, SAMPLE_SEED)   # flat over [3][D][D]
    out = dict(
        D=D, g=1.0, f_c=FC, t_rho=TRHO, rho=rho, t=t, seed=SEED, nbumps=16,
        depth="1 + 0.3 sin(2 pi x) cos(2 pi y)",
        reference="oracle Chebyshev-Bessel series (varh.chebyshev_expm)",
        norm_u=float(np.linalg.norm(u)), w_energy_f=float(varh.w_energy(op, f)),
        w_energy_u=float(varh.w_energy(op, u)),
        index=[int(i) for i in idx], value=[float(v) for v in u.reshape(-1)[idx]])
    with open(os.path.join(HERE, f"varh2048_trho{int(TRHO)}.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main(float(sys.argv[1]) if len(sys.argv) > 1 else 100.0)
