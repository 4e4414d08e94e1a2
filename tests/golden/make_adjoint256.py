"""Writes adjoint256_trho500.json: the gradient workload of the adjoint path
(constant depth g = H = 1, f_c = 10, 256^2, t rho = 500 with rho the exact
discrete spectral radius; loss J = |P u - y|^2 with P sampling 1024 eta
points, seed 43; y = P exp(tA) f* for a hidden state f*, 4 bumps, seed 41;
the state f, 4 bumps, seed 42).  Stored: the sample indices and y, and the
oracle's gradients of the REXII approximant for the pole set of tol 1e-10
(h = 0.5): J, dJ/dH and dJ/df at 8192 sampled points with its norm; also
the exact exponential's dJ/dH.  Calls only the oracle and the input
generators.

    python tests/golden/make_adjoint256.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import adjoint as adj  # noqa: E402
from oracle import coeffs as oc  # noqa: E402
from oracle import expm_modes as em  # noqa: E402
from oracle import lrsw  # noqa: E402
from paper_2008_11607_amd import inputs  # noqa: E402

D, FC, TRHO, NSAMP, TOL = 256, 10.0, 500.0, 1024, 1e-10
SEED_FSTAR, SEED_F, SEED_IDX, SAMPLE_SEED, NOUT = 41, 42, 43, 544, 8192


def main():
    op = lrsw.LRSW(D, D, g=1.0, fc=FC)
    rho = lrsw.rho(op)
    t = TRHO / rho
    fstar = inputs.gaussian_bumps(D, nbumps=4, seed=SEED_FSTAR)
    f = inputs.gaussian_bumps(D, nbumps=4, seed=SEED_F)
    idx = inputs.sample_indices(D, D, NSAMP, SEED_IDX)
    y = adj.sample(em.expm_closed_real(op, fstar, t), idx)
    c = oc.api_coeffs(t, rho, h=0.5, tol=TOL)
    J, dJdf, dJdH = adj.grad_rexii(op, f, t, c["z"], c["w"], idx, y)
    J_ex, _, dJdH_ex = adj.grad_exact(op, f, t, idx, y)
    out_idx = inputs.sample_indices(3 * D, D, NOUT, SAMPLE_SEED)  # flat over [3][D][D]
    out = dict(D=D, g=1.0, H=1.0, f_c=FC, t_rho=TRHO, rho=rho, t=t, tol=TOL, h=0.5, P=len(c["z"]),
               seed_fstar=SEED_FSTAR, seed_f=SEED_F, nbumps=4, sample_index=[int(i) for i in idx],
               y=[float(v) for v in y],
               reference="oracle gradients of the REXII approximant (adjoint.grad_rexii) for the pole set "
                         "of tol 1e-10; dJdH_exact from adjoint.grad_exact",
               J=float(J), dJdH=float(dJdH), J_exact=float(J_ex), dJdH_exact=float(dJdH_ex),
               norm_dJdf=float(np.linalg.norm(dJdf)),
               index=[int(i) for i in out_idx], dJdf=[float(v) for v in dJdf.reshape(-1)[out_idx]])
    with open(os.path.join(HERE, "adjoint256_trho500.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
