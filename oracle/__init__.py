"""Plain FP64 CPU oracle for the REXII exponential integrator (Caliari,
Einkemmer, Moriggl, Ostermann, arXiv 2008.11607).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
tables or constants with the HIP library (its Table A is a separate
transcription from the paper's Appendix A).

Modules
-------
table_a      the paper's Appendix A coefficients (mu, a_l), own transcription
coeffs       scalar REXII: b_m (Sec. 2.1 step 1), c_{1,n}, c_{2,n} (eq.
             modifiedRexi), C_{1,n}, C_{2,n} (Sec. 2.2), the reduced sum over
             n >= 0 (eq. modifiedRexiMatrixReducedSum) in partial fractions,
             the accuracy rule (eqs. Mformula / matrixAccuracyBound) and m0(tol)
             (Appendix B)
lrsw         the centred-difference linear rotating shallow-water operator,
             dense assembly, Fourier symbol, spectral radius (Sec. 4)
expm_modes   exact exp(tA)f per Fourier mode (closed form and eigh) and
             dense expm (Sec. 2.1, eqs. AisVEV / REXI_VEV_DECOMP)
rexii_modes  the exact REXII approximant r(tA)f per Fourier mode and per
             pole resolvents, without Krylov solves
adjoint      gradients of J = |P exp(tA) f - y|^2 w.r.t. f and the depth H
varh         variable-depth (flux form) operator: dense expm on small grids,
             Chebyshev-Bessel series reference
spectral     the paper's own spectral LRSW operator and test scenarios
             (Sec. 4, wave scenarios 1/2 and the Gaussian scenario)
matrix_cases the matrix test cases A_1, A_2 and f_0 of Sec. 3.2, circulant
             matrices, and REXII / the original REXI / REXIE (eq. REXIE, with
             the shift of Sec. 2.2) by dense solves and per Fourier mode
refit        a refit of the Gaussian's rational approximation (Sec. 2.1 step
             2, eqs. A(x,mu) and minl2approx): least squares on Leja-ordered
             points

Where a function has no independent pin in ``tests/`` its docstring says
"parity unpinned".
"""
