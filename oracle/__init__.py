"""CPU oracle for the SGN constraint solve and time stepping (test infrastructure).

This package is a plain, slow, FP64 NumPy implementation of what the device
path computes, written from the paper (Feng, Shirokoff, Choi, "Preconditioning
and Linearly Implicit Time Integration for the Serre-Green-Naghdi Equations",
arXiv 2506.16045).  It exists only to check the device path: tests,
the smoke check and the CPU baseline leg of the benchmark use it; the product
path never imports it.  It shares no code with the HIP library; only the seeded
input generators (paper_2506_16045_amd.inputs) serve both.

Modules:
  spectral     grid wavenumbers and the spectral derivative D (section 6.1)
  operators    G_{eta,h} (Def:G), its dense assembly, A and its inverse
               (Def:A, section 6.1), the coefficients sigma*, alpha*, kappa_ub
               (Eq:FlatbathCoeff, Eq:Optcoeff, Eq:Optcoeffb)
  krylov       textbook PCG (section 3.2) and restarted right-preconditioned GMRES
  rhs          the constraint-form right-hand side f(w, p) with forcing F
               (Eq:DSWEcf, Def:bigF, Eq:DAE_DSWE), and its de-aliased form
               on a zero-padded grid (subsec:dswe_1d, remark on aliasing)
  walls        G, A^{-1} and PCG between walls (homogeneous Neumann, Subsec:DAEform,
               Subsec:linop): cosine / sine series on a cell-centred grid
  stepping     RK4 (Eq:ERK), Adams-Bashforth 2-4 (Eq:AB, Table LMMCoeffs) and
               the linearly implicit SBDF2 scheme (Eq:MM)
  linimp       linearly implicit schemes of up to three steps (Eq:IMEX_DAE), the
               zero-stability checker of Eq:CharEq, and the third-order family
               with the joint choice of A's scale (section 5.4)
  diagnostics  mass, energy (Remark 2.1), the G-norm error (def:discrete_Gerr)

Every function that has no independent pin says "parity unpinned" in its
docstring; the pins live in tests/test_oracle_*.py.
"""
from . import spectral, operators, krylov, rhs, stepping, diagnostics, walls, linimp  # noqa: F401
