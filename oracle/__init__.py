"""Plain FP64 CPU reference for ESP long-range electrostatics.

TEST INFRASTRUCTURE ONLY. Nothing in the library imports, links or runs this
package; only the tests, the benchmark's CPU-baseline leg and the smoke check
use it. It shares no code, tables or constants with the GPU path: it
computes its own PSWF, parameters, influence function and five-step
pipeline from the paper's definitions.

Modules
  pswf      psi_0^c from the prolate differential operator in the even
            Legendre basis (Methods, PSWF section); the paper's own definition
            (Nystrom discretisation of the finite Fourier operator) serves only
            as an independent cross-check that pins it.
  split     the general radial kernel split (eq. kernelsplitting) for the PSWF
            kernel (eq. pswf) and, as a textbook special case, the Gaussian.
  ewald     classical Ewald summation (eq. ewalderf): physics ground truth.
  spectral  structure factors and the truncated spectral sum (eq.
            spectralpart) as a direct non-uniform DFT; the local sum (eq.
            localpart).
  fivestep  the five-step method (eqs. spread..interp) with the exact window
            and a plain matrix DFT, every stage exposed.
  params    the parameter rules (Table 2, eqs. pswfparameters and
            errorformula).
  metrics   relative RMS force error (eq. Deltadef).
  box, cell orthorhombic boxes and triclinic cells; classical: the Gaussian
            split with a B-spline window (eq. cem).

Every sum is evaluated by numpy's own loops (no BLAS call); the only LAPACK
use is the small PSWF eigenproblem.

Pins (see tests/test_oracle_*.py): Table 2 shape parameters, the Fig. 5 cut-off
numbers, the NaCl Madelung constant, brute-force image sums, the
Gaussian-split special case (exactly classical Ewald), Parseval, translation
invariance, and agreement of two independent PSWF solvers.
"""
