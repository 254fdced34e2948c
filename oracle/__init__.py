"""Plain FP64 CPU oracle for the multi-sphere T-matrix method (CELES, Egel et
al. 2017).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it.  It is written for obvious correctness, not speed: dense matrices, exact
rational Wigner-3j symbols, library special functions and plain loops.  It
shares no code with the HIP library; both read the same seeded inputs from
`celes_inputs`.

Modules (each function cites the passage of the paper it follows):
  special      spherical Bessel/Hankel, normalized Legendre, pi/tau functions
  wigner       exact Wigner-3j symbols (Racah formula, rational arithmetic)
  translation  a5/b5 coefficients, SVWF translation operator, dense W
  rotation     Wigner-d basis rotation, rotation-translation-rotation form of A
  svwf         spherical and plane vector wave functions (field evaluation)
  mie          sphere T-matrix (paper formula) and an independent Mie series
  incident     plane-wave and Gaussian-beam initial-field coefficients
  lut          cubic-Hermite Hankel lookup table
  solve        master equation, dense LU, block-diagonal preconditioner, GMRES
  observables  cross sections, far field, near field
  mlp          FP64 reference network for the learned initial guess

Every function is pinned by tests against facts that do not come from the
oracle itself (see tests/test_oracle_*.py); any function without such a pin
says "parity unpinned" in its docstring.
"""
