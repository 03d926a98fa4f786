"""FP64 CPU oracle for the disconnected-loop noise-subtraction method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy restatement of what the paper (Baral, Whyte, Wilcox, Morgan,
"Disconnected Loop Subtraction Methods in Lattice QCD", arXiv:1903.06986)
computes.  Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path never does, and it shares no
code with the HIP library (they meet only at the seeded input generators in
``synth``).

Modules
  lattice   conventions: gamma basis, site / vector indexing, parity
  noise     Z(4) noise from the SplitMix64 counter generator
  wilson    the Wilson matrix M = 1 - kappa P, its even/odd reduction, M gamma5
  krylov    GMRES-DR, GMRES-Proj, hermitian eigenpairs (Rayleigh-Ritz)
  subtract  PS, POLY, HFES, HFPS, HFPOLY subtraction vectors and the exact
            trace corrections
  estimate  the subtracted trace estimator, standard errors, relative
            efficiency
  gradient  d Tr / d kappa and d Tr / dU (adjoint form and dense check)

Parity status per function is stated in each module header.
"""
