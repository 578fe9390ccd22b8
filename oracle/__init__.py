"""Plain FP64 CPU oracle for incremental full configuration interaction (iFCI).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The device path does
not use it, and it uses nothing of the device path: it builds every
Hamiltonian matrix element from the original full-space integrals by the
Slater-Condon rules on explicit spin-orbital bit strings, diagonalises densely
with LAPACK (numpy.linalg.eigh) and sums the incremental expansion with
math.fsum.

What it computes (paper: Methods, "Incremental Full Configuration Interaction"):

* eq. 1: the correlation energy as a sum of one-, two-, three-, four-, ...
  body increments over groups of occupied orbitals ("bodies");
* eqs. 2-5: each increment is the correlation energy of the calculation that
  includes only those bodies, minus every increment of its proper non-empty
  subsets;
* the correlation energy of a calculation is its energy minus the energy of
  the single reference determinant (Methods, GVB-PP paragraph: the reference
  energy is the energy of one determinant in the localized orbital basis).

The paper solves each increment with selected CI (HBCI) in a truncated
natural-orbital space; the exact-FCI limit of that solver is computed here
(fci.py states how an increment restricted to some bodies is read here).

Modules:
  strings      one-spin occupation strings, combinatorial addresses, E_pq
  hamiltonian  Slater-Condon Hamiltonian (and an operator-algebra build)
  fci          increment determinant space, symmetric-sector eigensolve
  ifci         increments, weights, reference energy, eqs. 1-5
  rdm          one- and two-particle density matrices, iFCI gradient
  certify      matrix-free sigma rows and residual bounds for large spaces
"""
