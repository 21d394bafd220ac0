"""FP64 CPU oracle for the PQ/PH pair-truncated coupled-cluster path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code, headers, tables or helpers with the
HIP library; the only common dependency is the seeded input generator in
``inputs`` (which holds none of the method's arithmetic).

What it computes (Sec. II of the paper, Theory):

* the model: amplitudes t_mu for every excitation mu from the closed-shell
  reference whose orbitals lie in at most k pairs (k = 2: perfect quadruples,
  PQ; k = 3: perfect hextuples, PH), Sec. II and the amplitude decomposition
  of Eq. (1); the two-electron integrals are truncated to label sets of at
  most k pairs (Table I caption), the Fock matrix f is kept whole;
* the projected residual R_mu = <mu| e^{-T} H_k e^{T} |0> and the correlation
  energy E_c = <0| H_k e^{T} |0> - E_ref (Eqs. (2)-(3) give the doubles part
  of that energy in subtensor form);
* Jacobi updates with orbital-energy denominators and DIIS (Sec. III and the
  "denominator application" line of Table IV);
* the energy gradient with respect to f and the pair-block integrals through
  the Lagrangian with de-excitation amplitudes lambda (Sec. II: lambda, gamma
  and Gamma are truncated like t).

Modules:
  layout       packed amplitude / integral layouts (as declared in include/pqph.h)
  integrals    MO Fock matrix and pair-block integrals from the site basis
  determinants determinant strings and fermion operators
  tier_a       definitional residual/energy in the full determinant space
  tier_b       the same quantities at any size by sub-cluster inclusion-exclusion
  solver       Jacobi + DIIS amplitude solver on top of either tier
  gradient     energy gradient by the Lagrangian (lambda) route
"""
