"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the PQ/PH method itself.  It builds the
model Hamiltonian that stands in for the paper's polyene pi systems (a
Pariser-Parr-Pople chain), solves the closed-shell Hartree-Fock problem that
supplies the orbitals (the paper takes its orbitals from external SCF programs,
Sec. III, RI/CD paragraph), pairs the orbitals in the mirror order of Fig. 1,
and draws seeded random amplitudes and integral factors.  The integral
transformation into pair blocks, the residuals, energies, solves and gradients
are computed separately by the oracle and by the HIP library.
"""
from .ppp import (ppp_chain, rhf, mirror_pairing, chain_problem, ChainProblem,  # noqa: F401
                  batch_problems)
from .random_inputs import (  # noqa: F401
    random_amplitudes, random_vector, random_fock, random_bfactors, batch_chain_specs,
    n_amp_pq, n_amp_ph, n_eri_pq, n_eri_ph,
)
