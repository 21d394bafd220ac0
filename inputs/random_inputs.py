"""Seeded random amplitudes, Fock matrices and integral factors.

Only random numbers and sizes live here.  The amplitude vector length follows
the packed layout declared in include/pqph.h: 3 single-pair entries per pair,
29 entries per pair of pairs and 303 per triple of pairs (Table II counts the
same amplitudes by subtensor; 3/29/303 are the unique excitations per label
set).
"""
from __future__ import annotations

from math import comb

import numpy as np


def n_amp_pq(npair: int) -> int:
    return 3 * npair + 29 * comb(npair, 2)


def n_amp_ph(npair: int) -> int:
    return n_amp_pq(npair) + 303 * comb(npair, 3)


def n_eri_pq(npair: int) -> int:
    return 6 * npair + 43 * comb(npair, 2)


def n_eri_ph(npair: int) -> int:
    return n_eri_pq(npair) + 84 * comb(npair, 3)


def random_amplitudes(npair: int, model: str = "pq", seed: int = 0,
                      scale: float = 0.1) -> np.ndarray:
    """Uniform(-scale, scale) values for every packed amplitude slot."""
    n = n_amp_pq(npair) if model == "pq" else n_amp_ph(npair)
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, n)


def random_vector(n: int, seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Uniform(-scale, scale) values of length n (test directions, multipliers)."""
    return np.random.default_rng(seed).uniform(-scale, scale, n)


def random_fock(npair: int, seed: int = 0, offdiag: float = 0.1) -> np.ndarray:
    """Symmetric 2N x 2N one-body matrix in the paired orbital order.

    Occupied diagonal entries lie in [-1.5, -1], virtual ones in [1, 1.5], so
    every orbital-energy denominator is bounded away from zero.
    """
    rng = np.random.default_rng(seed)
    n = 2 * npair
    A = rng.uniform(-offdiag, offdiag, (n, n))
    f = 0.5 * (A + A.T)
    d = np.concatenate([-1.0 - 0.5 * rng.random(npair), 1.0 + 0.5 * rng.random(npair)])
    f[np.diag_indices(n)] = d
    return f


def random_bfactors(npair: int, naux: int | None = None, seed: int = 0,
                    scale: float = 0.3) -> np.ndarray:
    """Random three-index factors B[K, p, q], symmetric in p, q.

    (pq|rs) = sum_K B[K,p,q] B[K,r,s] then has the full 8-fold symmetry of
    real two-electron integrals (the RI/CD form of Sec. III).
    """
    n = 2 * npair
    naux = naux or n
    rng = np.random.default_rng(seed)
    B = rng.normal(0.0, scale, (naux, n, n))
    return 0.5 * (B + B.transpose(0, 2, 1))


def batch_chain_specs(nbatch: int = 256, seed: int = 256, nmin: int = 10,
                      nmax: int = 120, umin: float = 2.0, umax: float = 6.0):
    """(n_sites, U, chain_seed) for a batch of chains of uneven pair counts."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(nbatch):
        npair = int(rng.integers(nmin, nmax + 1))
        U = float(rng.uniform(umin, umax))
        cseed = int(rng.integers(0, 2**31 - 1))
        specs.append((2 * npair, U, cseed))
    return specs
