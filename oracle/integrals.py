"""MO Fock matrix and pair-block two-electron integrals (oracle side).

Sec. III (RI/CD paragraph): the two-electron integrals are formed from three
index factors, (pq|rs) = sum_K B[K,pq] B[K,rs], which lets the program pick
only the elements it needs; here only the label sets of at most k pairs are
formed (Table I caption).  For a zero-differential-overlap site Hamiltonian
the factor is the product of MO coefficients on each site and the metric is
the site interaction matrix V:
    (pq|rs) = sum_{ij} C[i,p] C[i,q] V[i,j] C[j,r] C[j,s].
The Fock matrix is supplied by the SCF in the site basis and transformed,
f = C^T F C (Sec. III: Fock and B matrices come from the SCF program).
"""
from __future__ import annotations

from math import comb

import numpy as np

from . import layout


def mo_fock(F_site: np.ndarray, C: np.ndarray) -> np.ndarray:
    return C.T @ F_site @ C


def eri_dense_zdo(C: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Full (n^4) MO integrals of a ZDO site Hamiltonian (small n only)."""
    X = np.einsum("ip,iq->ipq", C, C)
    return np.einsum("ipq,ij,jrs->pqrs", X, V, X, optimize=True)


def eri_dense_from_b(B: np.ndarray) -> np.ndarray:
    return np.einsum("Kpq,Krs->pqrs", B, B, optimize=True)


def _packed_positions(npair: int, k: int):
    """For every packed slot: global (p, q, r, s)."""
    pos = np.zeros((layout.eri_count(npair, k), 4), dtype=np.int64)
    for size in range(1, k + 1):
        quads = layout.eri_quads(size)
        nsets = comb(npair, size)
        off = layout.eri_block_offset(npair, size)
        for labels in layout.label_sets(npair, size):
            si = layout.set_index(labels)
            for u, quad in enumerate(quads):
                pos[off + u * nsets + si] = [layout.local_to_global(labels, npair, x) for x in quad]
    return pos


def eri_packed_zdo(C: np.ndarray, V: np.ndarray, npair: int, k: int) -> np.ndarray:
    """Packed pair-block integrals computed element by element from the
    site-basis factors (valid at any size)."""
    n = C.shape[0]
    pos = _packed_positions(npair, k)
    X = np.einsum("ip,iq->ipq", C, C).reshape(n, n * n)
    Y = V @ X
    pq = pos[:, 0] * n + pos[:, 1]
    rs = pos[:, 2] * n + pos[:, 3]
    out = np.empty(len(pos))
    chunk = 1 << 16
    for a in range(0, len(pos), chunk):
        b = min(len(pos), a + chunk)
        out[a:b] = np.einsum("ix,ix->x", X[:, pq[a:b]], Y[:, rs[a:b]])
    return out


def eri_packed_from_b(B: np.ndarray, npair: int, k: int) -> np.ndarray:
    naux, n, _ = B.shape
    pos = _packed_positions(npair, k)
    Bf = B.reshape(naux, n * n)
    pq = pos[:, 0] * n + pos[:, 1]
    rs = pos[:, 2] * n + pos[:, 3]
    return np.einsum("Kx,Kx->x", Bf[:, pq], Bf[:, rs])


def chain_integrals(problem, k: int):
    """(f, packed eri) of a chain problem for the model with k-pair blocks."""
    f = mo_fock(problem.F_site, problem.C)
    eri = eri_packed_zdo(problem.C, problem.V, problem.npair, k)
    return f, eri
