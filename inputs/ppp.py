"""Pariser-Parr-Pople chains, closed-shell Hartree-Fock and mirror pairing.

The chain stands in for the pi space of the linear polyenes studied in the
paper (Sec. IV.B, Table VI: the active space is one orbital per carbon atom).
Recipe (fixed here, it is not from the paper):

* sites i = 0..n-1 at unit spacing, n even, half filling (n electrons);
* hopping h[i,i+1] = (-1.0 if i is even else -0.8) + eps_i, eps_i ~ U(-noise, noise)
  drawn in bond order from ``numpy.random.default_rng(seed)``; the chain starts
  and ends on a strong bond like a polyene;
* Ohno interaction V[i,j] = U / sqrt(1 + (i-j)^2), so V[i,i] = U;
* core-charge form: h[i,i] = -sum_{k != i} V[i,k] and E_core = sum_{i<j} V[i,j],
  so that H = sum h a+a + sum_i U n_iu n_id + sum_{i<j} V_ij (n_i - 1)(n_j - 1).

In the zero-differential-overlap site basis the two-electron integrals are
(ij|kl) = delta_ij delta_kl V[i,k].

The orbitals are paired in the mirror order of Fig. 1: pair P holds the
occupied orbital HOMO-P and the virtual orbital LUMO+P, P = 0..N-1.  The
paired MO matrix has columns [o_0 .. o_{N-1}, v_0 .. v_{N-1}].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def ppp_chain(n: int, U: float = 4.0, seed: int = 0, noise: float = 0.05,
              t_strong: float = -1.0, t_weak: float = -0.8):
    """Site-basis one-body matrix h, Ohno matrix V and core energy of a chain."""
    if n < 2 or n % 2:
        raise ValueError("the chain needs an even number of sites >= 2")
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-noise, noise, n - 1)
    h = np.zeros((n, n))
    for i in range(n - 1):
        hop = (t_strong if i % 2 == 0 else t_weak) + eps[i]
        h[i, i + 1] = h[i + 1, i] = hop
    r = np.abs(np.subtract.outer(np.arange(n), np.arange(n))).astype(float)
    V = U / np.sqrt(1.0 + r * r)
    offdiag = V.sum(axis=1) - np.diag(V)
    h[np.diag_indices(n)] = -offdiag
    E_core = float(np.triu(V, 1).sum())
    return h, V, E_core


def _fock(h, V, P):
    # F = h + J - K/2 in the ZDO site basis
    F = h + np.diag(V @ np.diag(P)) - 0.5 * V * P
    return F


def rhf(h, V, nocc: int, E_core: float = 0.0, tol: float = 1e-12,
        max_iter: int = 1000, diis_dim: int = 8, shift: float = 0.0):
    """Closed-shell RHF with DIIS, converged to max|FP - PF| <= tol.

    Returns (C, eps, F, P, E) with orbitals sorted by ascending energy.  If
    plain DIIS stalls, the solve is repeated with a virtual-space level shift
    (which changes the path, not the converged orbitals).
    """
    try:
        return _rhf(h, V, nocc, E_core, tol, 300 if shift == 0.0 else max_iter, diis_dim, shift)
    except RuntimeError:
        if shift != 0.0:
            raise
    for s in (0.5, 2.0):
        try:
            return _rhf(h, V, nocc, E_core, tol, max_iter, diis_dim, s)
        except RuntimeError:
            continue
    raise RuntimeError("RHF did not converge even with level shifts")


def _rhf(h, V, nocc, E_core, tol, max_iter, diis_dim, shift):
    n = h.shape[0]
    eps, C = np.linalg.eigh(h)          # Hueckel guess
    P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    focks, errs = [], []
    for it in range(max_iter):
        F = _fock(h, V, P)
        err = F @ P - P @ F
        errmax = float(np.abs(err).max())
        if errmax <= tol:
            break
        focks.append(F)
        errs.append(err)
        if len(focks) > diis_dim:
            focks.pop(0)
            errs.pop(0)
        m = len(focks)
        if m >= 2:
            B = -np.ones((m + 1, m + 1))
            B[m, m] = 0.0
            for i in range(m):
                for j in range(m):
                    B[i, j] = np.vdot(errs[i], errs[j])
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            try:
                c = np.linalg.solve(B, rhs)[:m]
                F = sum(ci * Fi for ci, Fi in zip(c, focks))
            except np.linalg.LinAlgError:
                pass
        if shift:
            F = F + shift * (np.eye(n) - 0.5 * P)
        eps, C = np.linalg.eigh(F)
        P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    else:
        raise RuntimeError(f"RHF did not converge (max|FP-PF| = {errmax:.3e})")
    F = _fock(h, V, P)
    eps, C = np.linalg.eigh(F)
    P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    F = _fock(h, V, P)
    E = 0.5 * float(np.sum(P * (h + F))) + E_core
    return C, eps, F, P, E


def mirror_pairing(C, eps, nocc: int):
    """Reorder MOs into [o_0..o_{N-1}, v_0..v_{N-1}] with o_P = HOMO-P, v_P = LUMO+P.

    The active space is all orbitals, so the number of virtuals must equal
    nocc.  Each column's sign is fixed so that its largest-magnitude
    component is positive (ties: the lowest site index decides).
    """
    n = C.shape[0]
    if n != 2 * nocc:
        raise ValueError("mirror pairing needs as many virtuals as occupied orbitals")
    order = [nocc - 1 - P for P in range(nocc)] + [nocc + P for P in range(nocc)]
    Cp = C[:, order].copy()
    ep = np.asarray(eps)[order].copy()
    for k in range(n):
        col = Cp[:, k]
        a = np.abs(col)
        i = int(np.flatnonzero(a >= a.max() - 1e-12)[0])
        if col[i] < 0:
            Cp[:, k] = -col
    return Cp, ep


@dataclass
class ChainProblem:
    n_sites: int
    U: float
    seed: int
    h_site: np.ndarray
    V: np.ndarray
    E_core: float
    C: np.ndarray          # paired MO coefficients, columns [o_0..o_{N-1}, v_0..v_{N-1}]
    eps: np.ndarray        # orbital energies in paired order
    F_site: np.ndarray     # converged Fock matrix in the site basis
    E_rhf: float

    @property
    def npair(self) -> int:
        return self.n_sites // 2


def chain_problem(n_sites: int, U: float = 4.0, seed: int = 0,
                  noise: float = 0.05) -> ChainProblem:
    """Chain Hamiltonian plus paired RHF orbitals, the input of every solve."""
    h, V, E_core = ppp_chain(n_sites, U=U, seed=seed, noise=noise)
    nocc = n_sites // 2
    C, eps, F, _, E = rhf(h, V, nocc, E_core=E_core)
    Cp, ep = mirror_pairing(C, eps, nocc)
    return ChainProblem(n_sites, U, seed, h, V, E_core, Cp, ep, F, E)


def _problem_of(spec):
    n, U, seed = spec
    return chain_problem(n, U=U, seed=seed)


def _single_thread_blas():
    from threadpoolctl import threadpool_limits
    global _LIMIT
    _LIMIT = threadpool_limits(limits=1)


def batch_problems(specs, processes: int = 8):
    """chain_problem for every (n_sites, U, seed) spec, in a process pool of
    single-threaded workers (a threaded BLAS per worker would oversubscribe)."""
    import multiprocessing as mp
    if processes <= 1 or len(specs) < 4:
        return [_problem_of(s) for s in specs]
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_single_thread_blas) as pool:
        return pool.map(_problem_of, specs, chunksize=2)
