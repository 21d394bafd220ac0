"""Jacobi + DIIS amplitude solver (Sec. III: DIIS accelerates the CC
amplitudes; Table IV: denominator application).

Update t <- t - R/D with D_mu = sum of f_aa over the particles of mu minus the
sum of f_ii over its holes (optionally plus a level shift); DIIS (Pulay)
extrapolates the amplitudes from the last m iterates with error vectors
Delta t = -R/D, starting once two iterates exist.  The iteration stops when
the 2-norm of R over the packed (unique) amplitudes is at most tol.

An excitation-rank limit (Sec. V: PH with only singles and doubles, or up to
quadruples) keeps t = 0 on the excitations of more than max_rank holes and
solves R = 0 on the others only.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import layout


def denominators(f: np.ndarray, npair: int, k: int, shift: float = 0.0) -> np.ndarray:
    D = np.zeros(layout.amp_count(npair, k))
    for pos, labels, tup in layout.iter_amp_slots(npair, k):
        d = 0.0
        for P, e in zip(labels, tup):
            if e & 1:
                d -= f[P, P]
            if e & 2:
                d -= f[P, P]
            if e & 4:
                d += f[npair + P, npair + P]
            if e & 8:
                d += f[npair + P, npair + P]
        D[pos] = d + shift
    return D


def slot_ranks(npair: int, k: int) -> np.ndarray:
    """Number of holes (occupied spin orbitals removed) of every packed slot."""
    rk = np.zeros(layout.amp_count(npair, k), dtype=np.int64)
    for pos, _, tup in layout.iter_amp_slots(npair, k):
        rk[pos] = sum(bin(e & 3).count("1") for e in tup)
    return rk


@dataclass
class SolveResult:
    t: np.ndarray
    energy: float
    rnorm: float
    iterations: int
    converged: bool
    history: list = field(default_factory=list)


def solve(residual_fn, energy_fn, D: np.ndarray, t0: np.ndarray | None = None,
          tol: float = 1e-10, max_iter: int = 200, diis_dim: int = 8,
          diis_start: int = 2, keep: np.ndarray | None = None) -> SolveResult:
    """residual_fn(t) -> R; energy_fn(t) -> E_c.  keep (boolean per slot, or
    None for all): the slots that are solved for; the others stay zero."""
    t = np.zeros_like(D) if t0 is None else t0.copy()
    if keep is not None:
        t[~keep] = 0.0
    ts, es, hist = [], [], []
    for it in range(1, max_iter + 1):
        R = residual_fn(t)
        if keep is not None:
            R = np.where(keep, R, 0.0)
        rn = float(np.linalg.norm(R))
        hist.append(rn)
        if not np.isfinite(rn):
            return SolveResult(t, float("nan"), rn, it, False, hist)
        if rn <= tol:
            return SolveResult(t, energy_fn(t), rn, it, True, hist)
        dt = -R / D
        tn = t + dt
        ts.append(tn)
        es.append(dt)
        if len(ts) > diis_dim:
            ts.pop(0)
            es.pop(0)
        m = len(ts)
        if it >= diis_start and m >= 2:
            B = np.empty((m + 1, m + 1))
            B[:m, :m] = np.array([[np.dot(a, b) for b in es] for a in es])
            B[m, :m] = B[:m, m] = -1.0
            B[m, m] = 0.0
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            try:
                c = np.linalg.solve(B, rhs)[:m]
                tn = sum(ci * ti for ci, ti in zip(c, ts))
            except np.linalg.LinAlgError:
                pass
        t = tn
    R = residual_fn(t)
    if keep is not None:
        R = np.where(keep, R, 0.0)
    return SolveResult(t, energy_fn(t), float(np.linalg.norm(R)), max_iter, False, hist)


def newton(residual_fn, jacobian_fn, energy_fn, t0: np.ndarray, tol: float = 1e-10,
           max_steps: int = 50) -> SolveResult:
    """Newton's method on R(t) = 0 with the dense Jacobian J = dR/dt (small
    systems), backtracking the step until ||R|| decreases.  The same fixed
    point as the Jacobi/DIIS iteration, reached where that iteration stalls or
    diverges (Sec. IV.B)."""
    t = t0.copy()
    hist = []
    for it in range(1, max_steps + 1):
        R = residual_fn(t)
        rn = float(np.linalg.norm(R))
        hist.append(rn)
        if not np.isfinite(rn):
            return SolveResult(t, float("nan"), rn, it, False, hist)
        if rn <= tol:
            return SolveResult(t, energy_fn(t), rn, it, True, hist)
        dt = np.linalg.solve(jacobian_fn(t), -R)
        lam = 1.0
        while lam > 1e-4:
            tn = t + lam * dt
            if np.linalg.norm(residual_fn(tn)) < (1.0 - 1e-4 * lam) * rn:
                break
            lam *= 0.5
        t = tn
    R = residual_fn(t)
    return SolveResult(t, energy_fn(t), float(np.linalg.norm(R)), max_steps, False, hist)
