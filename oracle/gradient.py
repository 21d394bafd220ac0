"""Energy gradient of the PQ/PH models through the Lagrangian (oracle side).

At converged amplitudes (R(t) = 0) the correlation energy is stationary in
the Lagrangian L = E_c(t) + sum_mu lambda_mu R_mu(t), with the de-excitation
amplitudes lambda solving J^T lambda = -dE/dt, J = dR/dt (Sec. II: lambda is
truncated like t; Table IV caption: t, lambda and the densities are solved
for).  The gradient with respect to any Hamiltonian parameter theta is then
dE/dtheta = dE_c/dtheta + lambda . dR/dtheta at fixed t.

Every derivative here is a complex-step derivative of the definitional
residual (exact to rounding, since R and E_c are polynomials in t and linear
in f and the integrals).  Parameters: f as a general 2N x 2N matrix and each
stored (unique) integral of the packed layout.  Small N only.
"""
from __future__ import annotations

import numpy as np

from . import layout
from .tier_a import TierA

H = 1e-30


def lagrangian_gradient(N: int, k: int, f: np.ndarray, eri_packed: np.ndarray, t: np.ndarray):
    """(dE/df [2N x 2N], dE/d(packed eri), lambda) at converged amplitudes t."""
    ta = TierA(N, k)
    eri_t = layout.unpack_eri(eri_packed, N, k)
    A = len(t)
    J = np.zeros((A, A))
    dEdt = np.zeros(A)
    for j in range(A):
        tc = t.astype(complex)
        tc[j] += 1j * H
        R, E = ta.residual(f.astype(complex), eri_t.astype(complex), tc)
        J[:, j] = R.imag / H
        dEdt[j] = E.imag / H
    lam = np.linalg.solve(J.T, -dEdt)
    n = 2 * N
    gf = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            fc = f.astype(complex)
            fc[p, q] += 1j * H
            R, E = ta.residual(fc, eri_t.astype(complex), t.astype(complex))
            gf[p, q] = (E.imag + lam @ R.imag) / H
    ge = np.zeros(len(eri_packed))
    for u in range(len(eri_packed)):
        ec = eri_packed.astype(complex)
        ec[u] += 1j * H
        R, E = ta.residual(f.astype(complex), layout.unpack_eri(ec, N, k), t.astype(complex))
        ge[u] = (E.imag + lam @ R.imag) / H
    return gf, ge, lam


def vjp(N: int, k: int, f: np.ndarray, eri_packed: np.ndarray, t: np.ndarray,
        lam: np.ndarray, energy_weight: float):
    """Gradient of phi = lam . R(t) + w E_c(t) with respect to t, f (general
    2N x 2N) and the packed integrals, at any t (converged or not): the
    transposed-residual contraction.  Complex-step derivatives."""
    ta = TierA(N, k)
    eri_t = layout.unpack_eri(eri_packed, N, k)

    def phi(fc, ec, tc):
        R, E = ta.residual(fc, ec, tc)
        return (lam @ R + energy_weight * E).imag / H

    fc0, ec0, tc0 = f.astype(complex), eri_t.astype(complex), t.astype(complex)
    tbar = np.zeros(len(t))
    for j in range(len(t)):
        tc = tc0.copy()
        tc[j] += 1j * H
        tbar[j] = phi(fc0, ec0, tc)
    n = 2 * N
    hbar = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            fc = fc0.copy()
            fc[p, q] += 1j * H
            hbar[p, q] = phi(fc, ec0, tc0)
    eribar = np.zeros(len(eri_packed))
    for u in range(len(eri_packed)):
        ec = eri_packed.astype(complex)
        ec[u] += 1j * H
        eribar[u] = phi(fc0, layout.unpack_eri(ec, N, k), tc0)
    return tbar, hbar, eribar


def directional_vjp_blocks(N: int, k: int, f, eri_packed, t, lam_blocks: dict,
                           energy_weight: float, dt, df, deri, keep_cache: bool = False) -> float:
    """d/ds [sum_mu lam_mu R_mu + w E_c] along (dt, df, deri), where lam is
    nonzero only on the slots of lam_blocks ({label tuple: {slot: value}}).
    Evaluated at any N by the sub-cluster sums (one complex step)."""
    from .tier_b import TierB
    tb = TierB(N, k, f + 1j * H * df, eri_packed + 1j * H * deri)
    tc = t + 1j * H * dt
    total = energy_weight * tb.energy(tc)
    for L, vals in lam_blocks.items():
        R = tb.residual_block(L, tc)
        total += sum(v * R[s] for s, v in vals.items())
        if not keep_cache:
            tb.clear()
    return float(np.imag(total) / H)


def densities(N: int, k: int, f: np.ndarray, eri_packed: np.ndarray, t: np.ndarray):
    """Unrelaxed response densities of the Lagrangian at converged t (Table IV
    caption: the densities follow the lambda solve; Sec. IV.B and Fig. 7 use
    the natural occupation numbers).

    gamma_pq = <E_pq> = 2 delta_pq [p occupied] + dE_c/df_pq (f multiplies the
    spin-summed E_pq in H; the reference part of the energy carries the
    2 delta_pq), Gamma = dE_c/d(packed eri), and the natural occupation
    numbers, the eigenvalues of (gamma + gamma^T)/2 in descending order.
    Returns (gamma, Gamma, noons)."""
    gf, ge, _ = lagrangian_gradient(N, k, f, eri_packed, t)
    gamma = gf.copy()
    gamma[np.arange(N), np.arange(N)] += 2.0
    noons = np.sort(np.linalg.eigvalsh(0.5 * (gamma + gamma.T)))[::-1]
    return gamma, ge, noons
