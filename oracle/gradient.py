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
