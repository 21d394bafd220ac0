"""Definitional residual and energy in the full determinant space (small N).

This tier derives no equations.  For a system of n pairs it builds, in the
space of all determinants with n electrons of each spin in 2n orbitals:

  * the Hamiltonian H_k of the model: the Fock matrix f kept whole and the
    two-electron integrals truncated to label sets of at most k pairs
    (Sec. II and Table I caption), written in bare form with the one-body
    matrix h~ = f - sum_{i occ} [2(pq|ii) - (pi|iq)] so that its
    normal-ordered one-body part is exactly f;
  * T = sum over the pair-truncated manifold of t_mu g^mu (Eq. (1) and its
    PH extension), g^mu as defined in the packed layout;
  * chi = e^{-T} (H_k - E_ref) e^{T} |0>;

and reads R_mu = <g^mu 0 | chi> for every slot and E_c = <0|chi>.
It also gives the full-CI ground state of the same Hamiltonian.
"""
from __future__ import annotations

import numpy as np

from . import layout
from .determinants import StringSpace, SpinSplitOperator, generator_ops


def truncate_eri(eri_full: np.ndarray, npair: int, k: int) -> np.ndarray:
    """Zero every (pq|rs) whose orbitals span more than k pairs."""
    n = 2 * npair
    lab = np.arange(n) % npair
    out = eri_full.copy()
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    if len({lab[p], lab[q], lab[r], lab[s]}) > k:
                        out[p, q, r, s] = 0.0
    return out


class TierA:
    """Determinant-space evaluator for an n-pair system and model k."""

    def __init__(self, npair: int, k: int):
        self.n, self.k = npair, k
        self.norb = 2 * npair
        self.space = StringSpace(self.norb, npair)
        ns = len(self.space)
        self.ref = int(self.space.lookup[(1 << npair) - 1])
        # one-particle excitation maps E_pq on strings (same for both spins)
        self.epq = {}
        for p in range(self.norb):
            for q in range(self.norb):
                self.epq[p, q] = self.space.apply([(True, p), (False, q)])
        # amplitude slots in packed order
        self.slots = []
        for pos, labels, tup in layout.iter_amp_slots(npair, k):
            ops = []
            for role, e in zip(labels, tup):
                ops += generator_ops(npair, role, e)
            op = SpinSplitOperator(self.space, ops)
            img = op.image_of(self.ref, self.ref)
            assert img is not None
            self.slots.append((pos, op, img))
        self.nslot = len(self.slots)
        self.shape = (ns, ns)

    # ------------------------------------------------------------ operators
    def _e(self, p, q, vec):
        src, dst, sg = self.epq[p, q]
        out = np.zeros_like(vec)
        out[dst, :] += sg[:, None] * vec[src, :]
        out[:, dst] += sg[None, :] * vec[:, src]
        return out

    def sigma(self, hmat: np.ndarray, eri: np.ndarray, vec: np.ndarray) -> np.ndarray:
        """H vec for H = sum h_pq E_pq + 1/2 sum (pq|rs) (E_pq E_rs - d_qr E_ps)."""
        n = self.norb
        D = np.stack([self._e(p, q, vec) for p in range(n) for q in range(n)])
        K = np.einsum("pqqs->ps", eri)
        heff = (hmat - 0.5 * K).reshape(-1)
        out = np.tensordot(heff, D, axes=1)
        G = np.tensordot(eri.reshape(n * n, n * n), D, axes=1)
        for p in range(n):
            for q in range(n):
                out += 0.5 * self._e(p, q, G[p * n + q])
        return out

    def bare_onebody(self, f: np.ndarray, eri: np.ndarray) -> np.ndarray:
        occ = range(self.n)
        J = sum(eri[:, :, i, i] for i in occ)
        Kx = sum(eri[:, i, i, :] for i in occ)
        return f - (2.0 * J - Kx)

    def apply_T(self, t: np.ndarray, vec: np.ndarray, scale: float = 1.0) -> np.ndarray:
        out = np.zeros_like(vec)
        for (pos, op, _), _unused in zip(self.slots, range(self.nslot)):
            tv = t[pos]
            if tv != 0.0:
                op.apply_add(scale * tv, vec, out)
        return out

    def exp_T(self, t: np.ndarray, vec: np.ndarray, sign: float = 1.0) -> np.ndarray:
        out = vec.copy()
        term = vec
        for m in range(1, 2 * self.n + 2):
            term = self.apply_T(t, term, sign / m)
            if not term.any():
                break
            out += term
        return out

    def reference(self, dtype=float) -> np.ndarray:
        v = np.zeros(self.shape, dtype=dtype)
        v[self.ref, self.ref] = 1.0
        return v

    # -------------------------------------------------------------- results
    def residual(self, f: np.ndarray, eri_trunc: np.ndarray, t: np.ndarray):
        """(R packed, E_c) at amplitudes t; eri_trunc is the dense truncated tensor."""
        hb = self.bare_onebody(f, eri_trunc)
        dt = np.result_type(f, eri_trunc, t)      # complex inputs allow complex-step derivatives
        ref = self.reference(dt)
        e_ref = self.sigma(hb, eri_trunc, ref)[self.ref, self.ref]
        psi = self.exp_T(t, ref, 1.0)
        phi = self.sigma(hb, eri_trunc, psi) - e_ref * psi
        chi = self.exp_T(t, phi, -1.0)
        R = np.zeros(layout.amp_count(self.n, self.k), dtype=dt)
        for pos, _, (sg, ia, ib) in self.slots:
            R[pos] = sg * chi[ia, ib]
        e = chi[self.ref, self.ref]
        return R, (e if np.iscomplexobj(e) else float(e))

    def jacobian(self, f, eri_trunc, t, h: float = 1e-30) -> np.ndarray:
        """J = dR/dt by complex-step derivatives (exact to rounding: R is a
        polynomial in t)."""
        fc, ec = f.astype(complex), eri_trunc.astype(complex)
        J = np.zeros((len(t), len(t)))
        for j in range(len(t)):
            tc = t.astype(complex)
            tc[j] += 1j * h
            J[:, j] = self.residual(fc, ec, tc)[0].imag / h
        return J

    def energy(self, f, eri_trunc, t) -> float:
        """E_c = <0| (H_k - E_ref) e^T |0>."""
        hb = self.bare_onebody(f, eri_trunc)
        ref = self.reference()
        e_ref = self.sigma(hb, eri_trunc, ref)[self.ref, self.ref]
        psi = self.exp_T(t, ref, 1.0)
        phi = self.sigma(hb, eri_trunc, psi)
        return float(phi[self.ref, self.ref] - e_ref)

    def reference_energy(self, f, eri_trunc) -> float:
        hb = self.bare_onebody(f, eri_trunc)
        ref = self.reference()
        return float(self.sigma(hb, eri_trunc, ref)[self.ref, self.ref])

    def fci(self, f, eri_full):
        """Lowest eigenvalue of the untruncated Hamiltonian minus E_ref."""
        hb = self.bare_onebody(f, eri_full)
        ns = self.shape[0] * self.shape[1]
        H = np.zeros((ns, ns))
        e = np.zeros(self.shape)
        for i in range(ns):
            e.flat[i] = 1.0
            H[:, i] = self.sigma(hb, eri_full, e).reshape(-1)
            e.flat[i] = 0.0
        w = np.linalg.eigvalsh(0.5 * (H + H.T))
        e_ref = H[self.ref * self.shape[1] + self.ref, self.ref * self.shape[1] + self.ref]
        return float(w[0] - e_ref), float(e_ref)
