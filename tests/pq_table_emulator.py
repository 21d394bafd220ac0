"""Numpy emulation of the HIP PQ residual driven by the generated tables.

It follows the kernel plan of paper_1609_00077_amd/derive/codegen.py step by
step (vertices, unpacked amplitudes, interpreted classes, R2S1 GEMMs, R2S2
vertex contraction) so that the tables can be checked against the oracle on
the CPU.  Slow; small N only.
"""
from math import comb

import numpy as np


def unpack_factor(code):
    kind = (code >> 28) & 0xF
    r = [(code >> 24) & 0xF, (code >> 20) & 0xF, (code >> 16) & 0xF]
    return kind, r, code & 0xFFFF


class Emu:
    def __init__(self, tb, N, f, eri, lane=False, mixed=True):
        self.tb, self.N, self.f, self.eri = tb, N, f, eri
        self.lane = lane          # evaluate the two-pair local terms through the lane tables
        self.mixed = mixed        # include the doubly-mixed two-spectator terms
        self.np2 = comb(N, 2)
        self.h1 = np.zeros((len(tb.h1_keys), N))
        self.h2 = np.zeros((len(tb.h2_keys), N, N))
        orb = lambda lab, x: lab[x // 2] + N * (x % 2)
        for i, ent in enumerate(tb.h1_sym):
            for P in range(N):
                v = 0.0
                for w, kind, a, b, _, _ in ent:
                    if kind == 0:
                        v += w * f[orb((P,), a), orb((P,), b)]
                    else:
                        v += w * eri[a * N + P]
                self.h1[i, P] = v
        for i, ent in enumerate(tb.h2_sym):
            for P in range(N):
                for Q in range(N):
                    if P == Q:
                        continue
                    v = 0.0
                    for w, kind, a, b, _, _ in ent:
                        if kind == 0:
                            v += w * f[orb((P, Q), a), orb((P, Q), b)]
                        else:
                            u = a if P < Q else b
                            lo, hi = min(P, Q), max(P, Q)
                            v += w * eri[6 * N + u * self.np2 + hi * (hi - 1) // 2 + lo]
                    self.h2[i, P, Q] = v

    def set_t(self, t):
        N, tb = self.N, self.tb
        self.t1 = t[:3 * N].reshape(3, N)
        self.t2 = np.zeros((29, N, N))
        for m in range(29):
            for Q in range(N):
                for P in range(Q):
                    v = t[3 * N + m * self.np2 + Q * (Q - 1) // 2 + P]
                    self.t2[m, P, Q] = v
                    self.t2[tb.swap2[m], Q, P] = tb.swap2_sign[m] * v

    def fval(self, code, lab, S=None):
        kind, r, idx = unpack_factor(code)
        if kind == 0:
            return 1.0
        if kind == 1:
            return self.t1[idx, lab[r[0]]]
        if kind == 2:
            return self.t2[idx, lab[r[0]], lab[r[1]]]
        if kind == 3:
            return self.h1[idx, lab[r[0]]]
        if kind == 4:
            return self.h2[idx, lab[r[0]], lab[r[1]]]
        if kind == 5:
            return S(idx)
        if kind == 6:
            return self.Wall[idx, lab[r[0]], lab[r[1]]]
        if kind == 7:
            return self.D[idx, lab[r[0]], lab[r[1]]]
        raise ValueError(kind)

    def interp(self, table, lab, S=None):
        nout = len(table.start) - 1
        out = np.zeros(nout)
        for m in range(nout):
            acc = 0.0
            for i in range(table.start[m], table.start[m + 1]):
                v = table.coef[i]
                for c in table.fac[i]:
                    if c == 0:
                        continue
                    v *= self.fval(int(c), lab, S)
                    if v == 0.0:
                        break
                acc += v
            out[m] = acc
        return out

    def spec(self, codes, lab):
        v = 1.0
        for c in codes:
            v *= self.fval(int(c), lab)
        return v

    def r2_lane_sum(self, P, Q, Spairs):
        """No- and one-spectator terms of the two-pair outputs through the
        lane tables (streamed factor x staged amplitudes of the pair)."""
        tb, N = self.tb, self.N
        V = tb.r2_lane
        loc = np.zeros(36)
        loc[0:3] = self.t1[:, P]
        loc[3:6] = self.t1[:, Q]
        loc[6:35] = self.t2[:, P, Q]
        loc[35] = 1.0
        # per chunk, one accumulator per output slot; then each output sums
        # its slots in the kernels' order
        slot = np.zeros(len(V["slot_m"]))
        for c in range(len(V["ch_lo"])):
            base = V["ch_slot0"][c]
            local = {m: base + j for j, m in enumerate(V["slot_m"][base:V["ch_slot0"][c + 1]])}
            for sg in range(V["ch_lo"][c], V["ch_hi"][c]):
                kind, idx = V["seg_kind"][sg], V["seg_idx"][sg]
                sv = (self.h1[idx, P] if kind == 0 else self.h1[idx, Q] if kind == 1
                      else self.h2[idx, P, Q] if kind == 2 else Spairs[idx, P, Q])
                for i in range(V["seg_lo"][sg], V["seg_hi"][sg]):
                    k = V["tidx"][4 * i: 4 * i + 4]
                    slot[local[V["term_m"][i]]] += sv * V["coef"][i] * loc[k[0]] * loc[k[1]] * loc[k[2]] * loc[k[3]]
        out = np.zeros(29)
        for m in range(29):
            for k in range(V["m_slot_start"][m], V["m_slot_start"][m + 1]):
                out[m] += slot[V["m_slots"][k]]
        return out

    def r1s2_factorised(self):
        """One-pair two-spectator terms through the X.Z.Y groups (amplitudes
        already set): M = G Mid per group, closed by each row of C."""
        tb, N = self.tb, self.N
        F = []
        for sp in tb.r1s2_x + tb.r1s2_y + tb.r1s2_z:
            Fm = np.zeros((N, N))
            for a in range(N):
                for b in range(N):
                    if a != b:
                        Fm[a, b] = self.spec(sp, (a, b))
            F.append(Fm)
        nx, ny, nz = len(tb.r1s2_x), len(tb.r1s2_y), len(tb.r1s2_z)
        out = np.zeros((3, N))
        for (zsel, side, gen), lst in tb.r1s2_groups:
            Z = F[nx + ny + zsel] if zsel < nz else F[nx + ny + zsel - nz].T
            G = F[gen] if side == 0 else F[nx + gen]
            M = G @ Z
            for cl, c, m in lst:
                C = F[nx + cl] if side == 0 else F[cl]
                out[m] += c * np.sum(M * C, axis=1)
        return out

    def residual(self, t):
        tb, N = self.tb, self.N
        self.set_t(t)
        R = np.zeros(3 * N + 29 * self.np2)
        C = tb.classes
        for P in range(N):
            acc = self.interp(C["R1S0"], (P,))
            for A in range(N):
                if A != P:
                    acc += self.interp(C["R1S1"], (P, A))
            for A in range(N):
                for B in range(N):
                    if len({P, A, B}) == 3:
                        acc += 0.5 * self.interp(C["R1S2"], (P, A, B))
            R[np.arange(3) * N + P] = acc
        # R2S2 vertices (and transposes), one-sided link products, dressed vertices
        W = np.zeros((len(tb.r2s2_w), N, N))
        for i, sp in enumerate(tb.r2s2_w):
            for A in range(N):
                for B in range(N):
                    if A != B:
                        W[i, A, B] = self.spec(sp, (A, B))
        self.Wall = np.concatenate([W, W.transpose(0, 2, 1)])
        lam = np.zeros((len(tb.r2s2_lam), N, N))
        for i, sp in enumerate(tb.r2s2_lam):
            for a in range(N):
                for b in range(N):
                    if a != b:
                        lam[i, a, b] = self.spec(sp, (a, b))
        self.D = np.zeros((len(tb.r2s2_dress), N, N))
        for k, (li, we) in enumerate(tb.r2s2_dress):
            L = np.ones((N, N)) if li < 0 else lam[li]
            self.D[k] = L @ self.Wall[we].T          # D(s, A) = sum_B L(s, B) W(A, B)
        # R2S1 intermediates
        X = np.zeros((len(tb.r2s1_x), N, N))
        Y = np.zeros((len(tb.r2s1_y), N, N))
        for i, sp in enumerate(tb.r2s1_x):
            for P in range(N):
                for A in range(N):
                    if P != A:
                        X[i, P, A] = self.spec(sp, (P, A))
        for i, sp in enumerate(tb.r2s1_y):
            for Q in range(N):
                for A in range(N):
                    if Q != A:
                        Y[i, Q, A] = self.spec(sp, (Q, A))
        Spairs = np.einsum("xpa,xqa->xpq", X[tb.r2s1_pairs[:, 0]], Y[tb.r2s1_pairs[:, 1]])
        for Q in range(N):
            for P in range(Q):
                if self.lane:
                    acc = self.r2_lane_sum(P, Q, Spairs)
                else:
                    acc = self.interp(C["R2S0"], (P, Q))
                    acc += self.interp(C["R2S1"], (P, Q), S=lambda i: Spairs[i, P, Q])
                specA = [A for A in range(N) if A not in (P, Q)]
                Lv = {}
                for li, sp in enumerate(tb.r2s2_l):
                    Lv[li] = np.array([self.spec(sp, (P, Q, A)) if A not in (P, Q) else 0.0
                                       for A in range(N)])
                Wall = self.Wall                                   # vertices nw + w: transposed
                for (wi, ai), lst in (tb.r2s2_groups if self.mixed else []):
                    V = Lv[ai] @ Wall[wi]       # V[B] = sum_A L_a(A) W(A,B) (or transposed)
                    for bi, c, m in lst:
                        acc[m] += c * np.dot(V, Lv[bi])
                R[3 * N + np.arange(29) * self.np2 + Q * (Q - 1) // 2 + P] = acc
        return R

    def energy(self, t):
        self.set_t(t)
        N = self.N
        e = 0.0
        for P in range(N):
            e += self.interp(self.tb.classes["E1"], (P,))[0]
            for Q in range(N):
                if Q != P:
                    e += 0.5 * self.interp(self.tb.classes["E2"], (P, Q))[0]
        return e
