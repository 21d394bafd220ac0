"""Determinant strings and fermion operators for the definitional oracle.

A determinant of an n-pair system has 2n spatial orbitals (local orbital r is
o_r for r < n and v_{r-n} otherwise) and n electrons of each spin.  It is the
state (prod_{p in alpha, ascending} a+_{p alpha}) (prod_{p in beta, ascending}
a+_{p beta}) |vac>, stored as a pair of bit strings.  Vectors over the
determinant space are (n_strings x n_strings) arrays indexed [alpha, beta].
"""
from __future__ import annotations

from math import comb

import numpy as np

_POPC = np.array([bin(i).count("1") for i in range(1 << 16)], dtype=np.int64)


class StringSpace:
    """All bit strings with nel set bits among norb orbitals."""

    def __init__(self, norb: int, nel: int):
        if norb > 16:
            raise ValueError("string space limited to 16 orbitals")
        self.norb, self.nel = norb, nel
        allstr = np.arange(1 << norb, dtype=np.int64)
        self.strings = allstr[_POPC[allstr] == nel]
        self.lookup = np.full(1 << norb, -1, dtype=np.int64)
        self.lookup[self.strings] = np.arange(len(self.strings))
        assert len(self.strings) == comb(norb, nel)

    def __len__(self):
        return len(self.strings)

    def apply(self, ops):
        """Apply an operator product to every string.

        ops lists (is_creation, orbital) from left to right; the product acts
        right to left.  Returns (src, dst, sign) for the strings it does not
        annihilate; the sign counts occupied orbitals below each operator.
        """
        s = self.strings.copy()
        sign = np.ones(len(s))
        ok = np.ones(len(s), dtype=bool)
        for cre, p in reversed(list(ops)):
            bit = np.int64(1) << p
            occ = (s & bit) != 0
            odd = (_POPC[s & (bit - 1)] & 1).astype(bool)
            ok &= ~occ if cre else occ
            s = (s | bit) if cre else (s & ~bit)
            sign = np.where(odd, -sign, sign)
        src = np.flatnonzero(ok)
        dst = self.lookup[s[src]]
        assert (dst >= 0).all()
        return src, dst, sign[src]


def generator_ops(npair: int, role: int, pattern: int):
    """Operators of g_role^pattern (bit order 0..3) as (is_creation, orbital, spin)."""
    ops = []
    if pattern & 1:
        ops.append((False, role, 0))
    if pattern & 2:
        ops.append((False, role, 1))
    if pattern & 4:
        ops.append((True, npair + role, 0))
    if pattern & 8:
        ops.append((True, npair + role, 1))
    return ops


class SpinSplitOperator:
    """An operator product written as (sign) x (alpha part) (beta part).

    Moving every alpha operator to the left of every beta operator costs the
    sign of the interchanges; the beta part then passes the n alpha creators
    of the determinant, one factor (-1)^n per beta operator.
    """

    def __init__(self, space: StringSpace, ops):
        nswap = 0
        nbeta_seen = 0
        for _, _, spin in ops:
            if spin == 1:
                nbeta_seen += 1
            else:
                nswap += nbeta_seen
        alpha = [(c, p) for c, p, s in ops if s == 0]
        beta = [(c, p) for c, p, s in ops if s == 1]
        self.const = (-1.0) ** (nswap + space.nel * len(beta))
        self.sa, self.da, self.ga = space.apply(alpha)
        self.sb, self.db, self.gb = space.apply(beta)
        self.sign = self.const * np.outer(self.ga, self.gb)

    def apply_add(self, coef: float, vec: np.ndarray, out: np.ndarray):
        out[np.ix_(self.da, self.db)] += coef * self.sign * vec[np.ix_(self.sa, self.sb)]

    def image_of(self, ia: int, ib: int):
        """(sign, ia', ib') of one determinant, or None if annihilated."""
        wa = np.flatnonzero(self.sa == ia)
        wb = np.flatnonzero(self.sb == ib)
        if len(wa) == 0 or len(wb) == 0:
            return None
        return self.sign[wa[0], wb[0]], int(self.da[wa[0]]), int(self.db[wb[0]])
