"""Enumeration of the residual terms of one output block and spectator class.

An output block is the set of residual components on a label set L (roles
0..|L|-1); a spectator class adds roles |L|..|L|+s-1 that every term must
touch through the Hamiltonian and close completely (no open lines).  A term
is sign * c_h * prod_i t(slot_i) contributing to one output pattern tuple.
Summing a class over spectator labels (all distinct, unordered) and over the
classes with 0..k spectators gives the residual (Sec. II: every term of H_k
acts on at most k pairs, so at most k spectators appear).
"""
from __future__ import annotations

import itertools
from collections import namedtuple

from .algebra import (derive_monomial, hamiltonian_terms, partition_products,
                      pattern_tuples, slot_monomial, sort_sign)

Term = namedtuple("Term", "mu sign hroles hkey slots")
# mu: output pattern tuple (one pattern per output role)
# sign: +-1
# hroles: tuple of roles of the Hamiltonian term; hkey: (I, J)
# slots: tuple of (roles, patterns) amplitude factors


def all_slots(roles, k):
    out = []
    for size in range(1, k + 1):
        for rho in itertools.combinations(sorted(roles), size):
            for pats in pattern_tuples(size):
                out.append((rho, pats, slot_monomial(rho, pats)))
    return out


def _mask(gens):
    m = 0
    for g in gens:
        m |= 1 << g
    return m


def _disjoint_products(cands, I):
    """The combinations of itertools.product(*cands), in the same order,
    whose remaining generators repeat neither each other nor those of I; the
    others multiply to zero (a generator squares to zero), so skipping them
    early changes no term."""
    masks = [[_mask(c[3]) for c in cl] for cl in cands]
    out = []
    pick = [None] * len(cands)

    def rec(i, used):
        if i == len(cands):
            out.append(tuple(pick))
            return
        for c, m in zip(cands[i], masks[i]):
            if used & m:
                continue
            pick[i] = c
            rec(i + 1, used | m)

    i0 = _mask(I)
    if len(set(I)) == len(I):
        rec(0, i0)
    return out


def enumerate_class(k: int, nout: int, nspec: int, energy: bool = False, only_hroles=None,
                    part=(0, 1)):
    """All terms of the output block with roles 0..nout-1 and spectators
    nout..nout+nspec-1.  With energy=True (nout=0) it gives E_c terms.
    only_hroles restricts the Hamiltonian term to those role sets and
    part = (i, n) to every n-th of their terms from the i-th, so that the
    enumeration can run in pieces."""
    out_roles = tuple(range(nout))
    spec_roles = tuple(range(nout, nout + nspec))
    allroles = out_roles + spec_roles
    out_set, spec_set = set(out_roles), set(spec_roles)
    slots = all_slots(allroles, k)
    terms = []
    for hsize in range(1, k + 1):
        for hroles in itertools.combinations(allroles, hsize):
            if not spec_set <= set(hroles):
                continue
            if only_hroles is not None and hroles not in only_hroles:
                continue
            for ih, ((I, J), _coef) in enumerate(hamiltonian_terms(hroles, k).items()):
                if ih % part[1] != part[0]:
                    continue
                if any(g // 4 in spec_set for g in I):
                    continue
                for psign, blocks in partition_products(J):
                    cands = []
                    for K in blocks:
                        c = []
                        for rho, pats, mono in slots:
                            s, rem = derive_monomial(K, mono)
                            if s == 0 or any(g // 4 in spec_set for g in rem):
                                continue
                            c.append((rho, pats, s, rem))
                        if not c:
                            break
                        cands.append(c)
                    else:
                        for combo in _disjoint_products(cands, I):
                            seq = list(I)
                            sg = psign
                            for _, _, s, rem in combo:
                                seq += rem
                                sg *= s
                            s2, mu = sort_sign(seq)
                            if s2 == 0:
                                continue
                            if {g // 4 for g in mu} != out_set:
                                continue
                            pats = []
                            for r in out_roles:
                                e = 0
                                for g in mu:
                                    if g // 4 == r:
                                        e |= 1 << (g % 4)
                                pats.append(e)
                            terms.append(Term(tuple(pats), sg * s2, hroles, (I, J),
                                              tuple((rho, p) for rho, p, _, _ in combo)))
    return terms


def merge_terms(terms):
    """Combine terms that differ only in the order of their amplitude factors."""
    acc = {}
    for t in terms:
        key = (t.mu, t.hroles, t.hkey, tuple(sorted(t.slots)))
        acc[key] = acc.get(key, 0) + t.sign
    return [Term(mu, s, hr, hk, sl) for (mu, hr, hk, sl), s in acc.items() if s != 0]
