"""Slow evaluator of the derived term lists (test infrastructure).

Sums every enumerated term of every output block and spectator class over
all label assignments, reading amplitudes from the packed layout with the
reordering sign of the pair operators.  Used only to check the derivation
against the oracle on small systems."""
import itertools, numpy as np
from math import comb
from paper_1609_00077_amd.derive import terms as T
from paper_1609_00077_amd.derive.algebra import hamiltonian_terms, pattern_tuples
from oracle import layout

def popc(e): return bin(e).count('1')

def amp(t, N, labels, pats):
    # coefficient of g_{l0}^{e0} g_{l1}^{e1}... in role order -> packed
    items = list(zip(labels, pats))
    if len(set(labels)) != len(labels): return 0.0
    sgn = 1
    # bubble sort by label with sign for odd-odd swaps
    items = list(items)
    for i in range(len(items)):
        for j in range(len(items)-1-i):
            if items[j][0] > items[j+1][0]:
                if popc(items[j][1]) % 2 and popc(items[j+1][1]) % 2: sgn = -sgn
                items[j], items[j+1] = items[j+1], items[j]
    ls = tuple(x[0] for x in items); ps = tuple(x[1] for x in items)
    m = pattern_tuples(len(ls)).index(ps)
    return sgn * t[layout.amp_slot(N, ls, m)]

def hval(f, eri, N, hroles, hkey, lab):
    coef = hamiltonian_terms(hroles, 2 if len(hroles)<=2 else 3)  # k only matters for v inclusion
    d = coef[hkey]
    def orb(x):
        role, typ = divmod(x, 2); return lab[role] + N*typ
    v = 0.0
    for sym, w in d.items():
        if sym[0] == 'f': v += w * f[orb(sym[1]), orb(sym[2])]
        else: v += w * eri[orb(sym[1]), orb(sym[2]), orb(sym[3]), orb(sym[4])]
    return v

def residual(k, N, f, eri, t):
    R = np.zeros(layout.amp_count(N, k))
    classes = {}
    for nout in range(1, k+1):
        for nspec in range(0, k+1):
            classes[nout, nspec] = T.merge_terms(T.enumerate_class(k, nout, nspec))
    for nout in range(1, k+1):
        for L in itertools.combinations(range(N), nout):
            others = [x for x in range(N) if x not in L]
            for nspec in range(0, k+1):
                fac = 1.0 / np.prod(range(1, nspec+1))
                for S in itertools.permutations(others, nspec):
                    lab = L + S
                    for tm in classes[nout, nspec]:
                        hv = hval(f, eri, N, tm.hroles, tm.hkey, lab)
                        if hv == 0.0: continue
                        p = tm.sign * hv * fac
                        for rho, pats in tm.slots:
                            p *= amp(t, N, tuple(lab[r] for r in rho), pats)
                            if p == 0.0: break
                        m = pattern_tuples(nout).index(tm.mu)
                        R[layout.amp_slot(N, L, m)] += p
    return R
