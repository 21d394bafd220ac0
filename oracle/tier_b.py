"""Residual and energy at any size by sub-cluster inclusion-exclusion.

Every term of H_k acts on at most k pairs, and T only excites.  In
<mu| e^{-T} H_k e^{T} |0> a term h contributes only through amplitudes whose
pairs lie in X = labels(mu) U labels(h): amplitudes touching other pairs leave
those pairs excited, and nothing but h can return them to the reference.  So
with R^{(Y)} the residual of the sub-system made of the pairs Y alone (same f,
v and t restricted to Y, evaluated by the definitional tier),

  R_mu = sum_{X >= labels(mu), |X| <= |labels(mu)| + k} dR^{(X)}_mu,
  dR^{(X)} = sum_{labels(mu) <= Y <= X} (-1)^{|X|-|Y|} R^{(Y)}            (Moebius)

and likewise E_c = sum_{|X| <= k} dE^{(X)} (only h acts on the reference).
Each dR^{(X)} is the part connected across exactly the pairs X, so the sum
over X stays well conditioned.  Cost: one small definitional evaluation per
sub-cluster, so any single output block is available at any N.
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np

from . import layout
from .tier_a import TierA


class TierB:
    def __init__(self, npair: int, k: int, f: np.ndarray, eri_packed: np.ndarray):
        self.N, self.k = npair, k
        self.f = f
        self.eri = eri_packed
        self._engines = {}
        self._cache = {}

    def engine(self, n: int) -> TierA:
        if n not in self._engines:
            self._engines[n] = TierA(n, self.k)
        return self._engines[n]

    # ------------------------------------------------------------ sub-systems
    def sub_inputs(self, Y, t):
        """f, dense truncated integrals and amplitudes of the pairs Y."""
        N, k = self.N, self.k
        n = len(Y)
        orbs = list(Y) + [N + y for y in Y]
        f_sub = self.f[np.ix_(orbs, orbs)]
        dt = np.result_type(self.f, self.eri, t if t is not None else 0.0)
        sub_eri = np.zeros(layout.eri_count(n, k), dtype=dt)
        for size in range(1, min(k, n) + 1):
            quads = layout.eri_quads(size)
            goff = layout.eri_block_offset(N, size)
            gsets = comb(N, size)
            loff = layout.eri_block_offset(n, size)
            lsets = comb(n, size)
            for loc in itertools.combinations(range(n), size):
                glob = tuple(Y[i] for i in loc)
                gi = layout.set_index(glob)
                li = layout.set_index(loc)
                for u in range(len(quads)):
                    sub_eri[loff + u * lsets + li] = self.eri[goff + u * gsets + gi]
        eri_sub = layout.unpack_eri(sub_eri, n, k)
        t_sub = np.zeros(layout.amp_count(n, k), dtype=dt)
        gmap = np.zeros(layout.amp_count(n, k), dtype=np.int64)
        for pos, loc, tup in layout.iter_amp_slots(n, k):
            m = layout.pattern_tuples(len(loc)).index(tup)
            g = layout.amp_slot(N, tuple(Y[i] for i in loc), m)
            gmap[pos] = g
            if t is not None:
                t_sub[pos] = t[g]
        return f_sub, eri_sub, t_sub, gmap

    def sub_residual(self, Y, t):
        """(R^{(Y)} keyed by global slot, E^{(Y)}) with caching per Y."""
        key = tuple(Y)
        if key not in self._cache:
            f_sub, eri_sub, t_sub, gmap = self.sub_inputs(key, t)
            R, E = self.engine(len(key)).residual(f_sub, eri_sub, t_sub)
            self._cache[key] = (dict(zip(gmap.tolist(), R.tolist())), E)
        return self._cache[key]

    def clear(self):
        self._cache.clear()

    # ---------------------------------------------------------------- results
    def prefetch(self, subs, t, workers: int):
        """Evaluate the sub-systems subs (sorted tuples) over a process pool into
        the cache; the sums below then read them from there."""
        todo = [Y for Y in subs if Y not in self._cache]
        global _POOL_STATE
        _POOL_STATE = (self, t)
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            for Y, (gmap, RY, _, E) in zip(todo, pool.imap(_sub_residual_arrays, todo, chunksize=4)):
                self._cache[Y] = (dict(zip(gmap.tolist(), RY.tolist())), E)

    def residual_block(self, L, t, workers: int = 1):
        """R for every slot whose label set is exactly L (sorted tuple).

        Returns {global slot: value}.
        """
        L = tuple(sorted(L))
        N, k = self.N, self.k
        others = [x for x in range(N) if x not in L]
        if workers > 1:
            self.prefetch([tuple(sorted(L + add)) for extra in range(k + 1)
                           for add in itertools.combinations(others, extra)], t, workers)
        slots = [layout.amp_slot(N, L, m) for m in range(len(layout.pattern_tuples(len(L))))]
        total = {s: 0 for s in slots}
        for extra in range(0, k + 1):
            for add in itertools.combinations(others, extra):
                # dR^{(X)} for X = L + add
                d = {s: 0 for s in slots}
                for j in range(extra + 1):
                    for sub in itertools.combinations(add, j):
                        Y = tuple(sorted(L + sub))
                        RY, _ = self.sub_residual(Y, t)
                        sg = (-1.0) ** (extra - j)
                        for s in slots:
                            d[s] += sg * RY[s]
                for s in slots:
                    total[s] += d[s]
        return total

    def energy(self, t) -> float:
        N, k = self.N, self.k
        total = 0.0
        for size in range(1, k + 1):
            for X in itertools.combinations(range(N), size):
                d = 0.0
                for j in range(1, size + 1):
                    for Y in itertools.combinations(X, j):
                        d += (-1.0) ** (size - j) * self.sub_residual(Y, t)[1]
                total += d
        return total

    def mobius_weight(self, nlab: int, nsub: int) -> int:
        """sum over X >= Y, |X| <= nlab + k, of (-1)^{|X|-|Y|} for |Y| = nsub:
        the coefficient with which R^{(Y)} enters every output block on a
        label set L <= Y of size nlab once the two sums above are swapped."""
        return sum((-1) ** m * comb(self.N - nsub, m) for m in range(nlab + self.k - nsub + 1))

    def residual_all(self, t, workers: int = 1):
        """The full packed residual with every sub-system evaluated once.

        Swapping the sums of residual_block gives R_mu = sum over Y >= labels(mu),
        |Y| <= |labels(mu)| + k, of mobius_weight(|labels(mu)|, |Y|) R^{(Y)}_mu.
        The sub-systems (all label sets of at most 2k pairs) are independent, so
        they are spread over a process pool."""
        N, k = self.N, self.k
        subs = [Y for n in range(1, min(N, 2 * k) + 1) for Y in itertools.combinations(range(N), n)]
        R = np.zeros(layout.amp_count(N, k), dtype=np.result_type(self.f, self.eri, t))
        global _POOL_STATE
        _POOL_STATE = (self, t)
        if workers > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                parts = pool.imap(_sub_residual_arrays, subs, chunksize=16)
                self._accumulate(R, subs, parts)
        else:
            self._accumulate(R, subs, map(_sub_residual_arrays, subs))
        return R

    def _accumulate(self, R, subs, parts):
        for Y, (gmap, RY, nlab, _) in zip(subs, parts):
            for size in range(1, self.k + 1):
                if len(Y) - size > self.k:
                    continue
                w = self.mobius_weight(size, len(Y))
                sel = nlab == size
                np.add.at(R, gmap[sel], w * RY[sel])

    def residual(self, t):
        """The full packed residual (only for small N: every block is evaluated)."""
        R = np.zeros(layout.amp_count(self.N, self.k), dtype=np.result_type(self.f, self.eri, t))
        for size in range(1, self.k + 1):
            for L in itertools.combinations(range(self.N), size):
                for s, v in self.residual_block(L, t).items():
                    R[s] = v
        return R


_POOL_STATE = None


def _sub_residual_arrays(Y):
    """(global slots, R^{(Y)} on them, label-set size of each slot, E^{(Y)}) of
    one sub-system."""
    tb, t = _POOL_STATE
    f_sub, eri_sub, t_sub, gmap = tb.sub_inputs(tuple(Y), t)
    R, E = tb.engine(len(Y)).residual(f_sub, eri_sub, t_sub)
    nlab = np.array([len(loc) for _, loc, _ in layout.iter_amp_slots(len(Y), tb.k)])
    return gmap, R, nlab, E
