"""The PH term-table file (written by the package's PH table generator and
read by the HIP library) against the FP64 oracle, on the CPU.

The file is decoded here independently of the library and its terms are
summed over label assignments exactly as the file's format states; on small
systems the sums must equal the definitional PH residual and energy (Tier A,
k = 3).  This pins the encoding (slot codes, Hamiltonian symbols, pattern
and integral maps) before any kernel reads it."""
import itertools
import os
import struct
import zlib
from math import comb, factorial

import numpy as np
import pytest

from inputs import random_amplitudes, random_bfactors, random_fock
from oracle import integrals as oint
from oracle import layout, tier_a

PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_1609_00077_amd", "ph_terms.bin")

pytestmark = pytest.mark.skipif(not os.path.exists(PATH), reason="PH term tables not generated")


class Tables:
    def __init__(self, path):
        with open(path, "rb") as fh:
            data = fh.read()
        magic, n = struct.unpack("<iq", data[:12])      # zlib container
        assert magic == 0x315A4850
        data = zlib.decompress(data[12:])
        assert len(data) == n
        pos = 0

        def take(n, dtype="<i4"):
            nonlocal pos
            size = np.dtype(dtype).itemsize * n
            out = np.frombuffer(data, dtype=dtype, count=n, offset=pos)
            pos += size + (-size % 4)          # sections are padded to 4 bytes
            return out

        magic, ver, nclass, nh, nsym, nterm, ncw, nslot = (int(x) for x in take(8))
        assert magic == 0x31485450 and ver == 3
        self.classes = []
        for _ in range(nclass):
            nout, nspec, nt, off, npat = (int(x) for x in take(5))
            start = take(npat + 1)
            self.classes.append((nout, nspec, nt, off, npat, start))
        cw_dict = take(ncw)
        slot_dict = take(nslot)
        h = take(nterm, "<u2")
        cw = cw_dict[take(nterm, "<u1")]
        slots = slot_dict[take(4 * nterm, "<u2").reshape(4, nterm)]
        self.terms = np.stack([h.astype(np.int64), cw] + [slots[i] for i in range(4)], axis=1)
        self.hstart = take(nh + 1)
        self.sym_w = take(nsym, "<f8")
        self.sym_code = take(nsym)
        self.pat2m = take(16 + 256 + 4096)
        self.m2pat = take(3 + 29 + 303)
        self.canon = take(3 + 29 + 303)
        self.quad = take(3 * 1296)
        assert pos == len(data)


@pytest.fixture(scope="module")
def tb():
    return Tables(PATH)


def _amp(tb, t, N, lab, code):
    n = code & 3
    items = [(lab[(code >> (2 + 3 * i)) & 7], (code >> (11 + 4 * i)) & 15) for i in range(n)]
    sg = 1.0
    for i in range(n):                       # bubble sort, odd-odd swaps flip the sign
        for j in range(n - 1 - i):
            if items[j][0] > items[j + 1][0]:
                if bin(items[j][1]).count("1") % 2 and bin(items[j + 1][1]).count("1") % 2:
                    sg = -sg
                items[j], items[j + 1] = items[j + 1], items[j]
    packed = sum(p << (4 * i) for i, (_, p) in enumerate(items))
    m = tb.pat2m[(0, 16, 272)[n - 1] + packed]
    assert m >= 0
    labels = tuple(x for x, _ in items)
    return sg * t[layout.amp_slot(N, labels, int(m))]


def _h(tb, f, eri, N, lab, hidx):
    v = 0.0
    for j in range(tb.hstart[hidx], tb.hstart[hidx + 1]):
        c = int(tb.sym_code[j])
        x = [(c >> (4 + 4 * i)) & 15 for i in range(4)]
        if c & 15 == 0:
            o = [lab[y >> 1] + N * (y & 1) for y in x[:2]]
            v += tb.sym_w[j] * f[o[0], o[1]]
            continue
        labels = sorted({lab[y >> 1] for y in x})
        loc = [2 * labels.index(lab[y >> 1]) + (y & 1) for y in x]
        ns = len(labels)
        u = tb.quad[(ns - 1) * 1296 + ((loc[0] * 6 + loc[1]) * 6 + loc[2]) * 6 + loc[3]]
        assert u >= 0
        v += tb.sym_w[j] * eri[layout.eri_block_offset(N, ns) + u * comb(N, ns)
                               + layout.set_index(tuple(labels))]
    return v


def _class_sum(tb, cls, f, eri, t, N, L, m):
    nout, nspec, nt, off, npat, start = cls
    others = [x for x in range(N) if x not in L]
    acc = 0.0
    for S in itertools.permutations(others, nspec):
        lab = tuple(L) + S
        for q in range(off + start[m], off + start[m + 1]):
            tm = tb.terms[q]
            v = _h(tb, f, eri, N, lab, int(tm[0]))
            if v == 0.0:
                continue
            v *= (int(tm[1]) & 0xFFFF) - 32768
            for i in range(int(tm[1]) >> 16):
                v *= _amp(tb, t, N, lab, int(tm[2 + i]))
            acc += v
    return acc / factorial(nspec)


def test_table_structure(tb):
    got = {(c[0], c[1]) for c in tb.classes}
    assert got == {(o, s) for o in (1, 2, 3) for s in range(4)} | {(0, 1), (0, 2), (0, 3)}
    for nout, nspec, nt, off, npat, start in tb.classes:
        assert npat == (1, 3, 29, 303)[nout]
        assert start[0] == 0 and start[-1] == nt and np.all(np.diff(start) >= 0)
    assert sorted(int(m) for m in tb.pat2m if m >= 0) == sorted(
        list(range(3)) + list(range(29)) + list(range(303)))
    assert [int((tb.quad[s * 1296:(s + 1) * 1296] >= 0).sum()) > 0 for s in range(3)] == [True] * 3


def _check(tb, N, max_out, sample=None):
    f = random_fock(N, seed=60 + N)
    eri = oint.eri_packed_from_b(random_bfactors(N, seed=61 + N), N, 3)
    t = random_amplitudes(N, "ph", seed=62 + N, scale=0.1)
    RA, EA = tier_a.TierA(N, 3).residual(f, layout.unpack_eri(eri, N, 3), t)
    for pos, labels, tup in layout.iter_amp_slots(N, 3):
        if len(labels) > max_out and (sample is None or pos not in sample):
            continue
        n = len(labels)
        m = layout.pattern_tuples(n).index(tuple(tup))
        # terms are stored for the canonical reordering of the output tuple
        cn = int(tb.canon[(0, 3, 32)[n - 1] + m])
        order = [(cn >> (9 + 2 * i)) & 3 for i in range(n)]
        assert sorted(order) == list(range(n))
        assert layout.pattern_tuples(n)[cn & 511] == tuple(tup[i] for i in order)
        Lr = tuple(labels[i] for i in order)
        r = sum(_class_sum(tb, c, f, eri, t, N, Lr, cn & 511) for c in tb.classes
                if c[0] == n and c[1] <= N - n)
        r = -r if cn >> 15 & 1 else r
        assert abs(r - RA[pos]) <= 1e-12 * max(1.0, np.abs(RA).max()), (labels, tup)
    e = sum(_class_sum(tb, c, f, eri, t, N, (), 0) for c in tb.classes if c[0] == 0 and c[1] <= N)
    assert abs(e - EA) < 1e-12


def test_tables_reproduce_oracle_two_pairs(tb):
    """N = 2: every output block and the energy."""
    _check(tb, 2, 2)


def test_tables_reproduce_oracle_one_pair_outputs_three_pairs(tb):
    """N = 3, one-pair outputs with up to two spectators (three-pair
    integrals and amplitudes) and the energy with three-pair doubles."""
    _check(tb, 3, 1)


def test_tables_reproduce_oracle_three_pair_outputs(tb):
    """N = 3, sampled three-pair outputs (canonical and reordered tuples, odd
    and even patterns): the relabelling and reordering sign of the stored
    canonical terms."""
    base = 3 * 3 + 29 * 3
    rng = np.random.default_rng(5)
    sample = set((base + rng.choice(303, 10, replace=False)).tolist())
    _check(tb, 3, 1, sample=sample)


def test_tables_reproduce_oracle_four_pairs_sampled(tb):
    """N = 4: one-pair outputs with up to three spectators and sampled
    two-pair outputs with up to two spectators (the terms are stored once per
    orbit under renamings of the spectator roles, weighted by its size)."""
    base = 3 * 4
    rng = np.random.default_rng(7)
    sample = set((base + rng.choice(29 * 6, 4, replace=False)).tolist())
    _check(tb, 4, 1, sample=sample)
