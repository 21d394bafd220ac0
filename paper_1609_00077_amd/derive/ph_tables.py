"""Term tables of the PH residual (k = 3) for the interpreted HIP kernel.

Every output block (one, two or three labels) and spectator class (0..3
spectators, each touched by the Hamiltonian term; Sec. II: H_3 acts on at
most three pairs) is enumerated by the same derivation as the PQ tables and
written, with the lookup tables the kernel needs, to one little-endian binary
file that the library reads when a PH call first needs it.

File layout (int32 unless marked; the whole file is zlib-compressed):
  magic 0x31485450, version 3, nclass, nh, nsym, nterm, ncw, nslot
  per class: nout, nspec, nterm, term offset, npat; then start[npat + 1]
             (terms of output pattern m are start[m] .. start[m+1], relative)
  cw_dict    ncw coefficient words (nf << 16) | (coef + 32768)
  slot_dict  nslot amplitude slot codes, slot_dict[0] = 0 (no factor)
  term columns, each padded to 4 bytes:
             h     nterm uint16: Hamiltonian term
             cw    nterm uint8: index into cw_dict
             slots 4 x nterm uint16 (slot-major): indices into slot_dict
  hstart     nh + 1
  sym_w      nsym doubles
  sym_code   nsym: kind | x0 << 4 | x1 << 8 | x2 << 12 | x3 << 16, kind 0 = f,
             1 = chemists' v; x = 2 * role + type (type 0 = o, 1 = v)
  pat2m      16 + 256 + 4096: pattern tuple (bits p0 | p1 << 4 | p2 << 8 of
             an ascending label set) -> pattern number, -1 if not stored
  m2pat      3 + 29 + 303: pattern number -> packed pattern tuple
  canon      3 + 29 + 303: pattern number -> m_c | p0 << 9 | p1 << 11 |
             p2 << 13 | negative << 15: the output's terms are those of
             pattern m_c with output role i at label L[p_i], times -1 if
             negative (terms are stored for canonical tuples only)
  quad       3 x 1296: local (p, q, r, s), each 0..5, of a label set of
             1, 2, 3 pairs -> index of the stored integral, -1 if none

Slot code of an amplitude factor: nlab | r0 << 2 | r1 << 5 | r2 << 8 |
p0 << 11 | p1 << 15 | p2 << 19, roles and patterns in the term's role order.
A term contributes coef / nspec! * h * prod(t) for every ordered choice of
distinct spectator labels outside the output set.  Terms are kept for the
canonical output tuples only, and once per orbit under renamings of the
spectator roles, with coef summed over the orbit.
"""
from __future__ import annotations

import itertools
import multiprocessing as mp
import os
import struct
import sys
import zlib

import numpy as np

from . import algebra
from .codegen import eri_quads
from .terms import enumerate_class, merge_terms

K = 3
MAGIC = 0x31485450
ZMAGIC = 0x315A4850
# output classes (nout, nspec) then energy classes (0, nspec)
CLASSES = [(o, s) for o in (1, 2, 3) for s in range(K + 1)] + [(0, s) for s in (1, 2, 3)]


SPLIT = 16      # pieces per Hamiltonian role set of a three-label output class


def canonical(mu):
    """(canonical tuple, position order p) with canonical = (mu[p0], mu[p1], ...)
    the smallest reordering of the pattern tuple."""
    best = None
    for p in itertools.permutations(range(len(mu))):
        c = tuple(mu[i] for i in p)
        if best is None or c < best[0]:
            best = (c, p)
    return best


def reorder_sign(mu, p):
    """Sign that takes the operator g^{mu[p0]} g^{mu[p1]} ... (labels in the
    order p) back to ascending label order: -1 per inversion of two odd
    patterns."""
    odd = [bin(mu[i]).count("1") % 2 for i in p]
    inv = sum(1 for i in range(len(p)) for j in range(i + 1, len(p))
              if p[i] > p[j] and odd[i] and odd[j])
    return -1 if inv % 2 else 1


def _odd(e):
    return bin(e).count("1") % 2


def _relabel(t, pi, h_sign_cache):
    """The term t with its roles renamed by pi, written in the stored form
    (roles of every factor ascending, Hamiltonian key sorted), and the sign
    that rewriting costs; None if the renamed Hamiltonian key does not exist."""
    sign = t.sign
    slots = []
    for rho, pats in t.slots:
        items = sorted(zip((pi[r] for r in rho), pats))
        order = sorted(range(len(rho)), key=lambda i: pi[rho[i]])
        inv = sum(1 for i in range(len(order)) for j in range(i + 1, len(order))
                  if order[i] > order[j] and _odd(pats[order[i]]) and _odd(pats[order[j]]))
        sign *= -1 if inv % 2 else 1
        slots.append((tuple(r for r, _ in items), tuple(p for _, p in items)))
    hroles = tuple(sorted(pi[r] for r in t.hroles))
    key = (t.hroles, t.hkey, tuple(sorted(pi.items())))
    if key not in h_sign_cache:
        I, J = t.hkey
        sI, I2 = algebra.sort_sign([4 * pi[g // 4] + g % 4 for g in I])
        sJ, J2 = algebra.sort_sign([4 * pi[g // 4] + g % 4 for g in J])
        new = algebra.hamiltonian_terms(hroles, K).get((I2, J2))
        hs = None
        if new is not None and sI and sJ:
            old = algebra.hamiltonian_terms(tuple(t.hroles), K)[t.hkey]
            mx = lambda x: 2 * pi[x // 2] + x % 2
            ratios = set()
            for sym, w in old.items():
                if sym[0] == "f":
                    img = ("f", mx(sym[1]), mx(sym[2]))
                else:
                    img = ("v",) + algebra.eri_canon(*(mx(x) for x in sym[1:]))
                wn = new.get(img)
                ratios.add(None if wn is None else round(wn / w, 9))
            if len(ratios) == 1 and len(new) == len(old) and next(iter(ratios)) in (1.0, -1.0):
                hs = int(next(iter(ratios)))
        h_sign_cache[key] = None if hs is None else ((I2, J2), hs)
    hk = h_sign_cache[key]
    if hk is None:
        return None
    return t._replace(sign=sign * hk[1], hroles=hroles, hkey=hk[0], slots=tuple(slots))


def spectator_canonical(terms, nout, nspec):
    """One representative per orbit of the terms under renamings of the
    spectator roles, its coefficient summed over the orbit.  The kernels sum
    every term over ordered spectator tuples, and renaming the spectator roles
    of a term equals reordering the tuple, so an orbit contributes |orbit|
    times its representative."""
    if nspec < 2:
        return terms
    cache = {}
    out = []
    spec = list(range(nout, nout + nspec))
    perms = []
    for p in itertools.permutations(spec):
        pi = {r: r for r in range(nout)}
        pi.update(dict(zip(spec, p)))
        perms.append(pi)
    for t in terms:
        best = None
        for pi in perms:
            img = _relabel(t, pi, cache)
            assert img is not None
            k = (img.hroles, img.hkey, tuple(sorted(img.slots)))
            if best is None or k < best[0]:
                best = (k, img)
        out.append(best[1])
    return out


def _unit(args):
    """Terms of one piece, for the canonical output tuples only: the terms of
    a reordered tuple are the same terms with the output roles relabelled
    (the derivation never orders labels), so the kernel maps every output to
    its canonical tuple and a sign."""
    nout, nspec, hroles, part = args
    terms = enumerate_class(K, nout, nspec, energy=(nout == 0), only_hroles={hroles}, part=part)
    if nout >= 2:
        terms = [t for t in terms if canonical(t.mu)[0] == t.mu]
    return (nout, nspec), merge_terms(spectator_canonical(terms, nout, nspec))


def _units():
    out = []
    for nout, nspec in CLASSES:
        allroles = tuple(range(nout + nspec))
        for hsize in range(1, K + 1):
            for hroles in itertools.combinations(allroles, hsize):
                if set(range(nout, nout + nspec)) <= set(hroles):
                    n = SPLIT if nout == 3 else 1
                    out.extend((nout, nspec, hroles, (i, n)) for i in range(n))
    # biggest pieces first
    return sorted(out, key=lambda u: (-u[0], -len(u[2])))


def enumerate_all(procs=None):
    """{(nout, nspec): merged terms} for every PH class.  Pieces are merged
    as they come and joined in a fixed order (the tables do not depend on
    scheduling); the orbit representatives of one class can come from
    several pieces, so classes with two or more spectators are merged once
    more."""
    raw = {c: [] for c in CLASSES}
    units = _units()
    with mp.Pool(procs or min(8, os.cpu_count() or 1)) as pool:
        for i, (cls, terms) in enumerate(pool.imap(_unit, units)):
            raw[cls].extend(terms)
            print(f"piece {i + 1}/{len(units)} {units[i][:3]}: {len(terms)} terms", flush=True)
    for cls in raw:
        if cls[1] >= 2:
            raw[cls] = merge_terms(raw[cls])
    return raw


def _slot_code(rho, pats):
    r = list(rho) + [0] * (3 - len(rho))
    p = list(pats) + [0] * (3 - len(pats))
    return len(rho) | r[0] << 2 | r[1] << 5 | r[2] << 8 | p[0] << 11 | p[1] << 15 | p[2] << 19


def _pack_pats(pats):
    p = list(pats) + [0] * (3 - len(pats))
    return p[0] | p[1] << 4 | p[2] << 8


def build(classes):
    hkeys, hindex = [], {}
    syms_w, syms_c, hstart = [], [], [0]

    def h_of(hroles, hkey):
        key = (hroles, hkey)
        if key not in hindex:
            hindex[key] = len(hkeys)
            hkeys.append(key)
            for sym, w in sorted(algebra.hamiltonian_terms(hroles, K)[hkey].items()):
                xs = list(sym[1:]) + [0] * (5 - len(sym))
                syms_w.append(w)
                syms_c.append((0 if sym[0] == "f" else 1) | xs[0] << 4 | xs[1] << 8
                              | xs[2] << 12 | xs[3] << 16)
            hstart.append(len(syms_w))
        return hindex[key]

    cls_hdr, rows, nrow = [], [], 0
    for nout, nspec in CLASSES:
        terms = classes[(nout, nspec)]
        pats = algebra.pattern_tuples(nout) if nout else [()]
        pidx = {p: i for i, p in enumerate(pats)}
        crow = []
        for t in terms:
            assert len(t.slots) <= 4 and -32768 < t.sign < 32768
            codes = [_slot_code(rho, p) for rho, p in t.slots] + [0] * (4 - len(t.slots))
            m = pidx[t.mu] if nout else 0
            crow.append((m, [h_of(tuple(t.hroles), t.hkey), len(t.slots) << 16 | (t.sign + 32768)]
                         + codes))
        crow.sort(key=lambda x: x[0])
        start = np.zeros(len(pats) + 1, dtype=np.int64)
        for m, _ in crow:
            start[m + 1] += 1
        cls_hdr.append((nout, nspec, len(crow), nrow, len(pats), np.cumsum(start)))
        nrow += len(crow)
        rows.append(np.asarray([r for _, r in crow], dtype=np.int32).reshape(-1, 6))
        del crow

    pat2m = np.full(16 + 256 + 4096, -1, dtype=np.int64)
    m2pat, canon = [], []
    base = 0
    for size in (1, 2, 3):
        tuples = algebra.pattern_tuples(size)
        for m, p in enumerate(tuples):
            pat2m[base + _pack_pats(p)] = m
            m2pat.append(_pack_pats(p))
            c, order = canonical(p)
            o = list(order) + [0] * (3 - size)
            canon.append(tuples.index(c) | o[0] << 9 | o[1] << 11 | o[2] << 13
                         | (1 << 15 if reorder_sign(p, order) < 0 else 0))
        base += 16 ** size
    quad = np.full(3 * 1296, -1, dtype=np.int64)
    for size in (1, 2, 3):
        stored = {q: u for u, q in enumerate(eri_quads(size))}
        for p, q, r, s in itertools.product(range(2 * size), repeat=4):
            a, b = (p, q) if p >= q else (q, p)
            c, d = (r, s) if r >= s else (s, r)
            pq, rs = a * (a + 1) // 2 + b, c * (c + 1) // 2 + d
            key = (a, b, c, d) if pq >= rs else (c, d, a, b)
            if key in stored:
                quad[(size - 1) * 1296 + ((p * 6 + q) * 6 + r) * 6 + s] = stored[key]
    return cls_hdr, np.concatenate(rows), hstart, syms_w, syms_c, pat2m, m2pat, canon, quad


def write(path, tables):
    """The table file, zlib-compressed inside a 12-byte container header
    (magic 0x315A4850, int64 uncompressed size).  Terms are stored as columns
    of small dictionary indices (the Hamiltonian term, the coefficient word and
    the four amplitude slot codes), which keeps the file and the kernel's
    reads small."""
    cls_hdr, rows, hstart, syms_w, syms_c, pat2m, m2pat, canon, quad = tables
    rows = np.asarray(rows, dtype=np.int64).reshape(-1, 6)
    assert rows[:, 0].max() < 65536
    cw_vals, cw_idx = np.unique(rows[:, 1], return_inverse=True)
    assert len(cw_vals) <= 256
    slot_vals = np.unique(np.concatenate([[0], rows[:, 2:].ravel()]))
    assert slot_vals[0] == 0 and len(slot_vals) <= 65536
    slot_idx = np.searchsorted(slot_vals, rows[:, 2:])
    i32 = lambda a: np.asarray(a, dtype="<i4").tobytes()
    pad4 = lambda b: b + b"\0" * (-len(b) % 4)
    parts = [i32([MAGIC, 3, len(cls_hdr), len(hstart) - 1, len(syms_w), len(rows), len(cw_vals),
                  len(slot_vals)])]
    for nout, nspec, nterm, off, npat, start in cls_hdr:
        parts.append(i32([nout, nspec, nterm, off, npat]))
        parts.append(i32(start))
    parts += [i32(cw_vals), i32(slot_vals),
              pad4(rows[:, 0].astype("<u2").tobytes()),
              pad4(cw_idx.astype("<u1").tobytes()),
              pad4(np.ascontiguousarray(slot_idx.T).astype("<u2").tobytes()),
              i32(hstart), np.asarray(syms_w, dtype="<f8").tobytes(), i32(syms_c), i32(pat2m),
              i32(m2pat), i32(canon), i32(quad)]
    raw = b"".join(parts)
    with open(path + ".tmp", "wb") as fh:
        fh.write(struct.pack("<iq", ZMAGIC, len(raw)))
        fh.write(zlib.compress(raw, 6))
    os.replace(path + ".tmp", path)


def read(path) -> bytes:
    """Uncompressed table bytes of a file written by write()."""
    with open(path, "rb") as fh:
        data = fh.read()
    magic, n = struct.unpack("<iq", data[:12])
    assert magic == ZMAGIC
    raw = zlib.decompress(data[12:])
    assert len(raw) == n
    return raw


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    out = argv[0] if argv else os.path.join(os.path.dirname(os.path.dirname(__file__)),
                                            "ph_terms.bin")
    classes = enumerate_all()
    tables = build(classes)
    write(out, tables)
    for nout, nspec, nterm, *_ in tables[0]:
        print(f"class out={nout} spec={nspec}: {nterm} terms")
    print(f"{len(tables[2]) - 1} Hamiltonian terms, {len(tables[3])} symbols -> {out}")
    sys.stdout.flush()


if __name__ == "__main__":
    main()
