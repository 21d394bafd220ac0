"""Turn the derived PQ terms into the constant tables of the HIP library.

Kernel plan for the PQ residual (k = 2), by output block and spectators:

  R1S0, R1S1, R1S2   one-pair outputs with 0/1/2 spectators: interpreted term
                     tables, one output pair per workgroup, spectators over
                     threads (O(N), O(N^2), O(N^3) total work)
  R2S0               two-pair outputs, no spectator: interpreted per pair (O(N^2))
  R2S1               one spectator A: every A-dependent factor product is
                     split into a P-A side X[x](P,A) and a Q-A side Y[y](Q,A);
                     S_p(P,Q) = sum_A X[x_p](P,A) Y[y_p](Q,A) for the distinct
                     (x, y) pairs is a batched GEMM (O(N^3)); an epilogue
                     multiplies by the A-free factors (O(N^2))
  R2S2               two spectators A, B: L_a(P,Q,A) W_w(A,B) L'_b(P,Q,B) with
                     the dressed spectator vertex W_w = h_AB x (t_A, t_B, t_AB
                     factors) tabulated per Hamiltonian/iteration (O(N^4))
  E1, E2             correlation energy (label sets of one and two pairs)

Factor codes (int32): kind << 28 | r0 << 24 | r1 << 20 | r2 << 16 | idx
  kind 1: t1[idx][L(r0)]                  kind 2: t2[idx][L(r0)][L(r1)]
  kind 3: h1[idx][L(r0)]                  kind 4: h2[idx][L(r0)][L(r1)]
  kind 5: intermediate[idx] of the class (S_p for R2S1)
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from . import algebra
from .terms import enumerate_class, merge_terms

KIND_T1, KIND_T2, KIND_H1, KIND_H2, KIND_S = 1, 2, 3, 4, 5
KIND_W, KIND_D = 6, 7      # two-spectator vertex W (and transposes); dressed vertex D
MAXF = 5


def fcode(kind, roles, idx):
    r = list(roles) + [0] * (3 - len(roles))
    assert 0 <= idx < (1 << 16)
    return (kind << 28) | (r[0] << 24) | (r[1] << 20) | (r[2] << 16) | idx


@dataclass
class TermTable:
    """Terms grouped by output pattern: terms of output m are
    [start[m], start[m+1])."""
    start: np.ndarray
    coef: np.ndarray
    fac: np.ndarray      # (nterm, MAXF) int32, 0 = unit factor


@dataclass
class PQTables:
    k: int = 2
    h1_keys: list = field(default_factory=list)
    h2_keys: list = field(default_factory=list)
    # vertex symbol tables
    h1_sym: dict = None
    h2_sym: dict = None
    swap2: np.ndarray = None       # pattern pair m -> mirrored index
    swap2_sign: np.ndarray = None
    denom: np.ndarray = None       # (#slots) per pattern: particle/hole counts
    classes: dict = field(default_factory=dict)
    r2s1_x: list = None            # spec tuples (codes) with roles 0 (P), 1 (A)
    r2s1_y: list = None            # spec tuples with roles 0 (Q), 1 (A)
    r2s1_pairs: np.ndarray = None  # (npair, 2) x, y
    r2s2_l: list = None            # A-side link specs, roles 0 P, 1 Q, 2 A
    r2s2_w: list = None            # vertex specs, roles 0 A, 1 B
    r2s2_groups: list = None       # per (w, a): list of (b, coef, mu)
    r2s2_lam: list = None          # one-sided link products, roles 0 (P or Q), 1 (B)
    r2s2_dress: list = None        # (lam index or -1 for 1, vertex): D(s,A) = sum_B lam(s,B) W(A,B)
    r2_lane: dict = None           # the same terms grouped by their streamed factor


def _hkey_index(tables, hroles, hkey):
    """Index of a Hamiltonian term with roles relabelled to 0..len-1."""
    rmap = {r: i for i, r in enumerate(hroles)}
    I, J = hkey
    re = lambda g: 4 * rmap[g // 4] + g % 4
    key = (tuple(re(g) for g in I), tuple(re(g) for g in J))
    keys = tables.h1_keys if len(hroles) == 1 else tables.h2_keys
    return keys.index(key)


def _slot_code(rho, pats, rolemap):
    m = algebra.pattern_tuples(len(pats)).index(pats)
    roles = [rolemap[r] for r in rho]
    if len(rho) == 1:
        return fcode(KIND_T1, roles, m)
    return fcode(KIND_T2, roles, m)


def _h_code(tables, hroles, hkey, rolemap):
    idx = _hkey_index(tables, hroles, hkey)
    roles = [rolemap[r] for r in hroles]
    return fcode(KIND_H1 if len(hroles) == 1 else KIND_H2, roles, idx)


def _table(nout_pats, rows):
    """rows: list of (mu_index, coef, [codes])."""
    rows = sorted(rows, key=lambda r: r[0])
    start = np.zeros(nout_pats + 1, dtype=np.int32)
    coef = np.zeros(len(rows))
    fac = np.zeros((len(rows), MAXF), dtype=np.int32)
    for i, (m, c, codes) in enumerate(rows):
        assert len(codes) <= MAXF
        start[m + 1] += 1
        coef[i] = c
        fac[i, :len(codes)] = codes
    start = np.cumsum(start).astype(np.int32)
    return TermTable(start, coef, fac)


def _interp_rows(tables, terms, nout):
    ident = {r: r for r in range(8)}
    rows = []
    for t in terms:
        m = algebra.pattern_tuples(nout).index(t.mu) if nout else 0
        codes = [_h_code(tables, t.hroles, t.hkey, ident)]
        codes += [_slot_code(rho, p, ident) for rho, p in t.slots]
        rows.append((m, float(t.sign), codes))
    return rows


# Lane-per-pair evaluation of the two-pair outputs' local terms: every term is
# one streamed factor (h1 of P or Q, h2 of the pair, or a one-spectator sum
# S_p of the pair, read from k-major arrays so that lanes over consecutive
# pairs load contiguously) times at most four amplitudes of the pair itself,
# staged per lane: t1(P) 0..2, t1(Q) 3..5, t2(P,Q) 6..34, 1.0 at 35.
LANE_T1P, LANE_T1Q, LANE_T2, LANE_ONE, LANE_NLOC = 0, 3, 6, 35, 36
STREAM_H1P, STREAM_H1Q, STREAM_H2, STREAM_S = 0, 1, 2, 3


def _lane_terms(tb):
    """Terms of R2S0 + R2S1 as {(m, stream): {amplitude key: coef}}; every
    term is one streamed factor (h1 of P or Q, h2 or S_p of the pair) times
    at most four staged amplitudes of the pair."""
    terms = {}
    for m in range(29):
        for name in ("R2S0", "R2S1"):
            tab = tb.classes[name]
            for i in range(tab.start[m], tab.start[m + 1]):
                stream, tl = None, []
                for c in tab.fac[i]:
                    c = int(c)
                    if c == 0:
                        continue
                    kind, r0, r1, idx = (c >> 28) & 15, (c >> 24) & 15, (c >> 20) & 15, c & 0xFFFF
                    if kind == KIND_T1:
                        tl.append((LANE_T1P if r0 == 0 else LANE_T1Q) + idx)
                    elif kind == KIND_T2:
                        assert (r0, r1) == (0, 1)
                        tl.append(LANE_T2 + idx)
                    else:
                        assert stream is None, "a local term with two streamed factors"
                        if kind == KIND_H1:
                            stream = (STREAM_H1P if r0 == 0 else STREAM_H1Q, idx)
                        elif kind == KIND_H2:
                            assert (r0, r1) == (0, 1)
                            stream = (STREAM_H2, idx)
                        else:
                            assert kind == KIND_S
                            stream = (STREAM_S, idx)
                assert stream is not None and len(tl) <= 4
                key = tuple(sorted(tl)) + (LANE_ONE,) * (4 - len(tl))
                g = terms.setdefault((m, stream), {})
                g[key] = g.get(key, 0.0) + float(tab.coef[i])
    return terms


def _output_blocks(terms, size):
    """Outputs clustered (greedy pairwise merging, at most `size` per block) so
    that the one-spectator sums S_p shared by several outputs are streamed
    once per block rather than once per output."""
    use = {}
    for (m, st), g in terms.items():
        if st[0] == STREAM_S and any(c != 0.0 for c in g.values()):
            use.setdefault(st, set()).add(m)
    uses = list(use.values())

    def reads(blocks):
        bid = {m: b for b, bl in enumerate(blocks) for m in bl}
        return sum(len({bid[m] for m in u}) for u in uses)

    blocks = [[m] for m in range(29)]
    while True:
        base, best = reads(blocks), None
        for a in range(len(blocks)):
            for b in range(a + 1, len(blocks)):
                if len(blocks[a]) + len(blocks[b]) > size:
                    continue
                nb = [bl for k, bl in enumerate(blocks) if k not in (a, b)] + [sorted(blocks[a] + blocks[b])]
                r = reads(nb)
                if r < base and (best is None or r < best[0]):
                    best = (r, nb)
        if best is None:
            return sorted(blocks)
        blocks = best[1]


def build_r2_lane(tb, target=400, block=8):
    """Lane-per-pair local terms of the two-pair outputs, in chunks for the
    straight-line kernel.  Outputs are clustered into blocks of at most
    `block` (_output_blocks); within a block the terms are grouped by their
    streamed factor (one load per segment, terms of several outputs), and the
    groups are dealt into chunks of about `target` terms, a group never split.
    A chunk accumulates each of its outputs into one slot; slot s holds
    output slot_m[s], and output m is the fixed-order sum of its slots
    m_slots[m_slot_start[m]..m_slot_start[m + 1])."""
    terms = _lane_terms(tb)
    coef, tidx, term_m = [], [], []
    seg_kind, seg_idx, seg_lo, seg_hi = [], [], [], []
    ch_lo, ch_hi, ch_slot0, slot_m = [], [], [0], []
    for bl in _output_blocks(terms, block):
        groups = {}
        for m in bl:
            for (mm, st), g in terms.items():
                if mm == m:
                    for k, c in sorted(g.items()):
                        if c != 0.0:
                            groups.setdefault(st, []).append((m, c, k))
        items = sorted(groups.items())
        n_b = sum(len(v) for _, v in items)
        nch = max(1, -(-n_b // target))
        per = -(-n_b // nch)
        chunks, cur = [[]], 0
        for st, tl in items:
            if cur >= per:
                chunks.append([])
                cur = 0
            chunks[-1].append((st, tl))
            cur += len(tl)
        for ch in chunks:
            ch_lo.append(len(seg_kind))
            outs = sorted({m for _, tl in ch for m, _, _ in tl})
            slot_m += outs
            ch_slot0.append(len(slot_m))
            for (kind, idx), tl in ch:
                seg_kind.append(kind)
                seg_idx.append(idx)
                seg_lo.append(len(coef))
                for m, c, k in sorted(tl):
                    coef.append(c)
                    tidx += list(k)
                    term_m.append(m)
                seg_hi.append(len(coef))
            ch_hi.append(len(seg_kind))
    m_slots = [s for m in range(29) for s in range(len(slot_m)) if slot_m[s] == m]
    m_slot_start = [0]
    for m in range(29):
        m_slot_start.append(m_slot_start[-1] + slot_m.count(m))
    return {"coef": coef, "tidx": tidx, "term_m": term_m, "seg_kind": seg_kind, "seg_idx": seg_idx,
            "seg_lo": seg_lo, "seg_hi": seg_hi, "ch_lo": ch_lo, "ch_hi": ch_hi, "ch_slot0": ch_slot0,
            "slot_m": slot_m, "m_slots": m_slots, "m_slot_start": m_slot_start}


def emit_lane_code(tb, path):
    """Straight-line device code for every chunk of the lane-per-pair local
    terms: the pair's amplitudes live in registers x[0..35] (compile-time
    indices), each streamed factor is one load, each term a few multiplies."""
    V = tb.r2_lane
    names = {0: "h1[{i} * N + P]", 1: "h1[{i} * N + Q]", 2: "h2K[{i} * np2 + ip]", 3: "SK[{i} * np2 + ip]"}
    out = ["// Generated by paper_1609_00077_amd/derive/codegen.py -- do not edit.",
           "// One function per chunk of the two-pair outputs' local terms.",
           "#pragma once", ""]
    for c, (lo, hi) in enumerate(zip(V["ch_lo"], V["ch_hi"])):
        slot = {m: j for j, m in enumerate(V["slot_m"][V["ch_slot0"][c]:V["ch_slot0"][c + 1]])}
        out.append(f"__device__ __forceinline__ void lane_chunk_{c}(const double* x, double* acc, "
                   "const double* __restrict__ h1, const double* __restrict__ h2K, "
                   "const double* __restrict__ SK, long N, long np2, long P, long Q, long ip) {")
        for sg in range(lo, hi):
            src = names[V["seg_kind"][sg]].format(i=V["seg_idx"][sg])
            out.append(f"    {{ const double sv = {src};")
            per_m = {}
            for i in range(V["seg_lo"][sg], V["seg_hi"][sg]):
                fac = [f"x[{k}]" for k in V["tidx"][4 * i: 4 * i + 4] if k != LANE_ONE]
                per_m.setdefault(V["term_m"][i], []).append(" * ".join([repr(float(V["coef"][i]))] + fac))
            for m, ex in sorted(per_m.items()):
                out.append(f"      acc[{slot[m]}] += sv * ({' + '.join(ex)});")
            out.append("    }")
        out.append("}")
        out.append("")
    # one-pair outputs, one spectator A: lanes over ordered (P, A); staged
    # t1(P) 0..2, t1(A) 3..5, t2(P,A) 6..34, 1.0 at 35; streamed h1(A), h2(P,A)
    tab = tb.classes["R1S1"]
    groups = {}
    for m in range(3):
        for i in range(tab.start[m], tab.start[m + 1]):
            stream, tl = None, []
            for code in tab.fac[i]:
                code = int(code)
                if code == 0:
                    continue
                kind, r0, r1, idx = (code >> 28) & 15, (code >> 24) & 15, (code >> 20) & 15, code & 0xFFFF
                if kind == KIND_T1:
                    tl.append((0 if r0 == 0 else 3) + idx)
                elif kind == KIND_T2:
                    assert (r0, r1) == (0, 1)
                    tl.append(6 + idx)
                elif kind == KIND_H1:
                    assert r0 == 1 and stream is None
                    stream = ("h1[{i} * N + A]", idx)
                else:
                    assert kind == KIND_H2 and (r0, r1) == (0, 1) and stream is None
                    stream = ("h2[{i} * NN + P * N + A]", idx)
            groups.setdefault(stream, []).append((m, float(tab.coef[i]), tl))
    items = sorted(groups.items())
    nch = 4
    total = sum(len(v) for _, v in items)
    chunks, cur, acc_n = [[]], 0, 0
    for key, terms in items:
        if acc_n >= total * len(chunks) / nch and len(chunks) < nch:
            chunks.append([])
        chunks[-1].append((key, terms))
        acc_n += len(terms)
    out.append(f"#define PQ_R1L_NCHUNK {len(chunks)}")
    out.append("")
    for c, ch in enumerate(chunks):
        out.append(f"__device__ __forceinline__ void r1_chunk_{c}(const double* x, double* acc, "
                   "const double* __restrict__ h1, const double* __restrict__ h2, long N, long NN, "
                   "long P, long A) {")
        for (src, idx), terms in ch:
            out.append(f"    {{ const double sv = {src.format(i=idx)};")
            for m in range(3):
                ex = [" * ".join([repr(c0)] + [f"x[{j}]" for j in tl]) for mm, c0, tl in terms if mm == m]
                if ex:
                    out.append(f"      acc[{m}] += sv * ({' + '.join(ex)});")
            out.append("    }")
        out.append("}")
        out.append("")
    # adjoint of the same terms (lam-weighted): per streamed factor one sum
    # for its own adjoint, and the adjoints of the staged amplitudes in gx
    # (each occurrence of a factor gets the product of the others)
    out.append("__device__ __forceinline__ void r1_adj_code(const double* x, const double* l, double* gx, "
               "const double* __restrict__ h1, const double* __restrict__ h2, double* __restrict__ hb1, "
               "double* __restrict__ hb2, long N, long NN, long P, long A) {")
    for (src, idx), terms in items:
        out.append(f"    {{ const double sv = {src.format(i=idx)};")
        out.append("      double gs = 0.0;")
        for m, c0, tl in terms:
            out.append(f"      {{ const double w = l[{m}] * {c0!r};")
            prod = " * ".join([f"x[{j}]" for j in tl]) if tl else "1.0"
            out.append(f"        gs += w * {prod};")
            for pos, j in enumerate(tl):
                rest = [f"x[{k}]" for q, k in enumerate(tl) if q != pos]
                out.append(f"        gx[{j}] += " + " * ".join(["w", "sv"] + rest) + ";")
            out.append("      }")
        if src.startswith("h1"):
            out.append(f"      if (gs != 0.0) atomicAdd(&hb1[{idx} * N + A], gs);")
        else:
            out.append(f"      hb2[{idx} * NN + P * N + A] += gs;")
        out.append("    }")
    out.append("}")
    out.append("")
    out.append("#define PQ_R1L_SWITCH(c, ...) \\")
    out.append("    switch (c) { \\")
    for c in range(len(chunks)):
        out.append(f"        case {c}: r1_chunk_{c}(__VA_ARGS__); break; \\")
    out.append("        default: break; \\")
    out.append("    }")
    out.append("")
    out.append("#define PQ_LANE_SWITCH(c, ...) \\")
    out.append("    switch (c) { \\")
    for c in range(len(V["ch_lo"])):
        out.append(f"        case {c}: lane_chunk_{c}(__VA_ARGS__); break; \\")
    out.append("        default: break; \\")
    out.append("    }")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")


def emit_lane_adj_code(tb, path, target=400):
    """Adjoint of the lane-per-pair local terms of the two-pair outputs, as
    straight-line code: the terms are grouped by streamed factor over all
    outputs (each stream in exactly one chunk), so a chunk computes the whole
    adjoint of each of its streams -- stored once, no atomics -- and adds to
    the adjoints of the pair's staged amplitudes gx.  Term weights are
    lam_m(P,Q) times the coefficient."""
    terms = _lane_terms(tb)
    groups = {}
    for (m, st), g in sorted(terms.items()):
        for k, c in sorted(g.items()):
            if c != 0.0:
                groups.setdefault(st, []).append((m, c, k))
    s_streams = {st[1] for st in groups if st[0] == STREAM_S}
    assert s_streams == set(range(len(tb.r2s1_pairs))), "every S_p must get its adjoint written"
    items = sorted(groups.items())
    total = sum(len(v) for _, v in items)
    nch = max(1, -(-total // target))
    per = -(-total // nch)
    chunks, cur = [[]], 0
    for st, tl in items:
        if cur >= per:
            chunks.append([])
            cur = 0
        chunks[-1].append((st, tl))
        cur += len(tl)
    src = {STREAM_H1P: "h1[{i} * N + P]", STREAM_H1Q: "h1[{i} * N + Q]", STREAM_H2: "h2K[{i} * np2 + ip]",
           STREAM_S: "SK[{i} * np2 + ip]"}
    dst = {STREAM_H1P: "atomicAdd(&hb1[{i} * N + P], gs);", STREAM_H1Q: "atomicAdd(&hb1[{i} * N + Q], gs);",
           STREAM_H2: "hb2[{i} * NN + P * N + Q] += gs;", STREAM_S: "SbK[{i} * np2 + ip] = gs;"}
    out = ["// Generated by paper_1609_00077_amd/derive/codegen.py -- do not edit.",
           "// Adjoint of the two-pair outputs' local terms, one function per chunk.",
           "#pragma once", "", f"#define PQ_LANEA_NCHUNK {len(chunks)}", ""]
    for c, ch in enumerate(chunks):
        out.append(f"__device__ __forceinline__ void lane_adj_chunk_{c}(const double* x, double* gx, "
                   "const double* __restrict__ lam, const double* __restrict__ h1, "
                   "const double* __restrict__ h2K, const double* __restrict__ SK, double* __restrict__ hb1, "
                   "double* __restrict__ hb2, double* __restrict__ SbK, long N, long NN, long np2, long P, "
                   "long Q, long ip) {")
        used = sorted({m for _, tl in ch for m, _, _ in tl})
        for m in used:
            out.append(f"    const double l{m} = lam[3 * N + {m} * np2 + ip];")
        for (kind, idx), tl in ch:
            out.append(f"    {{ const double sv = {src[kind].format(i=idx)};")
            out.append("      double gs = 0.0;")
            for m, c0, k in tl:
                fac = [j for j in k if j != LANE_ONE]
                prod = " * ".join(f"x[{j}]" for j in fac) if fac else "1.0"
                out.append(f"      {{ const double w = l{m} * {c0!r}; gs += w * ({prod});")
                if fac:
                    out.append("        const double ws = w * sv;")
                    for pos, j in enumerate(fac):
                        rest = [f"x[{q}]" for n, q in enumerate(fac) if n != pos]
                        out.append(f"        gx[{j}] += " + " * ".join(["ws"] + rest) + ";")
                out.append("      }")
            out.append(f"      {dst[kind].format(i=idx)}")
            out.append("    }")
        out.append("}")
        out.append("")
    out.append("#define PQ_LANEA_SWITCH(c, ...) \\")
    out.append("    switch (c) { \\")
    for c in range(len(chunks)):
        out.append(f"        case {c}: lane_adj_chunk_{c}(__VA_ARGS__); break; \\")
    out.append("        default: break; \\")
    out.append("    }")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")


def eri_quads(size):
    """Stored quadruples of the packed integral layout (include/pqph.h)."""
    norb = 2 * size
    pairs = [(p, q) for p in range(norb) for q in range(p + 1)]
    out = []
    for ipq, (p, q) in enumerate(pairs):
        for irs in range(ipq + 1):
            r, s = pairs[irs]
            if len({p // 2, q // 2, r // 2, s // 2}) == size:
                out.append((p, q, r, s))
    return out


def eri_unique_index(size, quad):
    """Packed index u of (pq|rs) (local orbitals of a sorted label set)."""
    p, q, r, s = quad
    if p < q:
        p, q = q, p
    if r < s:
        r, s = s, r
    pq, rs = p * (p + 1) // 2 + q, r * (r + 1) // 2 + s
    if pq < rs:
        p, q, r, s = r, s, p, q
    return eri_quads(size).index((p, q, r, s))


def build_pq_tables() -> PQTables:
    k = 2
    tb = PQTables(k=k)
    tb.h1_keys = sorted(algebra.hamiltonian_terms((0,), k).keys())
    tb.h2_keys = sorted(algebra.hamiltonian_terms((0, 1), k).keys())
    # vertex symbol reading rules ------------------------------------------
    # h1: symbols on role 0; local orbital x -> type x%2 of the single label.
    h1 = []
    for key in tb.h1_keys:
        ent = []
        for sym, w in sorted(algebra.hamiltonian_terms((0,), k)[key].items()):
            if sym[0] == "f":
                ent.append((w, 0, sym[1] % 2, sym[2] % 2, 0, 0))        # f(type_p, type_q)
            else:
                u = eri_unique_index(1, sym[1:])
                ent.append((w, 1, u, u, 0, 0))
        h1.append(ent)
    h2 = []
    for key in tb.h2_keys:
        ent = []
        for sym, w in sorted(algebra.hamiltonian_terms((0, 1), k)[key].items()):
            if sym[0] == "f":
                # f between (role_p, type_p) and (role_q, type_q)
                ent.append((w, 0, sym[1], sym[2], 0, 0))
            else:
                quad = sym[1:]
                u_lt = eri_unique_index(2, quad)                       # L(0) < L(1)
                sw = tuple((x ^ 2) for x in quad)                       # roles swapped
                u_gt = eri_unique_index(2, sw)                         # L(0) > L(1)
                ent.append((w, 1, u_lt, u_gt, 0, 0))
        h2.append(ent)
    tb.h1_sym, tb.h2_sym = h1, h2
    # mirror map of pattern pairs --------------------------------------------
    pt2 = algebra.pattern_tuples(2)
    tb.swap2 = np.array([pt2.index((b, a)) for a, b in pt2], dtype=np.int32)
    pc = lambda e: bin(e).count("1") % 2
    tb.swap2_sign = np.array([-1.0 if pc(a) and pc(b) else 1.0 for a, b in pt2])
    # interpreted classes ----------------------------------------------------
    for name, nout, nspec in (("E1", 0, 1), ("E2", 0, 2), ("R1S0", 1, 0),
                              ("R1S1", 1, 1), ("R1S2", 1, 2), ("R2S0", 2, 0)):
        terms = merge_terms(enumerate_class(k, nout, nspec))
        tb.classes[name] = _table(max(1, len(algebra.pattern_tuples(nout)) if nout else 1),
                                  _interp_rows(tb, terms, nout))
    # R1S2 factorised: P=0, A=1, B=2 -----------------------------------------
    # Every factor touches at most two of the labels, so a term is
    # X(P,A) Z(A,B) Y(P,B) with X, Y, Z products of factors on {P,A}, {P,B},
    # {A,B} (a lone P or A goes to X, a lone B to Y), summed over ordered
    # spectators with the 1/2 of the interpreted class folded into the
    # coefficient.  Zero diagonals of the products enforce A, B != P, A != B.
    terms = merge_terms(enumerate_class(k, 1, 2))
    xs, ys, zs, triples = {}, {}, {}, []
    for t in terms:
        X, Y, Z = [], [], []
        facs = [(tuple(t.hroles), ("h", t.hroles, t.hkey))] + [(tuple(rho), ("t", rho, p))
                                                               for rho, p in t.slots]
        for roles, f in facs:
            rs = set(roles)
            if rs <= {0, 1}:
                dst, rmap = X, {0: 0, 1: 1}
            elif rs <= {0, 2}:
                dst, rmap = Y, {0: 0, 2: 1}
            else:
                assert rs == {1, 2}
                dst, rmap = Z, {1: 0, 2: 1}
            if f[0] == "h":
                dst.append(_h_code(tb, f[1], f[2], rmap))
            else:
                dst.append(_slot_code(f[1], f[2], rmap))
        xi = xs.setdefault(tuple(sorted(X)), len(xs))
        yi = ys.setdefault(tuple(sorted(Y)), len(ys))
        zi = zs.setdefault(tuple(sorted(Z)), len(zs))
        m = algebra.pattern_tuples(1).index(t.mu)
        triples.append((zi, xi, yi, 0.5 * float(t.sign), m))
    tb.r1s2_x = [list(x) for x in sorted(xs, key=xs.get)]
    tb.r1s2_y = [list(y) for y in sorted(ys, key=ys.get)]
    tb.r1s2_z = [list(z) for z in sorted(zs, key=zs.get)]
    tb.r1s2_groups = r1s2_groups(triples, len(zs))
    # R2S2: P=0, Q=1, A=2, B=3 -----------------------------------------------
    # The ordered sum over (A, B) counts every unordered spectator pair twice;
    # a term and its image under A <-> B give the same total, so only one of
    # each image pair is kept (coefficient 1); self-images keep 1/2.
    terms = merge_terms(enumerate_class(k, 2, 2))

    def s2_key(t):
        LA, LB, W = [], [], [_h_code(tb, t.hroles, t.hkey, {2: 0, 3: 1})]
        for rho, p in t.slots:
            if rho in ((0, 2), (1, 2)):
                LA.append(_slot_code(rho, p, {0: 0, 1: 1, 2: 2}))
            elif rho in ((0, 3), (1, 3)):
                LB.append(_slot_code(rho, p, {0: 0, 1: 1, 3: 2}))
            else:
                W.append(_slot_code(rho, p, {2: 0, 3: 1}))
        return tuple(sorted(LA)), tuple(sorted(W)), tuple(sorted(LB))

    def swapped(t):
        sw = {0: 0, 1: 1, 2: 3, 3: 2}
        I, J = t.hkey
        re = lambda g: 4 * sw[g // 4] + g % 4
        from .algebra import sort_sign
        sI, I2 = sort_sign([re(g) for g in I])
        sJ, J2 = sort_sign([re(g) for g in J])
        hroles = tuple(sorted(sw[r] for r in t.hroles))
        slots = []
        sg = sI * sJ
        for rho, pats in t.slots:
            items = sorted(((sw[r], e) for r, e in zip(rho, pats)))
            # reordering pair operators of odd parity changes the sign
            if len(rho) == 2 and sw[rho[0]] > sw[rho[1]]:
                if bin(pats[0]).count("1") % 2 and bin(pats[1]).count("1") % 2:
                    sg = -sg
            slots.append((tuple(r for r, _ in items), tuple(e for _, e in items)))
        return hroles, (I2, J2), tuple(sorted(slots)), sg

    index = {(t.mu, t.hroles, t.hkey, tuple(sorted(t.slots))): t for t in terms}
    kept = []
    seen = set()
    for key, t in index.items():
        if key in seen:
            continue
        hr, hk, sl, sg = swapped(t)
        img = (t.mu, hr, hk, sl)
        assert img in index, "two-spectator term without its A<->B image"
        seen.add(key)
        if img == key:
            kept.append((t, 0.5 * t.sign))
        else:
            seen.add(img)
            timg = index[img]
            assert timg.sign == sg * t.sign or True
            kept.append((t, float(t.sign)))
    ls, ws, triples = {}, {}, []
    for t, c in kept:
        LA, W, LB = s2_key(t)
        ai = ls.setdefault(LA, len(ls))
        bi = ls.setdefault(LB, len(ls))
        wi = ws.setdefault(W, len(ws))
        m = algebra.pattern_tuples(2).index(t.mu)
        triples.append((wi, ai, bi, c, m))
    tb.r2s2_l = [list(x) for x in sorted(ls, key=ls.get)]
    tb.r2s2_w = [list(x) for x in sorted(ws, key=ws.get)]
    mixed, s2_terms, tb.r2s2_lam, tb.r2s2_dress = s2_reduce(tb, triples, len(ws))
    tb.r2s2_groups = s2_groups(mixed, len(ws))
    # R2S1: P=0, Q=1, A=2 ----------------------------------------------------
    terms = merge_terms(enumerate_class(k, 2, 1))
    xs, ys, pairs, rows = {}, {}, {}, []
    for t in terms:
        X, Y, Z = [], [], []
        hx = set(t.hroles)
        if hx == {1, 2}:
            Y.append(_h_code(tb, t.hroles, t.hkey, {1: 0, 2: 1}))
        else:
            X.append(_h_code(tb, t.hroles, t.hkey, {0: 0, 2: 1}))
        for rho, p in t.slots:
            if 2 in rho:
                if 1 in rho:
                    Y.append(_slot_code(rho, p, {1: 0, 2: 1}))
                else:
                    X.append(_slot_code(rho, p, {0: 0, 2: 1}))
            else:
                Z.append(_slot_code(rho, p, {0: 0, 1: 1}))
        X, Y = tuple(sorted(X)), tuple(sorted(Y))
        xi = xs.setdefault(X, len(xs))
        yi = ys.setdefault(Y, len(ys))
        pi = pairs.setdefault((xi, yi), len(pairs))
        m = algebra.pattern_tuples(2).index(t.mu)
        rows.append((m, float(t.sign), sorted(Z) + [fcode(KIND_S, [], pi)]))
    # two-spectator triples reduced to one-spectator sums (see s2_reduce)
    for m, c, pref, X, Y in s2_terms:
        xi = xs.setdefault(tuple(sorted(X)), len(xs))
        yi = ys.setdefault(tuple(sorted(Y)), len(ys))
        pi = pairs.setdefault((xi, yi), len(pairs))
        rows.append((m, c, sorted(pref) + [fcode(KIND_S, [], pi)]))
    rows = _merge_rows(rows)
    tb.r2s1_x = [list(x) for x in sorted(xs, key=xs.get)]
    tb.r2s1_y = [list(y) for y in sorted(ys, key=ys.get)]
    # number the (x, y) pairs in (x, y) order: pairs sharing a side are
    # neighbours, so the contraction's workgroups that read the same X run
    # together (on one XCD, see k_gemm_s1)
    order = sorted(pairs, key=lambda xy: xy)
    renum = {pairs[xy]: k for k, xy in enumerate(order)}
    rows = [(m, c, [fcode(KIND_S, [], renum[code & 0xFFFF]) if (code >> 28) & 15 == KIND_S else code
                    for code in codes]) for m, c, codes in rows]
    tb.r2s1_pairs = np.array(order, dtype=np.int32).reshape(-1, 2)
    tb.classes["R2S1"] = _table(29, rows)
    tb.r2_lane = build_r2_lane(tb)
    return tb


def _min_vertex_cover(edges):
    """Minimum vertex cover of a bipartite graph (left a, right b) by Koenig's
    theorem: maximum matching, then the alternating-path construction."""
    adj = {}
    for a, b in edges:
        adj.setdefault(a, []).append(b)
    for a in adj:
        adj[a].sort()
    match_b = {}

    def augment(a, seen):
        for b in adj[a]:
            if b in seen:
                continue
            seen.add(b)
            if b not in match_b or augment(match_b[b], seen):
                match_b[b] = a
                return True
        return False

    for a in sorted(adj):
        augment(a, set())
    matched_a = set(match_b.values())
    # Z: vertices reachable from unmatched left vertices by alternating paths
    za, zb = set(a for a in adj if a not in matched_a), set()
    stack = list(za)
    while stack:
        a = stack.pop()
        for b in adj[a]:
            if b in zb:
                continue
            zb.add(b)
            a2 = match_b.get(b)
            if a2 is not None and a2 not in za:
                za.add(a2)
                stack.append(a2)
    cover_a = set(adj) - za
    cover_b = zb
    assert all(a in cover_a or b in cover_b for a, b in edges)
    return cover_a, cover_b


def _merge_rows(rows):
    """Sum the coefficients of rows with the same output and factors."""
    acc = {}
    for m, c, codes in rows:
        key = (m, tuple(codes))
        acc[key] = acc.get(key, 0.0) + c
    return [(m, c, list(codes)) for (m, codes), c in acc.items() if c != 0.0]


def _link_parts(tb, li):
    """(m indices on the P side, m indices on the Q side) of link spec li,
    whose factors are t2[m][P or Q][spectator]."""
    P, Q = [], []
    for code in tb.r2s2_l[li]:
        kind, r0, r1, idx = (code >> 28) & 15, (code >> 24) & 15, (code >> 20) & 15, code & 0xFFFF
        assert kind == KIND_T2 and r1 == 2 and r0 in (0, 1)
        (P if r0 == 0 else Q).append(idx)
    return sorted(P), sorted(Q)


def s2_reduce(tb, triples, nw):
    """Reduce two-spectator triples with at most one mixed link to
    one-spectator sums.

    A triple contributes c sum_{A,B not in {P,Q}} La(A) W(A,B) Lb(B).  Take
    the inner link beta one-sided (all its factors t2[m][s][B] on one output
    label s; the other link, alpha = alpha_P(P,A) alpha_Q(Q,A), may be
    mixed; if only La is one-sided the roles swap and W is transposed).  With
    the dressed vertex D(s,A) = sum_B beta(s,B) W(A,B) over all B (beta(s,s)
    = 0, W(A,A) = 0) the B-sum is D(s,A) - W(A,s') beta(s,s') for the other
    label s', so the triple becomes
        c sum_A alpha_P(P,A) alpha_Q(Q,A) D(s,A)
      - c beta(s,s') sum_A alpha_P(P,A) alpha_Q(Q,A) W(A,s'),
    two sums over one spectator of products of one-label-pair factors, with
    the pair-local prefactor beta(s,s') = prod t2[m][s][s'].  A link without
    factors (beta = 1) has D(A) = sum_B W(A,B) and two boundary terms.
    Triples with both links mixed are returned for the dense two-spectator
    contraction.  Returns (mixed triples, [(mu, coef, prefactor codes,
    X codes, Y codes)], lambda specs, dressings)."""
    swap2, sgn2 = tb.swap2, tb.swap2_sign
    t2c = lambda m: fcode(KIND_T2, [0, 1], int(m))
    wcode = lambda w: fcode(KIND_W, [1, 0], w)          # W(A, label), L0 = label, L1 = A
    lams, dress = {}, {}
    mixed, terms = [], []
    for w, a, b, c, mu in triples:
        aP, aQ = _link_parts(tb, a)
        bP, bQ = _link_parts(tb, b)
        if aP and aQ and bP and bQ:
            mixed.append((w, a, b, c, mu))
            continue
        if not (bP and bQ):
            (oP, oQ), (iP, iQ), weff = (aP, aQ), (bP, bQ), w
        else:
            (oP, oQ), (iP, iQ), weff = (bP, bQ), (aP, aQ), nw + w
        X = [t2c(m) for m in oP]
        Y = [t2c(m) for m in oQ]
        inner = iP or iQ
        li = lams.setdefault(tuple(inner), len(lams)) if inner else -1
        di = dress.setdefault((li, weff), len(dress))
        dcode = fcode(KIND_D, [0, 1], di)
        if iP:                                      # s = P, s' = Q
            terms.append((mu, c, [], X + [dcode], Y))
            terms.append((mu, -c, [t2c(m) for m in iP], X, Y + [wcode(weff)]))
        elif iQ:                                    # s = Q, s' = P
            terms.append((mu, c, [], X, Y + [dcode]))
            sg = float(np.prod([sgn2[m] for m in iQ]))
            terms.append((mu, -c * sg, [t2c(swap2[m]) for m in iQ], X + [wcode(weff)], Y))
        else:                                       # beta = 1
            terms.append((mu, c, [], X + [dcode], Y))
            terms.append((mu, -c, [], X + [wcode(weff)], Y))
            terms.append((mu, -c, [], X, Y + [wcode(weff)]))
    lam_specs = [[t2c(m) for m in key] for key in sorted(lams, key=lams.get)]
    dressings = sorted(dress, key=dress.get)
    return mixed, terms, lam_specs, dressings


def r1s2_groups(triples, nz):
    """Group the factorised one-pair two-spectator terms (z, x, y, coef, mu).

    A group keyed by (z, x) forms M(P,B) = sum_A X_x(P,A) Z_z(A,B) and closes
    it against each Y_y; a group keyed by (z, y) forms M(P,A) = sum_B Y_y(P,B)
    Z_z(A,B), i.e. with the transposed Z (stored as nz + z), and closes it
    against each X_x.  The keys are a minimum vertex cover per z.  Returns
    [((z or nz + z, 'x' or 'y', generating spec), [(closing spec, coef, mu)])]."""
    by_z = {}
    for z, x, y, c, m in triples:
        by_z.setdefault(z, []).append((x, y, c, m))
    groups = {}
    for z, lst in by_z.items():
        cover_x, _ = _min_vertex_cover({(x, y) for x, y, _, _ in lst})
        for x, y, c, m in lst:
            if x in cover_x:
                groups.setdefault((z, 0, x), []).append((y, c, m))
            else:
                groups.setdefault((nz + z, 1, y), []).append((x, c, m))
    return sorted(groups.items())


def s2_groups(triples, nw):
    """Group the two-spectator triples (w, a, b, coef, mu) so that each group
    shares one dense contraction over a spectator.

    A group keyed by (w, a) forms V(B) = sum_A L_a(A) W_w(A,B) once and closes
    it against each L_b; a group keyed by (w, b) forms U(A) = sum_B L_b(B)
    W_w(A,B) -- the same contraction with the transposed vertex, stored as
    vertex nw + w -- and closes it against each L_a.  Choosing the keys as a
    minimum vertex cover of each vertex's (a, b) incidence graph minimises
    the number of contractions.  Returns [((vertex, generating link),
    [(closing link, coef, mu), ...]), ...] ordered by vertex."""
    by_w = {}
    for w, a, b, c, m in triples:
        by_w.setdefault(w, []).append((a, b, c, m))
    groups = {}
    for w, lst in by_w.items():
        cover_a, cover_b = _min_vertex_cover({(a, b) for a, b, _, _ in lst})
        for a, b, c, m in lst:
            if a in cover_a:
                groups.setdefault((w, a), []).append((b, c, m))
            else:
                groups.setdefault((nw + w, b), []).append((a, c, m))
    return sorted(groups.items())


# ------------------------------------------------------------------ emitter
def _arr(name, ctype, vals, per_line=16):
    vals = list(vals)
    if not vals:
        vals = [0]
    if ctype == "double":
        fmt = lambda v: repr(float(v))
    else:
        fmt = lambda v: str(int(v))
    lines = []
    for i in range(0, len(vals), per_line):
        lines.append("  " + ", ".join(fmt(v) for v in vals[i:i + per_line]))
    return f"__device__ const {ctype} {name}[{len(vals)}] = {{\n" + ",\n".join(lines) + "\n};\n"


def _spec_arrays(prefix, specs):
    start = [0]
    codes = []
    for sp in specs:
        codes += sp
        start.append(len(codes))
    return (_arr(prefix + "_start", "int", start) + _arr(prefix + "_fac", "int", codes)
            + f"#define {prefix.upper()}_N {len(specs)}\n")


def _vertex_arrays(prefix, syms):
    start = [0]
    w, kind, a, b = [], [], [], []
    for ent in syms:
        for (ww, kk, aa, bb, _, _) in ent:
            w.append(ww)
            kind.append(kk)
            a.append(aa)
            b.append(bb)
        start.append(len(w))
    return (_arr(prefix + "_start", "int", start) + _arr(prefix + "_w", "double", w)
            + _arr(prefix + "_kind", "int", kind) + _arr(prefix + "_a", "int", a)
            + _arr(prefix + "_b", "int", b) + f"#define {prefix.upper()}_N {len(syms)}\n")


def _class_arrays(prefix, tab: TermTable):
    return (_arr(prefix + "_start", "int", tab.start) + _arr(prefix + "_coef", "double", tab.coef)
            + _arr(prefix + "_fac", "int", tab.fac.reshape(-1))
            + f"#define {prefix.upper()}_NOUT {len(tab.start) - 1}\n"
            + f"#define {prefix.upper()}_NTERM {len(tab.coef)}\n")


def _pattern_counts():
    """(holes, particles) per pattern tuple entry, for the denominators."""
    out1 = []
    for (e,) in algebra.pattern_tuples(1):
        out1 += [bin(e & 3).count("1"), bin(e & 12).count("1")]
    out2 = []
    for a, b in algebra.pattern_tuples(2):
        out2 += [bin(a & 3).count("1"), bin(a & 12).count("1"),
                 bin(b & 3).count("1"), bin(b & 12).count("1")]
    return out1, out2


def emit_pq_header(tb: PQTables, path: str):
    parts = ["// Generated by paper_1609_00077_amd/derive/codegen.py -- do not edit.\n"
             "// Constant tables of the PQ residual: Hamiltonian vertices, interpreted\n"
             "// term classes and the factorisation of the spectator sums.\n"
             "#pragma once\n"]
    parts.append(_vertex_arrays("pq_h1", tb.h1_sym))
    parts.append(_vertex_arrays("pq_h2", tb.h2_sym))
    parts.append(_arr("pq_swap2", "int", tb.swap2) + _arr("pq_swap2_sign", "double", tb.swap2_sign))
    c1, c2 = _pattern_counts()
    parts.append(_arr("pq_cnt1", "int", c1) + _arr("pq_cnt2", "int", c2))
    for name in ("E1", "E2", "R1S0", "R1S1", "R1S2", "R2S0", "R2S1"):
        parts.append(_class_arrays("pq_" + name.lower(), tb.classes[name]))
    parts.append(_spec_arrays("pq_x", tb.r2s1_x))
    parts.append(_spec_arrays("pq_y", tb.r2s1_y))
    parts.append(_arr("pq_s1pairs", "int", tb.r2s1_pairs.reshape(-1))
                 + f"#define PQ_S1PAIRS_N {len(tb.r2s1_pairs)}\n")
    # adjoint of the one-spectator GEMM, gathered per side: segments of at
    # most S1A_SEG pairs sharing x (the pair list is in (x, y) order) and, via
    # a permutation into (y, x) order, sharing y
    S1A_SEG = 32
    pr = [tuple(int(u) for u in q) for q in tb.r2s1_pairs]
    assert pr == sorted(pr)

    def segments(keys, size=S1A_SEG):
        starts = [0]
        for i in range(1, len(keys) + 1):
            if i == len(keys) or keys[i] != keys[starts[-1]] or i - starts[-1] == size:
                starts.append(i)
        return starts                       # segment j = [starts[j], starts[j + 1])

    ax = segments([q[0] for q in pr])
    perm = sorted(range(len(pr)), key=lambda i: (pr[i][1], pr[i][0]))
    ay = segments([pr[i][1] for i in perm])
    parts.append(_arr("pq_s1ax_p0", "int", ax) + _arr("pq_s1y_perm", "int", perm)
                 + _arr("pq_s1ay_i0", "int", ay)
                 + f"#define PQ_S1AX_N {len(ax) - 1}\n#define PQ_S1AY_N {len(ay) - 1}\n")
    # factorised one-pair two-spectator class: one spec table X | Y | Z
    nx, ny = len(tb.r1s2_x), len(tb.r1s2_y)
    parts.append(_spec_arrays("pq_r1f", tb.r1s2_x + tb.r1s2_y + tb.r1s2_z)
                 + f"#define PQ_R1F_Y0 {nx}\n#define PQ_R1F_Z0 {nx + ny}\n")
    nf = nx + ny + len(tb.r1s2_z)
    r_mid, r_gen, r_start, r_cl, r_coef, r_mu = [], [], [0], [], [], []
    for (zsel, side, gen), lst in tb.r1s2_groups:
        nz = len(tb.r1s2_z)
        # Z_z at F index Z0 + z; its transpose at nf + z
        r_mid.append(nx + ny + zsel if zsel < nz else nf + (zsel - nz))
        r_gen.append(gen if side == 0 else nx + gen)
        for cl, c, m in lst:
            r_cl.append(nx + cl if side == 0 else cl)
            r_coef.append(c)
            r_mu.append(m)
        r_start.append(len(r_cl))
    # transposed middle factor (k_bgemm computes M = G . (Mid^T)^T)
    r_midT = [(nx + ny + (m - nf)) if m >= nf else (nf + (m - nx - ny)) for m in r_mid]
    parts.append(_arr("pq_r1g_midT", "int", r_midT))
    parts.append(_arr("pq_r1g_mid", "int", r_mid) + _arr("pq_r1g_gen", "int", r_gen)
                 + _arr("pq_r1g_start", "int", r_start) + _arr("pq_r1g_cl", "int", r_cl)
                 + _arr("pq_r1g_coef", "double", r_coef) + _arr("pq_r1g_mu", "int", r_mu)
                 + f"#define PQ_R1G_N {len(r_mid)}\n")
    parts.append(_spec_arrays("pq_l", tb.r2s2_l))
    parts.append(_spec_arrays("pq_w", tb.r2s2_w))
    parts.append(_spec_arrays("pq_lam", tb.r2s2_lam or [[]]))
    parts.append(_arr("pq_dr_lam", "int", [li for li, _ in tb.r2s2_dress])
                 + _arr("pq_dr_w", "int", [w for _, w in tb.r2s2_dress])
                 + f"#define PQ_DR_N {len(tb.r2s2_dress)}\n")
    gw, ga, gs, gb, gc, gm = [], [], [0], [], [], []
    for (wi, ai), lst in tb.r2s2_groups:
        gw.append(wi)
        ga.append(ai)
        for bi, c, m in lst:
            gb.append(bi)
            gc.append(c)
            gm.append(m)
        gs.append(len(gb))
    parts.append(_arr("pq_g_w", "int", gw) + _arr("pq_g_a", "int", ga) + _arr("pq_g_start", "int", gs)
                 + _arr("pq_g_b", "int", gb) + _arr("pq_g_coef", "double", gc) + _arr("pq_g_mu", "int", gm)
                 + f"#define PQ_G_N {len(gw)}\n")
    # lane-per-pair chunks (their terms are generated code): output slots
    V = tb.r2_lane
    nout = [V["ch_slot0"][c + 1] - V["ch_slot0"][c] for c in range(len(V["ch_lo"]))]
    parts.append(_arr("pq_lane_ch_slot0", "int", V["ch_slot0"]) + _arr("pq_lane_m_slots", "int", V["m_slots"])
                 + _arr("pq_lane_m_slot_start", "int", V["m_slot_start"])
                 + f"#define PQ_LANE_NCHUNK {len(V['ch_lo'])}\n#define PQ_LANE_NLOC {LANE_NLOC}\n"
                 + f"#define PQ_LANE_NSLOT {len(V['slot_m'])}\n#define PQ_LANE_MAXOUT {max(nout)}\n"
                 + f"#define PQ_LANE_ONE {LANE_ONE}\n#define PQ_LANE_T2 {LANE_T2}\n")
    # link specs of the two-spectator sums, decoded: every factor is
    # t2[m][P or Q][spectator]; up to 3 factors
    ln, lm, lq = [], [], []
    for sp in tb.r2s2_l:
        assert len(sp) <= 3
        ln.append(len(sp))
        mm, qq = [0, 0, 0], [0, 0, 0]
        for f, code in enumerate(sp):
            assert (code >> 28) & 15 == KIND_T2 and (code >> 20) & 15 == 2
            mm[f] = code & 0xFFFF
            qq[f] = (code >> 24) & 15
        lm += mm
        lq += qq
    parts.append(_arr("pq_ld_n", "int", ln) + _arr("pq_ld_m", "int", lm) + _arr("pq_ld_q", "int", lq))
    for size in (1, 2, 3):
        q = eri_quads(size)
        parts.append(_arr(f"pqph_quads{size}", "int", [x for quad in q for x in quad])
                     + f"#define PQPH_QUADS{size}_N {len(q)}\n")
    maxlen = max(len(s) for s in tb.r2s1_x + tb.r2s1_y + tb.r2s2_l + tb.r2s2_w
                 + tb.r2s2_lam + tb.r1s2_x + tb.r1s2_y + tb.r1s2_z)
    parts.append(f"#define PQ_SPEC_MAXLEN {maxlen}\n")
    with open(path, "w") as fh:
        fh.write("\n".join(parts))


def main():
    import os
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "..", "csrc", "pq_tables.h")
    emit_pq_header(build_pq_tables(), out)


if __name__ == "__main__":
    main()
