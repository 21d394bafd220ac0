"""Write the oracle's expected values for the full-size parity tests.

Calls only oracle/ and the seeded input generators.  Each fixture holds the
residual of a few sampled output blocks (by sub-cluster inclusion-exclusion,
Sec. II) and the correlation energy for the 140-site PPP chain (the benchmark
workload: 140 electrons in 140 orbitals, 70 pairs) at seeded amplitudes.

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from inputs import chain_problem, random_amplitudes, random_vector  # noqa: E402
from oracle import gradient, integrals, layout, tier_b  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

WORKERS = min(8, os.cpu_count() or 1)

FIXTURES = {
    # name: (sites, U, chain seed, k, amplitude seed, amplitude scale, blocks)
    "pq140_blocks": (140, 4.0, 140, 2, 1400, 0.05, [(0,), (69,), (0, 1), (17, 52)]),
    # the same amplitudes; blocks at the ragged edges of the 16-wide pair tiles
    # (labels 64..69) and of the last 64-row block of pair indices (2368..2414)
    "pq140_edges": (140, 4.0, 140, 2, 1400, 0.05,
                    [(63,), (64,), (15, 16), (63, 64), (64, 65), (68, 69), (0, 69), (3, 68),
                     (64, 69)]),
    # 40-site chain, three-pair model: one- and two-pair output blocks (their
    # sub-systems have at most four and five pairs)
    "ph40_blocks": (40, 4.0, 40, 3, 4000, 0.05, [(0,), (7,), (19,), (0, 19), (18, 19)]),
}


def make(name):
    n, U, seed, k, aseed, scale, blocks = FIXTURES[name]
    prob = chain_problem(n, U=U, seed=seed)
    N = prob.npair
    f, eri = integrals.chain_integrals(prob, k)
    t = random_amplitudes(N, "pq" if k == 2 else "ph", seed=aseed, scale=scale)
    tb = tier_b.TierB(N, k, f, eri)
    out = {"sites": n, "U": U, "seed": seed, "k": k, "amp_seed": aseed, "amp_scale": scale,
           "citation": "R_mu = <mu|e^-T H_k e^T|0> (Sec. II, Eq. (1)); sub-cluster sum of the oracle",
           "blocks": {}}
    t0 = time.time()
    out["energy"] = tb.energy(t)
    for L in blocks:
        vals = tb.residual_block(L, t, workers=WORKERS)
        out["blocks"][",".join(map(str, L))] = {str(s): v for s, v in sorted(vals.items())}
        tb.clear()
        print(name, L, f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)


VJP_FIXTURES = {
    # name: (sites, U, chain seed, amplitude seed, scale, lambda seed, direction seed,
    #        energy weight, blocks carrying lambda)
    "pq140_vjp": (140, 4.0, 140, 1400, 0.05, 1401, 1402, 0.7, [(3,), (0, 1), (17, 52)]),
}


def vjp_inputs(N, lseed, dseed, blocks):
    """lambda on the slots of the given blocks, and the directions (dt, df, deri)."""
    lam_blocks = {}
    for b, L in enumerate(blocks):
        nslot = len(layout.pattern_tuples(len(L)))
        vals = random_vector(nslot, seed=lseed + b)
        lam_blocks[L] = {layout.amp_slot(N, L, m): float(vals[m]) for m in range(nslot)}
    dt = random_vector(layout.amp_count(N, 2), seed=dseed)
    df = random_vector(4 * N * N, seed=dseed + 1).reshape(2 * N, 2 * N)
    deri = random_vector(layout.eri_count(N, 2), seed=dseed + 2)
    return lam_blocks, dt, df, deri


def _directional(a):
    N, f, eri, t, lam_blocks, w, dirs = a
    return gradient.directional_vjp_blocks(N, 2, f, eri, t, lam_blocks, w, *dirs)


def make_vjp(name):
    n, U, seed, aseed, scale, lseed, dseed, w, blocks = VJP_FIXTURES[name]
    prob = chain_problem(n, U=U, seed=seed)
    N = prob.npair
    f, eri = integrals.chain_integrals(prob, 2)
    t = random_amplitudes(N, "pq", seed=aseed, scale=scale)
    lam_blocks, dt, df, deri = vjp_inputs(N, lseed, dseed, blocks)
    t0 = time.time()
    out = {"sites": n, "U": U, "seed": seed, "amp_seed": aseed, "amp_scale": scale,
           "lambda_seed": lseed, "direction_seed": dseed, "energy_weight": w,
           "blocks": [list(L) for L in blocks],
           "citation": "d/ds [lambda . R + w E_c] along (dt, df, deri): the transposed residual "
                       "contraction of the Lagrangian (Sec. II); sub-cluster sums of the oracle",
           "parts": {}}
    zt, zf, ze = np.zeros_like(dt), np.zeros_like(df), np.zeros_like(deri)
    parts = (("t", (dt, zf, ze)), ("f", (zt, df, ze)), ("eri", (zt, zf, deri)))
    args = [(N, f, eri, t, lam_blocks, w, dirs) for _, dirs in parts]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(len(parts)) as pool:
        vals = pool.map(_directional, args)
    for (part, _), v in zip(parts, vals):
        out["parts"][part] = v
    print(name, f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)


FULL_FIXTURES = {
    # name: (sites, U, chain seed, amplitude seed, amplitude scale)
    # 33 pairs: three 16-wide pair tiles with a ragged last one, and 528 pairs
    # of labels = eight full 64-row blocks and a ragged ninth
    "pq66_full": (66, 4.0, 66, 660, 0.05),
}


def make_full(name):
    n, U, seed, aseed, scale = FULL_FIXTURES[name]
    prob = chain_problem(n, U=U, seed=seed)
    N = prob.npair
    f, eri = integrals.chain_integrals(prob, 2)
    t = random_amplitudes(N, "pq", seed=aseed, scale=scale)
    tb = tier_b.TierB(N, 2, f, eri)
    t0 = time.time()
    R = tb.residual_all(t, workers=WORKERS)
    out = {"sites": n, "U": U, "seed": seed, "amp_seed": aseed, "amp_scale": scale,
           "citation": "R_mu = <mu|e^-T H_2 e^T|0> (Sec. II, Eq. (1)); every packed slot by "
                       "sub-cluster inclusion-exclusion of the oracle",
           "energy": tb.energy(t), "residual": [float(x) for x in R]}
    print(name, f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh)


PH_FIXTURES = {
    # name: (sites, U, chain seed, amplitude seed, amplitude scale)
    # 6 pairs: the first size where outputs on three pairs have three
    # spectators, so every PH class contributes
    "ph12_full": (12, 4.0, 12, 1200, 0.05),
}


def make_ph_full(name):
    from oracle import tier_a
    n, U, seed, aseed, scale = PH_FIXTURES[name]
    prob = chain_problem(n, U=U, seed=seed)
    N = prob.npair
    f, eri = integrals.chain_integrals(prob, 3)
    t = random_amplitudes(N, "ph", seed=aseed, scale=scale)
    t0 = time.time()
    R, E = tier_a.TierA(N, 3).residual(f, layout.unpack_eri(eri, N, 3), t)
    out = {"sites": n, "U": U, "seed": seed, "amp_seed": aseed, "amp_scale": scale,
           "citation": "R_mu = <mu|e^-T H_3 e^T|0> on the three-pair manifold (Sec. II); "
                       "definitional oracle (determinant space), every packed slot",
           "energy": float(E), "residual": [float(x) for x in R]}
    print(name, f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(FIXTURES) + list(VJP_FIXTURES) + list(PH_FIXTURES)
               + list(FULL_FIXTURES)):
        if nm in PH_FIXTURES:
            make_ph_full(nm)
        elif nm in FULL_FIXTURES:
            make_full(nm)
        else:
            (make_vjp if nm in VJP_FIXTURES else make)(nm)
