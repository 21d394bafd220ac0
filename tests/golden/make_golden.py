"""Write the oracle's expected values for the full-size parity tests.

Calls only oracle/ and the seeded input generators.  Each fixture holds the
residual of a few sampled output blocks (by sub-cluster inclusion-exclusion,
Sec. II) and the correlation energy for the 140-site PPP chain (BASELINE
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

from inputs import chain_problem, random_amplitudes  # noqa: E402
from oracle import integrals, layout, tier_b  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

FIXTURES = {
    # name: (sites, U, chain seed, k, amplitude seed, amplitude scale, blocks)
    "pq140_blocks": (140, 4.0, 140, 2, 1400, 0.05, [(0,), (69,), (0, 1), (17, 52)]),
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
        vals = tb.residual_block(L, t)
        out["blocks"][",".join(map(str, L))] = {str(s): v for s, v in sorted(vals.items())}
        tb.clear()
        print(name, L, f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(FIXTURES)):
        make(nm)
