#!/usr/bin/env python3
"""Benchmark of the PQ hot path on one MI355X.

Step = one complete PQ solve of the 140-site PPP chain (140 electrons in 140
orbitals, 70 pairs; U = 4, seed 140): integral transformation into pair
blocks, Jacobi/DIIS iterations from t = 0 to ||R|| <= 1e-8 (each iteration one
residual evaluation, the norm check, the Jacobi update and the DIIS
extrapolation) and the final correlation energy.  Value = residual
evaluations per second over the timed steps.  The orbitals come from a
host-side RHF outside the timed region (input preparation, like the paper's
external SCF); all inputs are resident in HBM before timing starts.

Prints one JSON line (rank 0).  Also reported: the back-to-back residual rate
at the converged amplitudes, per-kernel HIP-event times, the roofline of the
dominant kernel, and the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from math import comb

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sites", type=int, default=140)
    ap.add_argument("--U", type=float, default=4.0)
    ap.add_argument("--seed", type=int, default=140)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--profile-reps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-ph", action="store_true", help="skip the PH (three-pair) leg")
    ap.add_argument("--ph-sites", type=int, default=40,
                    help="sites of the PH configuration's chain (one timed residual)")
    ap.add_argument("--ph-reps", type=int, default=1, help="PH residuals timed back to back")
    ap.add_argument("--ph-solve-sites", type=int, default=12,
                    help="sites of the chain the PH leg solves from t = 0")
    ap.add_argument("--ph-solve", action="store_true",
                    help="solve the --ph-sites chain itself (15 minutes at 40 sites)")
    ap.add_argument("--ph-only", action="store_true", help="run only the PH leg")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--counter-run", type=int, default=0,
                    help="only run this many 140-site residuals and a 256 MiB copy (for rocprofv3 --pmc)")
    ap.add_argument("--grad-sites", type=int, default=400)
    ap.add_argument("--integrals-run", type=int, default=0,
                    help="only run this many integral transforms at --sites (for rocprofv3)")
    return ap.parse_args()


def _time_subclusters(tb, t, N, seconds, rng_seed):
    """Mean seconds per sub-cluster evaluation of each size (1..4 pairs),
    timed over random sub-clusters for a share of `seconds`."""
    import numpy as np
    rng = np.random.default_rng(rng_seed)
    per, nsamp = {}, {}
    budget = {1: 0.05, 2: 0.1, 3: 0.25, 4: 0.6}
    for s in (1, 2, 3, 4):
        tb.engine(s)                       # build the template outside timing
        n, t0 = 0, time.perf_counter()
        while True:
            Y = tuple(sorted(rng.choice(N, s, replace=False).tolist()))
            tb.clear()
            tb.sub_residual(Y, t)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget[s] * seconds or n >= 100000:
                break
        per[s] = el / n
        nsamp[s] = n
    return per, nsamp


def _pool_worker(args):
    from threadpoolctl import threadpool_limits
    seconds, seed = args
    with threadpool_limits(limits=1):
        per, nsamp = _time_subclusters(_POOL["tb"], _POOL["t"], _POOL["N"], seconds, seed)
    return per, nsamp


_POOL = {}


def cpu_baseline(prob, seconds: float):
    """The oracle as it stands (sub-cluster inclusion-exclusion over the
    definitional determinant-space evaluation), timed on a bounded sample,
    on one core and on every core of the process's affinity set.

    A full residual needs every sub-cluster of at most 4 pairs once (the
    oracle evaluates each once): C(N,s) evaluations of size s.  The sample
    times random sub-clusters of each size and scales by those counts; with
    all cores, one worker process per core times its own sample and the rate
    is the sum of the workers' rates.
    """
    import multiprocessing as mp
    import platform

    from threadpoolctl import threadpool_limits

    from inputs import random_amplitudes
    from oracle import integrals, tier_b

    N = prob.npair
    f, eri = integrals.chain_integrals(prob, 2)
    t = random_amplitudes(N, "pq", seed=1400, scale=0.05)
    tb = tier_b.TierB(N, 2, f, eri)
    with threadpool_limits(limits=1):
        per, nsamp = _time_subclusters(tb, t, N, seconds, 0)
    total = sum(comb(N, s) * per[s] for s in per)
    cores = min(16, len(os.sched_getaffinity(0)))     # the process's CPU share
    _POOL.update(tb=tb, t=t, N=N)
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_pool_worker, [(seconds, 1 + w) for w in range(cores)])
    rate_all = sum(1.0 / sum(comb(N, s) * p[s] for s in p) for p, _ in res)
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": rate_all, "unit": "residual evals/s", "cores": cores, "kind": "oracle",
            "sample": ("timed random sub-clusters of 1/2/3/4 pairs of the same chain and "
                       "amplitudes (%s on one core); one residual = C(70,s) sub-clusters of each "
                       "size s; all cores: %d worker processes, each timing its own sample of "
                       "~%.0f s, rates summed" % ("/".join(str(nsamp[s]) for s in (1, 2, 3, 4)),
                                                  cores, seconds)),
            "single_core_value": 1.0 / total, "single_core_seconds_per_residual": total,
            "cpu_model": model, "affinity_cores": cores,
            "seconds_per_subcluster": {str(s): per[s] for s in per}}


def ph_leg(args, pq, torch, dev):
    """PH (three-pair) model.  The configuration's chain (--ph-sites, 40
    sites = 20 pairs): one residual at seeded amplitudes (scale 0.05), timed
    with HIP events on the library's stream (a solve of this chain takes ~25
    residuals, 15 minutes: it is run on its own with --ph-only --ph-solve).
    And a full solve from t = 0 of a smaller chain (--ph-solve-sites, integral
    transform included)."""
    from inputs import chain_problem, random_amplitudes
    d = lambda x: torch.as_tensor(x, device=dev).contiguous()
    small = chain_problem(6, U=args.U, seed=6)                  # loads the term tables
    fs, es = pq.integrals(d(small.F_site), d(small.V), d(small.C), k=3)
    pq.ph_residual(fs, es, torch.zeros(pq.amp_len(3, "ph"), dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    out = {}
    prob = chain_problem(args.ph_sites, U=args.U, seed=args.ph_sites)
    N = prob.npair
    f, eri = pq.integrals(d(prob.F_site), d(prob.V), d(prob.C), k=3)
    t = d(random_amplitudes(N, "ph", seed=100 * args.ph_sites, scale=0.05))
    r = torch.empty_like(t)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.ph_reps):
        pq.ph_residual(f, eri, t, out=r)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.ph_reps
    nev, nfl = ph_term_evals(N)
    ach = nfl / (ms * 1e-3) / 1e12
    out["residual"] = {
        "workload": f"one PH residual of the {args.ph_sites}-site PPP chain ({N} pairs, U={args.U}, "
                    f"seed {args.ph_sites}) at seeded amplitudes", "amplitudes": pq.amp_len(N, "ph"),
        "residual_ms": ms, "residual_evals_per_s": 1e3 / ms,
        "term_evals_per_residual": nev, "term_evals_per_s": nev / (ms * 1e-3),
        "roofline": {"bound": "alu", "kernel": "k_ph_part", "achieved": ach,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": ach / 78.6,
                     "flops_per_launch": nfl,
                     "note": "interpreted work: one multiply per factor and one add per evaluated "
                             "term; the kernel is bound by its dependent table gathers"}}
    # the same residual at spin-symmetric amplitudes, as the spin-adapted solve
    # evaluates it (orbit representatives only): one iteration of that solve
    # from t = 0 (the interpreted work does not depend on the amplitude values)
    one = pq.ph_solve(f, eri, max_iter=1, diis_dim=0, spin_adapted=1, raise_on_failure=False)
    out["residual"]["spin_symmetric_solve_iteration_ms"] = one.solve_ms
    if args.ph_solve or args.ph_solve_sites != args.ph_sites:
        sites = args.ph_sites if args.ph_solve else args.ph_solve_sites
        sp = chain_problem(sites, U=args.U, seed=sites)
        for spin in ((1,) if args.ph_solve else (0, 1)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f, eri = pq.integrals(d(sp.F_site), d(sp.V), d(sp.C), k=3)
            res = pq.ph_solve(f, eri, tol=args.tol, spin_adapted=spin)
            torch.cuda.synchronize()
            out["solve_spin_adapted" if spin else "solve"] = {
                "workload": f"PH solve of a {sites}-site PPP chain ({sp.npair} pairs, "
                            f"U={args.U}, seed {sites}) from t=0 to ||R||<={args.tol:g}, "
                            "integral transform included" + (", closed-shell spin adaptation" if spin else ""),
                "solve_s": time.perf_counter() - t0, "iterations": res.iterations,
                "energy": res.energy, "status": res.status}
            print(f"ph solve {sites} sites spin_adapted={spin}: {time.perf_counter() - t0:.1f} s, "
                  f"{res.iterations} iterations, E = {res.energy:.12f}", file=sys.stderr, flush=True)
    return out


def ph_term_evals(N):
    """(term, ordered spectator tuple) evaluations of one PH residual, the
    work the interpreted kernels do, and its flops (one multiply per factor
    and one add per evaluation), counted from the term-table file."""
    from math import comb, perm

    import numpy as np

    from paper_1609_00077_amd.derive import ph_tables
    raw = ph_tables.read(os.path.join(ROOT, "paper_1609_00077_amd", "ph_terms.bin"))
    a = np.frombuffer(raw, dtype="<i4")
    nclass, nterm, ncw = int(a[2]), int(a[5]), int(a[6])
    pos, classes = 8, []
    for _ in range(nclass):
        nout, nspec, nt, off, npat = (int(x) for x in a[pos:pos + 5])
        classes.append((nout, nspec, off, a[pos + 5:pos + 6 + npat]))
        pos += 6 + npat
    cw_dict = a[pos:pos + ncw]
    nslot = int(a[7])
    byte = 4 * (pos + ncw + nslot) + (2 * nterm + 3) // 4 * 4      # past slot_dict and h
    cw = cw_dict[np.frombuffer(raw, dtype="<u1", count=nterm, offset=byte)]
    fl_term = (cw >> 16) + 1                                     # factors + 1 per evaluation
    cum = np.concatenate([[0], np.cumsum(fl_term, dtype=np.int64)])
    # the canonical map sits just before the integral map at the end of the file
    canon = a[len(a) - 3 * 1296 - 335:len(a) - 3 * 1296]
    tot = fl = 0
    for n in (1, 2, 3):
        if n > N:
            continue
        base = (0, 3, 32)[n - 1]
        for m in range((3, 29, 303)[n - 1]):
            mc = int(canon[base + m]) & 511
            for nout, nspec, off, start in classes:
                if nout == n and nspec <= N - n:
                    mult = perm(N - n, nspec) * comb(N, n)
                    q0, q1 = off + int(start[mc]), off + int(start[mc + 1])
                    tot += (q1 - q0) * mult
                    fl += int(cum[q1] - cum[q0]) * mult
    return tot, float(fl)


def batch_leg(args, pq, torch, dev):
    """Batched PQ config: chains with pair counts drawn from 10..120 (seeded),
    U from 2..6; RHF and integrals outside the timed region.  One batched
    solve (graph-replayed device-resident iterations, and the host-driven
    lockstep for comparison) vs the same solves one after another.  Every
    chain ends with a status (converged, diverged, stalled); all count as
    solves."""
    from collections import Counter

    from inputs import batch_chain_specs, batch_problems
    specs = batch_chain_specs(args.batch, 256)
    probs = batch_problems(specs, processes=min(16, os.cpu_count() or 1))
    hs, es = [], []
    for p in probs:
        d = lambda x: torch.as_tensor(x, device=dev).contiguous()
        f, e = pq.integrals(d(p.F_site), d(p.V), d(p.C), k=2)
        hs.append(f)
        es.append(e)
    torch.cuda.synchronize()
    out = {}
    for mode in ("graph", "lockstep"):
        pq.pq_solve_batched(hs[:8], es[:8], tol=args.tol, mode=mode)      # warm-up of the code paths
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = pq.pq_solve_batched(hs, es, tol=args.tol, mode=mode)
        torch.cuda.synchronize()
        out[mode] = (time.perf_counter() - t0, res)
    t0 = time.perf_counter()
    seq = [pq.pq_solve(f, e, tol=args.tol, raise_on_failure=False) for f, e in zip(hs, es)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    tb, res = out["graph"]
    tl, resl = out["lockstep"]
    ok = [i for i, s in enumerate(res.statuses) if s == "OK"]
    from paper_1609_00077_amd import workmodel
    fl = sum(sum(workmodel.pq_kernel_flops(p.npair).values()) * it
             for p, it in zip(probs, res.iterations))
    ach = fl / tb / 1e12
    return {"batched_solves_per_s": len(hs) / tb, "lockstep_solves_per_s": len(hs) / tl,
            "batched_converged_solves_per_s": len(ok) / tb,
            "sequential_converged_solves_per_s":
                sum(1 for r in seq if r.status == "OK") / ts,
            "roofline": {"bound": "alu", "achieved": ach, "peak": workmodel.PEAK_FP64_VECTOR_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / workmodel.PEAK_FP64_VECTOR_TFLOPS,
                         "note": "residual flops of every chain's iterations over the batched wall time"},
            "sequential_solves_per_s": len(hs) / ts, "batched_speedup": ts / tb,
            "batch_size": len(hs), "batch_statuses": dict(Counter(res.statuses)),
            "sequential_statuses": dict(Counter(r.status for r in seq)),
            "batch_total_pairs": sum(p.npair for p in probs),
            "batch_residual_evals": sum(res.iterations),
            "sequential_residual_evals": sum(r.iterations for r in seq),
            "batch_max_energy_diff_vs_sequential_converged":
                max((abs(res.energies[i] - seq[i].energy) for i in ok), default=None),
            "lockstep_max_energy_diff_vs_graph_converged":
                max((abs(res.energies[i] - resl.energies[i]) for i in ok), default=None)}


def grad_leg(args, pq, torch, dev):
    """PQ energy + adjoint gradient config: a 400-site chain (200 pairs).
    Times the energy alone (integrals given; solve from t = 0) and the energy
    with dE/dh and dE/d(eri) (the same solve, the lambda equations and the
    transposed contraction), on the stream, after one warm-up of each."""
    from inputs import chain_problem
    prob = chain_problem(args.grad_sites, U=4.0, seed=args.grad_sites)
    d = lambda x: torch.as_tensor(x, device=dev).contiguous()
    f, eri = pq.integrals(d(prob.F_site), d(prob.V), d(prob.C), k=2)
    pq.pq_solve(f, eri, tol=args.tol)
    pq.pq_energy_grad(f, eri, tol=args.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = pq.pq_solve(f, eri, tol=args.tol)
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = pq.pq_energy_grad(f, eri, tol=args.tol)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    from paper_1609_00077_amd import workmodel
    F = sum(workmodel.pq_kernel_flops(prob.npair).values())
    # t iterations: one residual each; lambda iterations: one transposed
    # contraction each, counted as twice the forward flops (the reverse of a
    # contraction forms both operand adjoints); the final VJP with the
    # Hamiltonian adjoints likewise, plus the forward it recomputes once
    fl = F * res.iterations + 2.0 * F * (g.iterations + 1) + F
    ach = fl / tg / 1e12
    return {"sites": args.grad_sites, "pairs": prob.npair, "energy": res.energy,
            "roofline": {"bound": "alu", "achieved": ach, "peak": workmodel.PEAK_FP64_VECTOR_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / workmodel.PEAK_FP64_VECTOR_TFLOPS,
                         "note": "energy + gradient: counted residual and adjoint flops over its wall time"},
            "energy_s": te, "energy_grad_s": tg, "grad_energy_ratio": tg / te,
            "t_iterations": res.iterations, "lambda_iterations": g.iterations,
            "grad_status": g.status,
            "homogeneity_residual": abs(float(torch.sum(g.dE_dh * f) + torch.sum(g.dE_deri * eri))
                                        - g.energy)}


COUNTERS = os.path.join(ROOT, "profiles", "pq_residual_counters_pq140.json")
# dense contractions on the FP64 matrix cores (peak 78.6 TFLOP/s, the same as FP64 vector)
MFMA_KERNELS = {"k_gemm_s1", "k_r2s2"}


def source_hash() -> str:
    """Hash of the kernel sources and generated-table inputs: counters taken
    from an older build do not describe the current kernels."""
    import hashlib
    h = hashlib.sha256()
    for sub in ("paper_1609_00077_amd/csrc", "paper_1609_00077_amd/derive"):
        d = os.path.join(ROOT, sub)
        for name in sorted(os.listdir(d)):
            generated = name.startswith(("pq_tables", "pq_lane_code", "pq_lane_adj_code"))
            if name.endswith((".hip", ".h", ".py")) and not generated:
                with open(os.path.join(d, name), "rb") as fh:
                    h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def kernel_variant(phase: str, N: int, tuning: dict) -> str:
    """The kernel a residual phase launches under the tuning in effect (the
    counters are keyed by it: variants move different bytes)."""
    ncb = (N + 15) // 16
    if phase == "k_gemm_s1":
        even = "true" if N % 2 == 0 else "false"
        return {1: "k_gemm_s1<true>", 2: "k_gemm_s1<false>", 3: f"k_gemm_s1p<{ncb}>",
                4: f"k_gemm_s1m<{ncb}, {even}>"}[tuning["s1_mode"]]
    if phase == "k_r2s2":
        if tuning["s2_variant"] == 2:
            return f"k_r2s2w<{ncb}>"
        nb = next(b for b in (1, 2, 3, 4, 5, 6, 8, 10, 13, 16) if ncb <= b)
        return f"k_r2s2<{nb}>"
    return phase


def hbm_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE and
    WRITE_SIZE counter runs, each scaled by the same counter's reading for a
    copy of known size; None when absent or taken on other sources."""
    if not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as fh:
        c = json.load(fh)
    if c.get("source_hash") != source_hash() or kernel not in c.get("kernels", {}):
        return None
    k = c["kernels"][kernel]
    return 1024.0 * (k["fetch_kib"] * c["fetch_scale"] + k["write_kib"] * c["write_scale"])


def densities_leg(pq, torch, dev, sites):
    """Densities and natural occupations of the benchmark chain: one
    pq_densities call from t = 0 (solve, lambda, densities) after a warm-up."""
    from inputs import chain_problem
    prob = chain_problem(sites, U=4.0, seed=sites)
    d = lambda x: torch.as_tensor(x, device=dev).contiguous()
    f, eri = pq.integrals(d(prob.F_site), d(prob.V), d(prob.C), k=2)
    pq.pq_densities(f, eri, tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = pq.pq_densities(f, eri, tol=1e-8)
    torch.cuda.synchronize()
    N = prob.npair
    return {"sites": sites, "seconds": time.perf_counter() - t0, "status": r.status,
            "trace_gamma": float(torch.trace(r.gamma)),
            "noons_around_gap": [round(x, 6) for x in r.noons[N - 4:N + 4]],
            "noon_min_max": [min(r.noons), max(r.noons)]}


def integrals_leg(pq, torch, dev, sites, reps=10):
    """Integral transformation into pair blocks at one chain size: HIP-event
    time per transform on the current stream and its MFMA roofline.  Work:
    Y = V X over every orbital pair (2 n^2 n(n+1)/2 flop) and f = C^T F C
    (2 x 2 n^3), both on the FP64 matrix cores; the packing dots are
    2 n per stored integral."""
    from inputs import chain_problem
    from paper_1609_00077_amd import workmodel
    prob = chain_problem(sites, U=4.0, seed=sites)
    d = lambda x: torch.as_tensor(x, device=dev).contiguous()
    F, V, Cm = d(prob.F_site), d(prob.V), d(prob.C)
    for _ in range(2):
        pq.integrals(F, V, Cm, k=2)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        pq.integrals(F, V, Cm, k=2)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    fl = workmodel.integral_flops(prob.npair)
    ach = fl / (ms * 1e-3) / 1e12
    return {"sites": sites, "ms": ms, "flops": fl,
            "roofline": {"bound": "mfma", "achieved": ach, "peak": workmodel.PEAK_FP64_VECTOR_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / workmodel.PEAK_FP64_VECTOR_TFLOPS}}


def counter_run(args, pq, torch, dev):
    from inputs import chain_problem, random_amplitudes
    prob = chain_problem(args.sites, U=args.U, seed=args.seed)
    d = lambda x: torch.as_tensor(x, device=dev).contiguous()
    f, eri = pq.integrals(d(prob.F_site), d(prob.V), d(prob.C), k=2)
    t = d(random_amplitudes(prob.npair, "pq", seed=1400, scale=0.05))
    r = torch.empty_like(t)
    N = prob.npair
    # every kernel choice the autotuner can make, counter_run residuals each
    for variant in ((1, 2) if (N + 15) // 16 <= 6 else (1,)):
        for mode in ((1, 2, 3, 4) if N <= 128 else (1, 2, 4)):
            pq.set_variant(N, variant)
            pq.set_s1_mode(N, mode)
            for _ in range(args.counter_run):
                pq.pq_residual(f, eri, t, out=r)
    pq.set_variant(N, 0)
    pq.set_s1_mode(N, 0)
    torch.cuda.synchronize()
    a = torch.full((32 * 1024 * 1024,), 1.0, dtype=torch.float64, device=dev)   # 256 MiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counter_run": args.counter_run, "copy_bytes": a.numel() * 8,
                      "source_hash": source_hash()}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1609_00077_amd as pq
    from paper_1609_00077_amd import workmodel
    from inputs import chain_problem

    dev = torch.device("cuda:0")
    if args.counter_run:
        return counter_run(args, pq, torch, dev)
    if args.integrals_run:
        print(json.dumps(integrals_leg(pq, torch, dev, args.sites, args.integrals_run)), flush=True)
        return
    if args.ph_only:
        print(json.dumps({"ph": ph_leg(args, pq, torch, dev)}), flush=True)
        return
    prob = chain_problem(args.sites, U=args.U, seed=args.seed)
    N = prob.npair
    F = torch.as_tensor(prob.F_site, device=dev).contiguous()
    V = torch.as_tensor(prob.V, device=dev).contiguous()
    Cm = torch.as_tensor(prob.C, device=dev).contiguous()
    torch.cuda.synchronize()

    def step():
        f, eri = pq.integrals(F, V, Cm, k=2)
        return pq.pq_solve(f, eri, tol=args.tol), f, eri

    # autotune the kernel variants for this size on the first Hamiltonian
    f0, eri0 = pq.integrals(F, V, Cm, k=2)
    variant = pq.autotune(f0, eri0, pq.pq_solve(f0, eri0, tol=1e-6).t)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    iters = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, f, eri = step()
        iters += res.iterations
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    value = iters / T
    # the same solves with the Jacobi/DIIS decisions on the device (opt-in mode)
    pq.set_solve_mode("device")
    step()
    torch.cuda.synchronize()
    iters_dev = 0
    t1 = time.perf_counter()
    for _ in range(args.steps):
        iters_dev += step()[0].iterations
    torch.cuda.synchronize()
    value_dev = iters_dev / (time.perf_counter() - t1)
    pq.set_solve_mode("host")

    # back-to-back residuals at the converged amplitudes (HIP events on the stream)
    t_conv = res.t
    r = torch.empty_like(t_conv)
    nrep = 20
    for _ in range(3):
        pq.pq_residual(f, eri, t_conv, out=r)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(nrep):
        pq.pq_residual(f, eri, t_conv, out=r)
    ev1.record()
    torch.cuda.synchronize()
    resid_ms = ev0.elapsed_time(ev1) / nrep

    # per-kernel times: events recorded by the library on its own stream
    acc = {}
    for _ in range(args.profile_reps):
        _, phases = pq.pq_residual_profile(f, eri, t_conv)
        for name, ms in phases:
            acc[name] = acc.get(name, 0.0) + ms / args.profile_reps
    flops = workmodel.pq_kernel_flops(N)
    dom = max(acc, key=acc.get)
    achieved = flops[dom] / (acc[dom] * 1e-3) / 1e12
    peak = workmodel.PEAK_FP64_VECTOR_TFLOPS
    line = {
        "metric": "PQ residual evals/s at 140e/140o",
        "value": value,
        "unit": "residual evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"PQ solve of a {args.sites}-site PPP chain ({N} pairs, "
                               f"U={args.U}, seed {args.seed}) from t=0 to ||R||<={args.tol:g}, "
                               "integral transform included", "sites": args.sites, "pairs": N,
                   "iterations_per_solve": res.iterations, "energy": res.energy,
                   "s2_variant": variant, "s1_mode": pq.tuning(N)["s1_mode"]},
        "roofline": {"bound": "mfma" if dom in MFMA_KERNELS else "alu", "kernel": kernel_variant(dom, N, pq.tuning(N)),
                     "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": hbm_traffic(kernel_variant(dom, N, pq.tuning(N))),
                     "flops_per_launch": flops[dom], "ms_per_launch": acc[dom]},
        "device_driven_solve_evals_per_s": value_dev,
        "residual_ms": resid_ms,
        "residual_evals_per_s_back_to_back": 1e3 / resid_ms,
        "residual_flops": sum(flops.values()),
        "residual_tflops": sum(flops.values()) / (resid_ms * 1e-3) / 1e12,
        "residual_compulsory_bytes": workmodel.pq_compulsory_bytes(N),
        "kernel_ms": acc,
    }
    line["integrals"] = {str(n): integrals_leg(pq, torch, dev, n) for n in (args.sites, args.grad_sites)}
    ceil = pq.measure_ceilings()
    line["ceilings_measured"] = ceil
    line["roofline"]["frac_of_measured_peak"] = achieved / ceil["fp64_mfma_TFLOPs"]
    # the two-pair-intermediate variant (doubly-mixed two-spectator terms left out)
    pq.set_pq_intermediates(N, 2)
    for _ in range(3):
        pq.pq_residual(f, eri, t_conv, out=r)
    ev0.record()
    for _ in range(nrep):
        pq.pq_residual(f, eri, t_conv, out=r)
    ev1.record()
    torch.cuda.synchronize()
    ms2 = ev0.elapsed_time(ev1) / nrep
    e2 = pq.pq_solve(f, eri, tol=args.tol).energy
    pq.set_pq_intermediates(N, 3)
    line["pq_two_pair_intermediates"] = {"residual_ms": ms2, "residual_evals_per_s": 1e3 / ms2,
                                         "energy": e2, "energy_exact_model": res.energy}
    if not args.no_grad:
        line["energy_gradient"] = grad_leg(args, pq, torch, dev)
        line["densities"] = densities_leg(pq, torch, dev, args.sites)
    if not args.no_batch:
        line["batched"] = batch_leg(args, pq, torch, dev)
    if not args.no_ph:
        line["ph"] = ph_leg(args, pq, torch, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
