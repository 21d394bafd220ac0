"""GPU parity of the adjoint path: the transposed residual contraction
(pq_vjp), the lambda solve and the energy gradient (pq_energy_grad) and the
autograd Function, against the oracle's complex-step derivatives of the
definitional residual (Sec. II: the Lagrangian with de-excitation amplitudes
truncated like t).

Tolerances: the adjoint kernels sum the same O(1e4) products per output as
the forward ones, in a different order and with FP64 atomics, so element-wise
agreement is bounded like the forward residual (1e-12 relative to the largest
entry); complex-step values are exact to rounding.  Gradients through the
lambda solve add the solve tolerance (1e-12 in ||R||) amplified by the
conditioning of J, hence 1e-9."""
import itertools
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs import (chain_problem, random_amplitudes, random_bfactors, random_fock,  # noqa: E402
                    random_vector)
from oracle import gradient, layout, solver, tier_a  # noqa: E402
from oracle import integrals as oint  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pq():
    import paper_1609_00077_amd as pq
    pq._lib.load()
    return pq


def _d(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _system(N, seed):
    f = random_fock(N, seed=seed, offdiag=0.05)
    eri = oint.eri_packed_from_b(random_bfactors(N, seed=seed + 1, scale=0.2), N, 2)
    return f, eri


def _close(got, ref, rel):
    err = np.abs(np.asarray(got) - np.asarray(ref)).max()
    assert err <= rel * max(1.0, np.abs(ref).max()), err


@pytest.mark.parametrize("N", [1, 2, 3])
def test_vjp_elementwise_matches_oracle(pq, N):
    f, eri = _system(N, 300 + N)
    t = random_amplitudes(N, seed=310 + N, scale=0.1)
    lam = random_vector(len(t), seed=320 + N)
    w = 0.7
    tb_ref, hb_ref, eb_ref = gradient.vjp(N, 2, f, eri, t, lam, w)
    tb, hb, eb = pq.pq_vjp(_d(f), _d(eri), _d(t), _d(lam), w)
    _close(tb.cpu().numpy(), tb_ref, 1e-12)
    _close(hb.cpu().numpy(), hb_ref, 1e-12)
    _close(eb.cpu().numpy(), eb_ref, 1e-12)
    # tbar alone (no Hamiltonian adjoint) is the same vector
    tb2, h2, e2 = pq.pq_vjp(_d(f), _d(eri), _d(t), _d(lam), w, with_hamiltonian=False)
    assert h2 is None and e2 is None
    _close(tb2.cpu().numpy(), tb_ref, 1e-12)


def _all_blocks(N, lam):
    blocks = {}
    for size in (1, 2):
        for L in itertools.combinations(range(N), size):
            slots = [layout.amp_slot(N, L, m) for m in range(len(layout.pattern_tuples(size)))]
            blocks[L] = {s: float(lam[s]) for s in slots}
    return blocks


@pytest.mark.parametrize("N", [4, 6, 9])
def test_vjp_directional_matches_oracle(pq, N):
    """Larger N (every kernel class from N = 4 on; odd N = 9): each of the
    three adjoints dotted with a random direction (at N = 9 their sum, to
    keep the oracle's time down) equals the oracle's one-step complex
    derivative of lam . R + w E_c."""
    f, eri = _system(N, 400 + N)
    t = random_amplitudes(N, seed=410 + N, scale=0.08)
    lam = random_vector(len(t), seed=420 + N)
    w = -0.4
    tb, hb, eb = pq.pq_vjp(_d(f), _d(eri), _d(t), _d(lam), w)
    tb, hb, eb = tb.cpu().numpy(), hb.cpu().numpy(), eb.cpu().numpy()
    dt = random_vector(len(t), seed=430 + N)
    df = random_vector(4 * N * N, seed=431 + N).reshape(2 * N, 2 * N)
    de = random_vector(len(eri), seed=432 + N)
    blocks = _all_blocks(N, lam)
    zt, zf, ze = np.zeros_like(dt), np.zeros_like(df), np.zeros_like(de)
    cases = [(tb @ dt, (dt, zf, ze)), (np.sum(hb * df), (zt, df, ze)), (eb @ de, (zt, zf, de))]
    if N > 6:
        cases = [(tb @ dt + np.sum(hb * df) + eb @ de, (dt, df, de))]
    for got, dirs in cases:
        ref = gradient.directional_vjp_blocks(N, 2, f, eri, t, blocks, w, *dirs, keep_cache=True)
        assert abs(got - ref) <= 1e-11 * max(1.0, abs(ref)), (got, ref)


def test_vjp_full_size_sampled_blocks(pq):
    """140-site chain (70 pairs): lambda on sampled output blocks, directional
    derivatives stored by tests/golden/make_golden.py from the oracle."""
    p = os.path.join(os.path.dirname(__file__), "golden", "pq140_vjp.json")
    if not os.path.exists(p):
        pytest.skip("golden fixture pq140_vjp not generated (tests/golden/make_golden.py)")
    with open(p) as fh:
        g = json.load(fh)
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import vjp_inputs
    prob = chain_problem(g["sites"], U=g["U"], seed=g["seed"])
    N = prob.npair
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    t = random_amplitudes(N, "pq", seed=g["amp_seed"], scale=g["amp_scale"])
    blocks = [tuple(L) for L in g["blocks"]]
    lam_blocks, dt, df, de = vjp_inputs(N, g["lambda_seed"], g["direction_seed"], blocks)
    lam = np.zeros(len(t))
    for vals in lam_blocks.values():
        for s, v in vals.items():
            lam[s] = v
    tb, hb, eb = pq.pq_vjp(f, eri, _d(t), _d(lam), g["energy_weight"])
    got = {"t": tb.cpu().numpy() @ dt, "f": np.sum(hb.cpu().numpy() * df),
           "eri": eb.cpu().numpy() @ de}
    for part, ref in g["parts"].items():
        assert abs(got[part] - ref) <= 1e-10 * max(1.0, abs(ref)), (part, got[part], ref)


def test_energy_gradient_matches_oracle_lagrangian(pq):
    N = 3
    f, eri = _system(N, 81)
    ta = tier_a.TierA(N, 2)
    et = layout.unpack_eri(eri, N, 2)
    ref = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t),
                       solver.denominators(f, N, 2), tol=1e-13, max_iter=400)
    assert ref.converged
    gf, ge, lam = gradient.lagrangian_gradient(N, 2, f, eri, ref.t)
    g = pq.pq_energy_grad(_d(f), _d(eri), tol=1e-13)
    assert g.status == "OK"
    assert abs(g.energy - ref.energy) < 1e-11
    _close(g.dE_dh.cpu().numpy(), gf, 1e-9)
    _close(g.dE_deri.cpu().numpy(), ge, 1e-9)
    _close(g.lam.cpu().numpy(), lam, 1e-9)
    # same result when the converged amplitudes are passed in
    res = pq.pq_solve(_d(f), _d(eri), tol=1e-13)
    g2 = pq.pq_energy_grad(_d(f), _d(eri), res.t, tol=1e-13)
    _close(g2.dE_deri.cpu().numpy(), ge, 1e-9)


def test_energy_gradient_finite_differences_chain(pq):
    """16-site chain: dE along a random symmetric (df, deri) equals the central
    difference of solved energies."""
    prob = chain_problem(16, U=4.0, seed=16)
    f, eri = oint.chain_integrals(prob, 2)
    g = pq.pq_energy_grad(_d(f), _d(eri), tol=1e-12)
    rng = np.random.default_rng(17)
    df = rng.normal(size=f.shape) * 0.1
    df = 0.5 * (df + df.T)
    de = rng.normal(size=eri.shape) * 0.1
    s = 1e-4
    ep = pq.pq_solve(_d(f + s * df), _d(eri + s * de), tol=1e-12).energy
    em = pq.pq_solve(_d(f - s * df), _d(eri - s * de), tol=1e-12).energy
    fd = (ep - em) / (2 * s)
    an = float(torch.sum(g.dE_dh * _d(df)) + torch.sum(g.dE_deri * _d(de)))
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (fd, an)


def test_energy_gradient_identities_full_size(pq):
    """140-site chain: homogeneity sum f dE/df + sum v dE/dv = E_c (R and E_c
    are linear in the Hamiltonian) and tr dE/df = 0 (f -> f + cI moves no
    energy difference)."""
    prob = chain_problem(140, U=4.0, seed=140)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    g = pq.pq_energy_grad(f, eri, tol=1e-10)
    assert g.status == "OK"
    hom = float(torch.sum(g.dE_dh * f) + torch.sum(g.dE_deri * eri))
    assert abs(hom - g.energy) < 1e-8, (hom, g.energy)
    assert abs(float(torch.trace(g.dE_dh))) < 1e-8


def test_autograd_function(pq):
    prob = chain_problem(12, U=3.0, seed=12)
    f, eri = oint.chain_integrals(prob, 2)
    h = _d(f).requires_grad_(True)
    e = _d(eri).requires_grad_(True)
    E = pq.pq_energy_autograd(h, e, tol=1e-12)
    (3.0 * E).backward()
    g = pq.pq_energy_grad(_d(f), _d(eri), tol=1e-12)
    assert abs(E.item() - g.energy) < 1e-12
    _close(h.grad.cpu().numpy(), 3.0 * g.dE_dh.cpu().numpy(), 1e-10)
    _close(e.grad.cpu().numpy(), 3.0 * g.dE_deri.cpu().numpy(), 1e-10)


def test_vjp_dot_product_above_128_pairs(pq):
    """Above 128 pairs the two-spectator adjoint splits its output columns
    over workgroups.  Property that holds at any size: <lam, J dt>, with J dt
    from central differences of the residual (parity-checked against the
    oracle), equals <J^T lam, dt> from the VJP.  R is quartic in t, so the
    difference error is O(eps^2)."""
    N = 136
    f, eri = _system(N, 901)
    t = random_amplitudes(N, "pq", seed=902, scale=0.02)
    lam = random_vector(len(t), seed=903)
    dt = random_vector(len(t), seed=904)
    eps = 1e-4
    fd, ed = _d(f), _d(eri)
    rp = pq.pq_residual(fd, ed, _d(t + eps * dt)).cpu().numpy()
    rm = pq.pq_residual(fd, ed, _d(t - eps * dt)).cpu().numpy()
    lhs = float(lam @ ((rp - rm) / (2 * eps)))
    tb, _, _ = pq.pq_vjp(fd, ed, _d(t), _d(lam), 0.0, with_hamiltonian=False)
    rhs = float(tb.cpu().numpy() @ dt)
    assert abs(lhs - rhs) <= 1e-6 * max(1.0, abs(lhs)), (lhs, rhs)


def test_energy_gradient_finite_differences_400_sites(pq):
    """The gradient configuration: a 400-site chain (200 pairs), 20 seeded
    directions delta ~ N(0,1) over (symmetric df, packed deri), normalised to
    unit length; central differences of energies solved to ||R|| <= 1e-12
    (each warm-started from the converged amplitudes) at step 1e-5 must match
    <dE/dh, df> + <dE/deri, deri> to 1e-6 max(1, |g.delta|)."""
    prob = chain_problem(400, U=4.0, seed=400)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    base = pq.pq_solve(f, eri, tol=1e-12, max_iter=400, stall_window=0)
    g = pq.pq_energy_grad(f, eri, base.t, tol=1e-12, max_iter=400, stall_window=0)
    assert g.status == "OK"
    rng = np.random.default_rng(4001)
    s = 1e-5
    worst = 0.0
    for _ in range(20):
        df = rng.normal(size=f.shape)
        df = 0.5 * (df + df.T)
        de = rng.normal(size=eri.shape)
        nrm = np.sqrt(np.sum(df * df) + np.sum(de * de))
        df, de = _d(df / nrm), _d(de / nrm)
        ep = pq.pq_solve(f + s * df, eri + s * de, base.t, tol=1e-12, max_iter=400,
                         stall_window=0)
        em = pq.pq_solve(f - s * df, eri - s * de, base.t, tol=1e-12, max_iter=400,
                         stall_window=0)
        fd = (ep.energy - em.energy) / (2 * s)
        an = float(torch.sum(g.dE_dh * df) + torch.sum(g.dE_deri * de))
        err = abs(fd - an) / max(1.0, abs(an))
        worst = max(worst, err)
        assert err < 1e-6, (fd, an)
    print(f"400-site gradient: worst relative FD error over 20 directions {worst:.2e}")
