"""The two-pair-intermediate PQ variant (pqph_set_pq_intermediates(.., 2);
Sec. III: the paper's PQ uses intermediates of up to three pairs and notes
that two-pair intermediates, O(N^3), cost accuracy).

Parity unpinned against the paper: which terms its two-pair-intermediate code
drops follows its unpublished intermediates.  Here the variant leaves out the
doubly-mixed two-spectator terms; the definitional oracle has no term
topology to drop, so the variant is checked against the oracle where it
must coincide with the exact model (three pairs), and against the CPU
emulation of the kernel tables with the same terms left out at four and five
pairs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs import chain_problem, random_amplitudes, random_bfactors, random_fock
from oracle import integrals as oint
from oracle import layout, tier_a

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pq():
    import paper_1609_00077_amd as pq
    pq._lib.load()
    return pq


@pytest.fixture(scope="module")
def tables():
    from paper_1609_00077_amd.derive.codegen import build_pq_tables
    return build_pq_tables()


def _d(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _system(N, seed):
    f = random_fock(N, seed=seed)
    return f, oint.eri_packed_from_b(random_bfactors(N, seed=seed + 1), N, 2)


@pytest.mark.parametrize("N", [3, 4, 5])
def test_two_pair_intermediates_residual(pq, tables, N):
    from pq_table_emulator import Emu
    f, eri = _system(N, 1500 + N)
    t = random_amplitudes(N, "pq", seed=1600 + N, scale=0.1)
    pq.set_pq_intermediates(N, 2)
    R2 = pq.pq_residual(_d(f), _d(eri), _d(t)).cpu().numpy()
    pq.set_pq_intermediates(N, 3)
    R3 = pq.pq_residual(_d(f), _d(eri), _d(t)).cpu().numpy()
    RA, _ = tier_a.TierA(N, 2).residual(f, layout.unpack_eri(eri, N, 2), t)
    tol = 1e-12 * max(1.0, np.abs(RA).max())
    assert np.abs(R3 - RA).max() <= tol
    if N == 3:
        assert np.abs(R2 - RA).max() <= tol
    else:
        ref = Emu(tables, N, f, eri, mixed=False).residual(t)
        assert np.abs(R2 - ref).max() <= tol
        assert np.abs(R2 - R3).max() > 1e-6


def test_two_pair_intermediates_solve_and_gradient(pq):
    """16-site chain: the variant's solve differs from the exact PQ energy (by
    little: the left-out terms are fourth order in the amplitudes), and its
    gradient matches central differences of its own solves."""
    prob = chain_problem(16, U=4.0, seed=16)
    f, eri = oint.chain_integrals(prob, 2)
    N = prob.npair
    e3 = pq.pq_solve(_d(f), _d(eri), tol=1e-12).energy
    pq.set_pq_intermediates(N, 2)
    try:
        e2 = pq.pq_solve(_d(f), _d(eri), tol=1e-12).energy
        g = pq.pq_energy_grad(_d(f), _d(eri), tol=1e-12)
        rng = np.random.default_rng(19)
        df = rng.normal(size=f.shape) * 0.1
        df = 0.5 * (df + df.T)
        de = rng.normal(size=eri.shape) * 0.1
        s = 1e-4
        ep = pq.pq_solve(_d(f + s * df), _d(eri + s * de), tol=1e-12).energy
        em = pq.pq_solve(_d(f - s * df), _d(eri - s * de), tol=1e-12).energy
    finally:
        pq.set_pq_intermediates(N, 3)
    assert abs(g.energy - e2) < 1e-11
    assert abs(e2 - e3) > 1e-13
    fd = (ep - em) / (2 * s)
    an = float(torch.sum(g.dE_dh * _d(df)) + torch.sum(g.dE_deri * _d(de)))
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (fd, an)
    print(f"16-site PQ: exact {e3:.10f}, two-pair intermediates {e2:.10f}")
