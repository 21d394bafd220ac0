"""The allocation-free PQ residual (workspace in a static per-GPU device
array) against the allocating entry point pq_residual, through the C ABI, on
two calls in a row, the second with a smaller input; and its limits."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs import random_amplitudes, random_bfactors, random_fock
from oracle import integrals as oint

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pq():
    import paper_1609_00077_amd as pq
    pq._lib.load()
    return pq


def _d(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _inputs(N, seed):
    f = random_fock(N, seed=seed)
    eri = oint.eri_packed_from_b(random_bfactors(N, seed=seed + 1), N, 2)
    t = random_amplitudes(N, "pq", seed=seed + 2, scale=0.05)
    return _d(f), _d(eri), _d(t)


def test_noalloc_matches_allocating_residual(pq):
    lib, ctx = pq._ctx(torch.device(DEV))
    for N, seed in ((32, 1100), (7, 1200), (32, 1300)):
        print(f"pq_residual_noalloc N={N}", flush=True)
        h, e, t = _inputs(N, seed)
        ref = pq.pq_residual(h, e, t).clone()
        out = torch.full_like(ref, np.nan)
        p = lambda x: C.c_void_p(x.data_ptr())
        st = lib.pq_residual_noalloc(ctx, N, p(h), p(e), p(t), p(out))
        assert st == 0, lib.pqph_last_error(ctx)
        torch.cuda.synchronize()
        tol = 1e-12 * max(1.0, ref.abs().max().item())
        assert (out - ref).abs().max().item() <= tol, (N, (out - ref).abs().max().item())
        assert torch.isfinite(out).all()


def test_noalloc_limits(pq):
    lib, ctx = pq._ctx(torch.device(DEV))
    h, e, t = _inputs(3, 1400)
    r = torch.empty_like(t)
    p = lambda x: C.c_void_p(x.data_ptr())
    assert lib.pq_residual_noalloc(ctx, 33, p(h), p(e), p(t), p(r)) == -1
    assert b"allocation-free" in lib.pqph_last_error(ctx)
    assert lib.pq_residual_noalloc(ctx, 0, p(h), p(e), p(t), p(r)) == -1
    assert lib.pq_residual_noalloc(ctx, 3, p(h), p(e), p(t), None) == -1
    assert lib.pq_residual_noalloc(ctx, 3, p(h), p(e), p(t), p(r)) == 0
    torch.cuda.synchronize()
    assert torch.allclose(r, pq.pq_residual(h, e, t), rtol=0, atol=1e-12)
