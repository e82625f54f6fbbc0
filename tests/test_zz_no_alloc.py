"""GPU test of the allocation-free product (femh_spmm_noalloc_dev), called
through the C ABI: its result equals femh_spmm_dev's (the allocating entry
point with the same kernel) bit for bit, on two calls in a row, the second
on a smaller problem, so the shared static scratch is reused with fewer
workgroups than before; narrower column counts are refused."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from paper_0704_2344_amd import femh as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    c = F.Context(0)
    yield c
    c.close()


def _blocks(torch, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 64)) + 1j * rng.standard_normal((n, 64))
    return torch.from_numpy(X).cuda(), torch.zeros((n, 64), dtype=torch.complex128, device="cuda")


@pytest.mark.parametrize("prec", [F.FEMH_FP64, F.FEMH_MIXED_MATRIX])
def test_noalloc_product_matches_the_allocating_one(ctx, torch, prec):
    big, _ = W.pec_sphere_batched(n=24, radius=0.6, nrhs=1, seed=3)
    small, _ = W.pec_sphere_shell(n=10, radius=0.25, shell=0.1, seed=5)
    for k, prob in enumerate((big, small)):
        P = F.Problem(ctx, prob)
        X, Y_ref = _blocks(torch, P.n_unknowns, 17 + k)
        P.spmm_dev(X, Y_ref, reps=1, precision=prec)
        Y = torch.full_like(Y_ref, float("nan"))
        st = ctx.lib.femh_spmm_noalloc_dev(P.handle, prec, 64, X.data_ptr(), Y.data_ptr())
        assert st == F.FEMH_OK, F.last_error()
        torch.cuda.synchronize()
        assert torch.equal(Y, Y_ref), (k, prec)
        P.close()


def test_noalloc_product_before_any_tuning_and_refusals(ctx, torch):
    """On a fresh problem (no tuned shape yet) the default grid gives the
    same product as the allocating entry point's tuned one; other column
    counts and precisions are refused with a message."""
    prob, _ = W.pec_sphere_batched(n=16, radius=0.4, nrhs=1, seed=7)
    P = F.Problem(ctx, prob)
    X, Y = _blocks(torch, P.n_unknowns, 29)
    assert ctx.lib.femh_spmm_noalloc_dev(P.handle, F.FEMH_FP64, 64, X.data_ptr(), Y.data_ptr()) == F.FEMH_OK
    torch.cuda.synchronize()
    Y_ref = torch.zeros_like(Y)
    P.spmm_dev(X, Y_ref, reps=1, precision=F.FEMH_FP64)
    assert torch.equal(Y, Y_ref)
    assert ctx.lib.femh_spmm_noalloc_dev(P.handle, F.FEMH_FP64, 32, X.data_ptr(), Y.data_ptr()) == F.FEMH_E_INVALID
    assert "64" in F.last_error()
    assert ctx.lib.femh_spmm_noalloc_dev(P.handle, F.FEMH_MIXED, 64, X.data_ptr(), Y.data_ptr()) == F.FEMH_E_INVALID
    assert ctx.lib.femh_spmm_noalloc_dev(P.handle, F.FEMH_FP64, 64, None, Y.data_ptr()) == F.FEMH_E_INVALID
    P.close()
