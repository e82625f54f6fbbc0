"""GPU tests of the degenerate inputs of the path: the smallest mesh (one
hexahedron, 8 nodes, 24 unknowns), a box whose every element is PEC (no
unknowns: refused with FEMH_E_INVALID), a box with a single active element
among PEC ones, and the batched solver's column limits.  The solutions are
checked against the oracle's dense LU (FP64 to 1e-9, mixed modes to 1e-6,
tolerances as in the other parity tests)."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, solve
from paper_0704_2344_amd import femh as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = F.Context(0)
    yield c
    c.close()


def _check_against_lu(ctx, prob, waves):
    A = fem.assemble(prob)
    X = solve.dense_solve(A, fem.rhs(prob, waves))
    Ho = fem.scatter_to_grid(prob, X)
    kappa = float(abs(np.linalg.cond(A.toarray(), 1)))
    P = F.Problem(ctx, prob)
    assert P.n_unknowns == A.shape[0]
    for prec, target in ((F.FEMH_FP64, 1e-9), (F.FEMH_MIXED_MATRIX, 1e-6), (F.FEMH_MIXED, 1e-6)):
        rtol = min(1e-10, 0.1 * target / kappa) if prec == F.FEMH_FP64 else 1e-9
        H, stats, st = P.solve(waves, precision=prec, rtol=rtol)
        assert st == F.FEMH_OK, (prec, stats)
        for r in range(len(waves)):
            err = np.linalg.norm(H[r] - Ho[r]) / np.linalg.norm(Ho[r])
            assert err <= target, (prec, r, err)
    P.close()


def test_single_hexahedron_matches_lu(ctx):
    prob, w = W.free_cube(1)
    rng = np.random.default_rng(3)
    _check_against_lu(ctx, prob, w + [W.random_wave(rng)])


def test_one_active_element_among_pec_matches_lu(ctx):
    """A 3x3x3 box whose only non-PEC element is a corner one: 8 active
    nodes, each with a full 8-node neighbourhood of one element."""
    prob, w = W.free_cube(3)
    prob.pec[:] = 1
    prob.pec.reshape(3, 3, 3)[0, 0, 0] = 0
    P = F.Problem(ctx, prob)
    assert P.n_nodes == 8 and P.nnzb == 64
    P.close()
    _check_against_lu(ctx, prob, w)


def test_all_pec_box_is_refused(ctx):
    prob, _ = W.free_cube(3)
    prob.pec[:] = 1
    with pytest.raises(F.FemhError) as e:
        F.Problem(ctx, prob)
    assert e.value.status == F.FEMH_E_INVALID
    assert "PEC" in F.last_error()


def test_batched_column_limits(ctx):
    """femh_solve_batched_dev takes 1..64 right-hand sides: 64 run as one
    wide batch and match the oracle; 0 and 65 are refused."""
    import torch
    prob, _ = W.free_cube(4)
    rng = np.random.default_rng(11)
    waves = [W.random_wave(rng) for _ in range(64)]
    P = F.Problem(ctx, prob)
    out = torch.zeros(P.grid_shape(64), dtype=torch.complex128, device="cuda")
    stats, st = P.solve_dev(waves, out, batched=True, precision=F.FEMH_FP64, rtol=1e-10)
    assert st == F.FEMH_OK, stats
    A = fem.assemble(prob)
    Ho = fem.scatter_to_grid(prob, solve.dense_solve(A, fem.rhs(prob, waves)))
    H = out.cpu().numpy()
    for r in (0, 31, 63):
        assert np.linalg.norm(H[r] - Ho[r]) / np.linalg.norm(Ho[r]) <= 1e-8
    ws = F.make_waves(waves + waves[:1])
    o = F.make_opts(precision=F.FEMH_FP64)
    st65 = (F.femh_solve_stats * 65)()
    big = torch.zeros(P.grid_shape(65), dtype=torch.complex128, device="cuda")
    assert ctx.lib.femh_solve_batched_dev(P.handle, 65, ws, F.C.byref(o), big.data_ptr(), st65) == F.FEMH_E_INVALID
    assert ctx.lib.femh_solve_batched_dev(P.handle, 0, ws, F.C.byref(o), big.data_ptr(), st65) == F.FEMH_E_INVALID
    P.close()
