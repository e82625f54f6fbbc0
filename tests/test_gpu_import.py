"""GPU tests of the matrix-import and solve-from-b hooks (femh_import_bsr,
femh_solve_rhs_dev, femh_spmv).

The oracle's own matrix (scalar CSR, summed by scipy from Gauss-point
element matrices) is cut into 3x3 blocks and imported, so the products and
the solver are checked on a matrix the HIP assembly never touched.  The
solve-from-b hook also reaches right-hand sides no plane wave produces: the
COCG breakdown vector (section 3.1.5's conjugate gradients read with the
unconjugated form r^T z, which vanishes for b = (1, j, 0, ...) scaled by the
square root of the diagonal).

  products on the imported matrix   <= 1e-13 (|A| |x|) per entry (complex128),
                                      complex64 values bit-exact roundings
  Jacobi inverse                      1 / diag(A) to 1e-14
  solves                              forward error vs LU <= 1e-9 (FP64),
                                      1e-6 (both mixed modes), rtol per the
                                      oracle's condition number
  imported GPU matrix                 bit-identical solve to the mesh path
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fem, solve
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


def _cases():
    rng = np.random.default_rng(21)
    p = W.random_small(rng, n=(5, 4, 6), n_pec=6, lossy=True)
    out = {"random_pec_lossy": (p, [W.random_wave(rng) for _ in range(2)])}
    out["sphere_shell_14"] = W.pec_sphere_shell(n=14, radius=0.3, shell=0.12, seed=3)
    out["free_cube_8"] = W.free_cube(8)
    return out


CASES = _cases()


def _oracle_blocks(prob):
    A = fem.assemble(prob)
    rp, ci = fem.block_pattern(prob)
    return A, rp, ci, fem.to_bsr_blocks(A, rp, ci)


@pytest.mark.parametrize("name", list(CASES))
def test_imported_oracle_matrix_products(ctx, torch, name):
    prob, _ = CASES[name]
    A, rp, ci, blocks = _oracle_blocks(prob)
    P = F.Problem.from_bsr(ctx, rp, ci, blocks)
    assert P.n_nodes == len(rp) - 1 and P.nnzb == len(ci) and P.grid_nodes == 0
    erp, eci, ev = P.export_bsr()
    np.testing.assert_array_equal(erp, rp)
    np.testing.assert_array_equal(eci, ci)
    np.testing.assert_array_equal(ev, blocks)
    np.testing.assert_array_equal(P.export_bsr_c64(), blocks.astype(np.complex64))
    np.testing.assert_allclose(P.export_jacobi(), 1.0 / A.diagonal(), rtol=1e-14, atol=0)
    rng = np.random.default_rng(4)
    n = P.n_unknowns
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    P.spmv_dev(xt, yt, precision=F.FEMH_FP64)
    y = yt.cpu().numpy()
    assert np.all(abs(y - A @ x) <= 1e-13 * (abs(A) @ abs(x)) + 1e-300)
    # the host-vector hook gives the device product bit for bit
    yh, t = P.spmv(x, precision=F.FEMH_FP64, reps=2)
    np.testing.assert_array_equal(yh, y)
    assert t > 0
    # complex64 matrix times complex128 vectors, FP64 arithmetic
    A32 = sp.bsr_matrix((blocks.astype(np.complex64).astype(np.complex128), ci, rp), shape=A.shape).tocsr()
    ym, _ = P.spmv(x, precision=F.FEMH_MIXED_MATRIX)
    assert np.all(abs(ym - A32 @ x) <= 1e-13 * (abs(A32) @ abs(x)) + 1e-300)
    # complex64 everything, FP32 accumulation (the host hook rounds x)
    x32 = x.astype(np.complex64).astype(np.complex128)
    y32, _ = P.spmv(x, precision=F.FEMH_MIXED)
    assert np.all(abs(y32 - A32 @ x32) <= 2e-6 * (abs(A32) @ abs(x32)) + 1e-30)
    P.close()


def _rtol_for(A, target):
    kappa = float(abs(np.linalg.cond(A.toarray(), 1)))
    return min(1e-10, 0.1 * target / kappa)


@pytest.mark.parametrize("name", ["random_pec_lossy", "sphere_shell_14"])
def test_imported_oracle_matrix_solves_match_lu(ctx, torch, name):
    prob, waves = CASES[name]
    A, rp, ci, blocks = _oracle_blocks(prob)
    B = fem.rhs(prob, waves)
    X = solve.dense_solve(A, B)
    P = F.Problem.from_bsr(ctx, rp, ci, blocks)
    bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    for prec, target in ((F.FEMH_FP64, 1e-9), (F.FEMH_MIXED_MATRIX, 1e-6), (F.FEMH_MIXED, 1e-6)):
        rtol = _rtol_for(A, target) if prec == F.FEMH_FP64 else 1e-9
        xt = torch.zeros_like(bt)
        stats, st = P.solve_rhs_dev(bt, xt, precision=prec, rtol=rtol)
        assert st == F.FEMH_OK, (prec, stats)
        xg = xt.cpu().numpy()
        for r in range(B.shape[1]):
            err = np.linalg.norm(xg[r] - X[:, r]) / np.linalg.norm(X[:, r])
            assert err <= target, (prec, r, err, stats[r])
            # the reported residual is the oracle's backward error of the iterate,
            # up to the rounding of two FP64 residual evaluations
            res = solve.residual(A, xg[r], B[:, r])
            bound = 256 * np.finfo(float).eps * np.linalg.norm(abs(A) @ abs(xg[r]) + abs(B[:, r])) / \
                np.linalg.norm(B[:, r])
            assert abs(res - stats[r]["rel_residual"]) <= bound, (res, stats[r], bound)
    P.close()


def test_imported_gpu_matrix_solves_like_the_mesh_path(ctx, torch):
    """The mesh problem's own matrix and right-hand side, exported and
    imported again, give the mesh path's solution bit for bit: the solver
    kernels see the same numbers either way."""
    prob, waves = CASES["sphere_shell_14"]
    Pm = F.Problem(ctx, prob)
    rp, ci, v = Pm.export_bsr()
    b = Pm.export_rhs(waves)
    H, stats, st = Pm.solve(waves, precision=F.FEMH_FP64, rtol=1e-10)
    assert st == F.FEMH_OK
    Pi = F.Problem.from_bsr(ctx, rp, ci, v)
    np.testing.assert_array_equal(Pi.export_jacobi(), Pm.export_jacobi())
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    si, sti = Pi.solve_rhs_dev(bt, xt, precision=F.FEMH_FP64, rtol=1e-10)
    assert sti == F.FEMH_OK
    active = fem.Mesh(prob).node_active
    for r in range(len(waves)):
        np.testing.assert_array_equal(xt[r].cpu().numpy(), H[r][active].reshape(-1))
        assert si[r]["iters"] == stats[r]["iters"]
    Pm.close()
    Pi.close()


@pytest.mark.parametrize("prec", [F.FEMH_FP64, F.FEMH_MIXED_MATRIX, F.FEMH_MIXED])
def test_breakdown_vector_reports_breakdown(ctx, torch, prec):
    """b_k = s_k sqrt(D_kk) with s = (1, j, 0, ...) gives r^T D^-1 r =
    1 + j^2 = 0 at the first step: the solver must report FEMH_E_BREAKDOWN
    (after its one restart from the true residual), not loop or diverge.
    Without preconditioning b = (1, j, 0, ...) itself does it."""
    prob, _ = CASES["free_cube_8"]
    A, rp, ci, blocks = _oracle_blocks(prob)
    P = F.Problem.from_bsr(ctx, rp, ci, blocks)
    n = P.n_unknowns
    D = A.diagonal()
    b = np.zeros(n, np.complex128)
    b[0] = np.sqrt(D[0])
    b[1] = 1j * np.sqrt(D[1])
    assert abs(np.sum(b * b / D)) <= 1e-14 * np.sum(abs(b) ** 2 / abs(D))
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    stats, st = P.solve_rhs_dev(bt, xt, precision=prec, rtol=1e-8)
    assert st == F.FEMH_E_BREAKDOWN and stats[0]["status"] == F.FEMH_E_BREAKDOWN, stats
    assert np.isfinite(stats[0]["rel_residual"])
    if prec != F.FEMH_MIXED:
        b2 = np.zeros(n, np.complex128)
        b2[0], b2[1] = 1.0, 1j
        bt2 = torch.from_numpy(b2).cuda()
        stats, st = P.solve_rhs_dev(bt2, xt, precision=prec, rtol=1e-8, precond=F.FEMH_PRECOND_NONE)
        assert st == F.FEMH_E_BREAKDOWN, stats
    P.close()


def test_import_rejects_malformed_matrices(ctx, torch):
    prob, waves = CASES["free_cube_8"]
    A, rp, ci, blocks = _oracle_blocks(prob)

    def status(rp_, ci_, v_):
        h = F.C.c_void_p()
        rp_ = np.ascontiguousarray(rp_, dtype=np.int32)
        ci_ = np.ascontiguousarray(ci_, dtype=np.int32)
        v_ = np.ascontiguousarray(v_, dtype=np.complex128)
        st = ctx.lib.femh_import_bsr(ctx.handle, len(rp_) - 1, len(ci_), rp_.ctypes.data, ci_.ctypes.data,
                                     v_.ctypes.data, F.C.byref(h))
        if st == F.FEMH_OK:
            ctx.lib.femh_problem_destroy(h)
        return st

    assert status(rp, ci, blocks) == F.FEMH_OK
    bad = blocks.copy()
    bad[5, 1, 2] = np.nan
    assert status(rp, ci, bad) == F.FEMH_E_NONFINITE
    bad = blocks.copy()
    d0 = np.nonzero(ci[rp[0]:rp[1]] == 0)[0][0]
    bad[rp[0] + d0, 1, 1] = 0.0
    assert status(rp, ci, bad) == F.FEMH_E_INVALID          # zero diagonal entry
    ci2 = ci.copy()
    ci2[rp[3]], ci2[rp[3] + 1] = ci2[rp[3] + 1], ci2[rp[3]]
    assert status(rp, ci2, blocks) == F.FEMH_E_INVALID       # not ascending
    ci3 = ci.copy()
    ci3[rp[2]:rp[3]] = np.where(ci3[rp[2]:rp[3]] == 2, -1, ci3[rp[2]:rp[3]])
    assert status(rp, np.sort(ci3), blocks) == F.FEMH_E_INVALID  # no diagonal / out of range
    rp4 = rp.copy()
    rp4[-1] += 1
    assert status(rp4, ci, blocks) == F.FEMH_E_INVALID       # row_ptr does not end at nnzb
    # a problem without a mesh refuses the plane-wave entry points
    P = F.Problem.from_bsr(ctx, rp, ci, blocks)
    w = F.make_waves(waves)
    st = np.zeros(1, np.int64)
    stats = (F.femh_solve_stats * 1)()
    out = np.zeros(64, np.complex128)
    assert ctx.lib.femh_solve(P.handle, 1, w, None, out.ctypes.data, stats) == F.FEMH_E_INVALID
    assert "no mesh" in F.last_error()
    assert ctx.lib.femh_export_rhs(P.handle, 1, w, out.ctypes.data) == F.FEMH_E_INVALID
    P.close()
    del st
