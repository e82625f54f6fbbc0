"""CPU checks of the block-incomplete-Cholesky experiment's machinery
(tests/bicp_experiment.py): its IC(0) is the eq. (5) factor (exact Cholesky
when the pattern is full), its block LU bound solves exactly, and its
Jacobi COCG is the oracle's COCG."""
import os
import sys

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import bicp_experiment as X  # noqa: E402
import workloads as W  # noqa: E402
from oracle import fem, solve  # noqa: E402


def test_ic0_on_a_full_pattern_is_the_complex_symmetric_cholesky_factor():
    rng = np.random.default_rng(3)
    n = 12
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = M @ M.T + 10 * n * np.eye(n)          # complex-symmetric, well away from singular
    L = X.ic0_blocks(sp.csr_matrix(A), n // 3).toarray()
    assert np.allclose(L, np.tril(L))
    np.testing.assert_allclose(L @ L.T, A, rtol=1e-12, atol=1e-10)   # L L^T, not L L^H


def test_ic0_keeps_the_pattern_and_stays_inside_blocks():
    p, _ = W.pec_sphere_shell(n=6, radius=0.15, shell=0.06, seed=2)
    A = fem.assemble(p).tocsr()
    Abd = X.block_diagonal(A, 8)
    L = X.ic0_blocks(Abd, 8).tocoo()
    assert np.all(L.row // 24 == L.col // 24)
    assert np.all(L.row >= L.col)
    low = sp.tril(Abd).tocsr()
    assert np.all(np.asarray(low[L.row, L.col]).ravel() != 0)


def test_block_lu_with_one_block_solves_in_one_step_and_jacobi_matches_the_oracle():
    rng = np.random.default_rng(5)
    p = W.random_small(rng, n=(3, 3, 3), n_pec=1)
    A = fem.assemble(p).tocsr()
    b = fem.rhs(p, [W.random_wave(rng)])[:, 0]
    m = X.preconditioner(A, "blu", A.shape[0] // 3)
    it, rel, true_rel = X.pcocg(A, b, m, 1e-10, 50)
    assert it == 1 and true_rel <= 1e-10
    mj = X.preconditioner(A, "jacobi")
    it_j, rel_j, _ = X.pcocg(A, b, mj, 1e-10, 5000)
    ref = solve.cocg(A, b, rtol=1e-10, maxiter=5000)
    assert it_j == ref.iters and rel_j == pytest_approx(ref.rel_res)


def pytest_approx(v):
    import pytest
    return pytest.approx(v, rel=1e-9)
