"""Oracle: solvers for the assembled system (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* dense_solve  -- LAPACK LU (numpy.linalg.solve), tiny systems;
* sparse_solve -- SuperLU (scipy.sparse.linalg.splu), small/medium systems;
* cocg         -- the paper's conjugate gradient (section 3.1.5) read for a
  complex-symmetric, non-Hermitian matrix: the unconjugated bilinear form
  x^T y replaces the inner product (the incomplete-Cholesky recurrences of
  eq. (5) likewise carry no conjugation), stopping on the Hermitian 2-norm
  of the recursive residual.  Diagonal preconditioning (section 3.1.5.1):
  z = D^-1 r with D the diagonal of the matrix.  x0 = 0;
* pcocg        -- the same recurrence with any preconditioner z = M^-1 r;
* bic0_factor, bic0_apply -- the block incomplete Cholesky preconditioner of
  sections 3.1.5.2-3.1.5.3: eq. (5)'s incomplete factor on the diagonal
  blocks of B consecutive nodes, applied by the forward and back
  substitution of eq. (6).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def dense_solve(A, b):
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.linalg.solve(Ad, b)


def sparse_solve(A, b):
    lu = spla.splu(sp.csc_matrix(A))
    return lu.solve(np.asarray(b, dtype=np.complex128))


def bilinear(x, y):
    """Unconjugated x^T y."""
    return np.sum(x * y)


@dataclasses.dataclass
class CocgResult:
    x: np.ndarray
    iters: int
    rel_res: float          # recursive residual norm / ||b||
    breakdown: bool
    history: list


def cocg(A, b, rtol=1e-10, maxiter=10000, jacobi=True, breakdown_tol=1e-14):
    """COCG with optional Jacobi preconditioning (see module doc).

    Breakdown is reported when |rho| or |p^T A p| falls below
    breakdown_tol times the squared norms that bound it."""
    b = np.asarray(b, dtype=np.complex128)
    dinv = 1.0 / A.diagonal() if jacobi else np.ones_like(b)
    return pcocg(A, b, lambda r: dinv * r, rtol, maxiter, breakdown_tol)


def pcocg(A, b, apply_m, rtol=1e-10, maxiter=10000, breakdown_tol=1e-14):
    """COCG with the preconditioner z = apply_m(r), M complex-symmetric
    (the recurrence of section 3.1.5 with the bilinear form x^T y)."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return CocgResult(x, 0, 0.0, False, [0.0])
    r = b.copy()
    z = apply_m(r)
    p = z.copy()
    rho = bilinear(r, z)
    hist = [1.0]
    if abs(rho) <= breakdown_tol * np.linalg.norm(r) * np.linalg.norm(z):
        return CocgResult(x, 0, 1.0, True, hist)
    for k in range(1, maxiter + 1):
        q = A @ p
        mu = bilinear(p, q)
        if abs(mu) <= breakdown_tol * np.linalg.norm(p) * np.linalg.norm(q):
            return CocgResult(x, k - 1, hist[-1], True, hist)
        alpha = rho / mu
        x = x + alpha * p
        r = r - alpha * q
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if rel <= rtol:
            return CocgResult(x, k, rel, False, hist)
        z = apply_m(r)
        rho_new = bilinear(r, z)
        if abs(rho_new) <= breakdown_tol * np.linalg.norm(r) * np.linalg.norm(z):
            return CocgResult(x, k, rel, True, hist)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return CocgResult(x, maxiter, hist[-1], False, hist)


def bic0_factor(A, nodes_per_block):
    """Block incomplete Cholesky (sections 3.1.5.2-3.1.5.3).  The unknowns
    are cut into blocks of B = nodes_per_block consecutive nodes (3 B
    unknowns; the last block may be shorter) and the couplings between
    blocks are dropped, as each processor of the paper keeps only its
    diagonal block.  Each block gets the incomplete factor of eq. (5) on its
    own lower pattern, column by column and without conjugation (A is
    complex-symmetric, A ~ L L^T).  The pattern is A's stored structure (all
    nine entries of the 3x3 block of every pair of nodes that share an
    element), not its nonzero values: summation leaves some entries that are
    zero in exact arithmetic at +-1e-18 on one side of the diagonal only.
        l_jj = sqrt(a_jj - sum_{k<j} l_jk^2)
        l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj,  i > j, (i, j) stored
    (the principal complex square root).  Returns L (CSR, lower triangular,
    block diagonal)."""
    A = sp.csr_matrix(A)
    S = A.copy()
    S.data = np.ones_like(S.data)
    n = A.shape[0]
    size = 3 * nodes_per_block
    rows, cols, vals = [], [], []
    for b0 in range(0, n, size):
        b1 = min(b0 + size, n)
        blk = A[b0:b1, b0:b1].toarray()
        keep = np.tril(S[b0:b1, b0:b1].toarray() != 0)
        L = np.where(keep, blk, 0.0).astype(np.complex128)
        m = b1 - b0
        for j in range(m):
            L[j, j] = np.sqrt(L[j, j] - np.sum(L[j, :j] * L[j, :j]))
            for i in range(j + 1, m):
                if keep[i, j]:
                    L[i, j] = (L[i, j] - np.sum(L[i, :j] * L[j, :j])) / L[j, j]
        r, c = np.nonzero(keep)
        rows.append(r + b0)
        cols.append(c + b0)
        vals.append(L[r, c])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def bic0_apply(L, r):
    """z = (L L^T)^-1 r: forward substitution L y = r, then back substitution
    L^T z = y (eq. (6))."""
    y = spla.spsolve_triangular(sp.csr_matrix(L), np.asarray(r, np.complex128), lower=True)
    return spla.spsolve_triangular(sp.csr_matrix(L.T), y, lower=False)


def residual(A, x, b):
    """Backward error ||b - A x||_2 / ||b||_2 (FP64)."""
    b = np.asarray(b)
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))


def condest(A, lu=None):
    """1-norm condition estimate ||A||_1 * est(||A^-1||_1): SuperLU solves
    inside the Hager-Higham estimator (scipy onenormest).  lu may be a
    SuperLU factorisation of A already at hand (see lu_solve_condest)."""
    if lu is None:
        lu = spla.splu(sp.csc_matrix(A))
    n = A.shape[0]
    inv = spla.LinearOperator((n, n), matvec=lu.solve,
                              rmatvec=lambda y: lu.solve(np.asarray(y, np.complex128), trans="H"),
                              dtype=np.complex128)
    return float(spla.norm(A, 1) * spla.onenormest(inv))


def lu_solve_condest(A, b):
    """SuperLU solution of A x = b and the 1-norm condition estimate from the
    same factorisation (one factorisation instead of two for large systems)."""
    lu = spla.splu(sp.csc_matrix(A))
    return lu.solve(np.asarray(b, dtype=np.complex128)), condest(A, lu)
