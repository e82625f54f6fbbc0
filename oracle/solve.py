"""Oracle: solvers for the assembled system (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* dense_solve  -- LAPACK LU (numpy.linalg.solve), tiny systems;
* sparse_solve -- SuperLU (scipy.sparse.linalg.splu), small/medium systems;
* cocg         -- the paper's conjugate gradient (section 3.1.5) read for a
  complex-symmetric, non-Hermitian matrix: the unconjugated bilinear form
  x^T y replaces the inner product (the incomplete-Cholesky recurrences of
  eq. (5) likewise carry no conjugation), stopping on the Hermitian 2-norm
  of the recursive residual.  Diagonal preconditioning (section 3.1.5.1):
  z = D^-1 r with D the diagonal of the matrix.  x0 = 0.
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
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return CocgResult(x, 0, 0.0, False, [0.0])
    r = b.copy()
    z = dinv * r
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
        z = dinv * r
        rho_new = bilinear(r, z)
        if abs(rho_new) <= breakdown_tol * np.linalg.norm(r) * np.linalg.norm(z):
            return CocgResult(x, k, rel, True, hist)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return CocgResult(x, maxiter, hist[-1], False, hist)


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
