"""Block incomplete Cholesky (BICP) against diagonal preconditioning, on the CPU.

Sections 3.1.5.2-3.1.5.3 precondition the conjugate gradient with an
incomplete Cholesky factor A ~ L L^T (eq. (5), no conjugation, so the
complex-symmetric reading holds) and, in the parallel version, keep only the
diagonal block of each processor's rows so that building and applying it
needs no messages (forward and back substitution, eq. (6), inside each
block).  This script measures whether that preconditioner cuts the number
of iterations on this build's workloads enough to pay for two triangular
solves per iteration, the question that decides whether it is built on the
GPU:

  * Jacobi        z = D^-1 r (section 3.1.5.1; what the GPU solvers use);
  * BIC(0)-B      IC(0) on the pattern of A inside blocks of B consecutive
                  nodes (3 B unknowns), z = L^-T L^-1 r per block;
  * BLU-B         the blocks' exact LU (an upper bound on what any
                  incomplete factor of the same blocks can achieve).

Each runs COCG (the oracle's recurrence with the preconditioner swapped in)
on the oracle's matrix and right-hand side to the relative residual `rtol`,
capped at `maxiter`; the output is iterations and the residual reached.

    python tests/bicp_experiment.py pec_sphere_shell_60 --blocks 64,512 --maxiter 60000
    python tests/bicp_experiment.py pec_cube_30

Nothing here is on the product path: it uses the oracle (test
infrastructure) and SciPy only.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fem  # noqa: E402


def block_diagonal(A, nodes_per_block):
    """A with every coupling between different blocks of consecutive nodes
    removed (block b = unknowns [3 B b, 3 B (b + 1)))."""
    A = A.tocoo()
    size = 3 * nodes_per_block
    keep = (A.row // size) == (A.col // size)
    return sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)


def ic0_blocks(Abd, nodes_per_block):
    """IC(0) of a block-diagonal complex-symmetric matrix on its own lower
    pattern, block by block: L_jj = sqrt(A_jj - sum_k L_jk^2) and, for i > j
    where A_ij is stored, L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj (eq. (5)
    read as standard IC(0), no conjugation).  Returns L as CSR."""
    from threadpoolctl import threadpool_limits

    n = Abd.shape[0]
    size = 3 * nodes_per_block
    Ad = Abd.tocsr()
    rows, cols, vals = [], [], []
    with threadpool_limits(1):  # many tiny products: threads only add overhead
        _ic0_loop(Ad, n, size, rows, cols, vals)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def _ic0_loop(Ad, n, size, rows, cols, vals):
    for b0 in range(0, n, size):
        b1 = min(b0 + size, n)
        blk = Ad[b0:b1, b0:b1].toarray()
        mask = np.tril(blk != 0)
        L = np.tril(blk).astype(np.complex128)
        m = b1 - b0
        for j in range(m):
            d = L[j, j] - np.dot(L[j, :j], L[j, :j])
            L[j, j] = np.sqrt(d)
            if j + 1 < m:
                col = (L[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
                L[j + 1:, j] = np.where(mask[j + 1:, j], col, 0.0)
        r, c = np.nonzero(L)
        rows.append(r + b0)
        cols.append(c + b0)
        vals.append(L[r, c])


def preconditioner(A, kind, nodes_per_block=0):
    """z = M^-1 r as a function, M complex-symmetric."""
    if kind == "jacobi":
        dinv = 1.0 / A.diagonal()
        return lambda r: dinv * r
    Abd = block_diagonal(A, nodes_per_block)
    if kind == "blu":
        lu = spla.splu(sp.csc_matrix(Abd))
        return lu.solve
    if kind == "bic0":
        L = ic0_blocks(Abd, nodes_per_block)
        # triangular solves through SuperLU with the natural order: the LU of
        # a triangular matrix has no fill, so solve() is the substitution
        fl = spla.splu(sp.csc_matrix(L), permc_spec="NATURAL", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        bl = spla.splu(sp.csc_matrix(L.T), permc_spec="NATURAL", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        return lambda r: bl.solve(fl.solve(r))
    raise ValueError(kind)


def pcocg(A, b, apply_m, rtol, maxiter, report_every=0, label=""):
    """COCG with a complex-symmetric preconditioner M: the oracle's
    recurrence (unconjugated r^T z, Hermitian norm for stopping), z = M^-1 r.
    Returns (iterations, recursive relative residual, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_m(r)
    p = z.copy()
    rho = np.sum(r * z)
    bn = np.linalg.norm(b)
    rel = 1.0
    k = 0
    t0 = time.perf_counter()
    for k in range(1, maxiter + 1):
        q = A @ p
        mu = np.sum(p * q)
        alpha = rho / mu
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / bn
        if rel <= rtol:
            break
        z = apply_m(r)
        rho_new = np.sum(r * z)
        p = z + (rho_new / rho) * p
        rho = rho_new
        if report_every and k % report_every == 0:
            print(f"  {label} iteration {k}: relative residual {rel:.3e} ({time.perf_counter() - t0:.0f} s)",
                  flush=True)
    true_rel = float(np.linalg.norm(b - A @ x) / bn)
    return k, float(rel), true_rel


WORKLOADS = {
    "pec_cube_30": lambda: W.pec_cube(30),
    "pec_sphere_shell_60": lambda: W.pec_sphere_shell(60),
    "pec_sphere_40": lambda: W.pec_sphere_batched(40, nrhs=1),
    "sphere_shell_14": lambda: W.pec_sphere_shell(n=14, radius=0.3, shell=0.12, seed=3),
}


def run(workload, blocks, rtol, maxiter, kinds=("jacobi", "bic0", "blu"), report_every=0):
    prob, waves = WORKLOADS[workload]()
    A = fem.assemble(prob).tocsr()
    b = fem.rhs(prob, waves)[:, 0]
    out = []
    for kind in kinds:
        for B in (blocks if kind != "jacobi" else [0]):
            t0 = time.perf_counter()
            m = preconditioner(A, kind, B)
            t1 = time.perf_counter()
            label = kind if kind == "jacobi" else f"{kind}-{B}"
            it, rel, true_rel = pcocg(A, b, m, rtol, maxiter, report_every, label)
            t2 = time.perf_counter()
            out.append({"workload": workload, "preconditioner": label, "iterations": it,
                        "rel_residual": rel, "true_rel_residual": true_rel,
                        "setup_s": t1 - t0, "solve_s": t2 - t1})
            print(out[-1], flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--blocks", default="64,512", help="nodes per block, comma-separated")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--maxiter", type=int, default=60000)
    ap.add_argument("--kinds", default="jacobi,bic0,blu")
    ap.add_argument("--report-every", type=int, default=1000)
    a = ap.parse_args()
    run(a.workload, [int(x) for x in a.blocks.split(",")], a.rtol, a.maxiter, tuple(a.kinds.split(",")),
        a.report_every)


if __name__ == "__main__":
    main()
