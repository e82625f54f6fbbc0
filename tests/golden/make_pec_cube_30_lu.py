"""Write tests/golden/pec_cube_30_lu.txt from the CPU oracle only.

The 3-wavelength PEC-cube workload (30^3 hexahedra, 87 186 unknowns) is too
large for a dense solve in a test and its sparse LU takes minutes, so its
exact discrete solution is computed once here: the oracle's scalar assembly
and right-hand side (eqs. (1)-(4)), SuperLU (a direct solve, forward error
about kappa * eps), and the oracle's 1-norm condition estimate.  The file
keeps kappa_1, ||x*||_2, ||x*||_inf and x* at 256 seeded unknowns (plus the
first and last), so the GPU forward-error test (the solve's relative error
against the exact discrete solution) needs no LU of its own.

    python tests/golden/make_pec_cube_30_lu.py
"""
import os
import sys

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fem, solve  # noqa: E402

OUT = os.path.join(HERE, "pec_cube_30_lu.txt")


def main():
    prob, waves = W.pec_cube(30)
    A = fem.assemble(prob)
    b = fem.rhs(prob, waves)[:, 0]
    n = A.shape[0]
    x, kappa = solve.lu_solve_condest(A, b)
    res = solve.residual(A, x, b)
    rng = np.random.default_rng(2030)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, size=256, replace=False)]))
    with open(OUT, "w") as f:
        f.write("# Exact discrete solution of the pec_cube_30 workload (30^3 hexahedra, centred PEC cube of one\n")
        f.write("# wavelength, ABC outer faces, the seeded wave of workloads.pec_cube), from the CPU oracle:\n")
        f.write("# scalar assembly, SuperLU solve and the 1-norm condition estimate.  Written by\n")
        f.write("# make_pec_cube_30_lu.py; unknown index = 3 * active node + component.\n")
        f.write(f"n_unknowns {n}\n")
        f.write(f"kappa1 {kappa:.17g}\n")
        f.write(f"lu_backward_error {res:.17g}\n")
        f.write(f"x_norm2 {np.linalg.norm(x):.17g}\n")
        f.write(f"x_norminf {np.abs(x).max():.17g}\n")
        f.write("# index re im\n")
        for i in idx:
            f.write(f"{i} {x[i].real:.17g} {x[i].imag:.17g}\n")
    print(f"wrote {OUT}: n={n} kappa1={kappa:.3e} backward error {res:.2e}")


def load():
    """(scalars dict, indices, values) from the golden file."""
    scal = {}
    idx, vals = [], []
    with open(OUT) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if len(parts) == 2:
                scal[parts[0]] = float(parts[1])
            else:
                idx.append(int(parts[0]))
                vals.append(complex(float(parts[1]), float(parts[2])))
    return scal, np.array(idx), np.array(vals)


if __name__ == "__main__":
    main()
