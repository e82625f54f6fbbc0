"""CPU FP64 oracle for the nodal-hexahedral H-field scattering solver.

TEST INFRASTRUCTURE.  This package is the plain, slow reference against which
the HIP library is checked.  Only the test suite, the smoke check
(`__graft_entry__.smoke`) and the CPU-baseline leg of `bench.py` may import
it; the product path never does, and it never imports the product package.
It shares no code, table or constant generator with the HIP library: both
sides only take the same seeded inputs (the `workloads` package).

Modules:
  fem    -- element tables by Gauss quadrature, global assembly, RHS (eqs. (1)-(4))
  solve  -- dense LU, sparse LU and COCG with diagonal preconditioning (section 3.1.5)
"""
from . import fem, solve  # noqa: F401
