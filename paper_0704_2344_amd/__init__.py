"""MI355X-native nodal-hexahedral H-field FEM scattering solver.

The solver is the HIP library libfemh.so (C ABI in include/femh.h); this
package holds its sources (csrc/), its build script (build.py) and the
ctypes binding (femh.py).  Importing the package does not load the library;
`femh.load()` (called by every binding object) does, and raises when it has
not been built.
"""
from . import femh  # noqa: F401

__all__ = ["femh"]
