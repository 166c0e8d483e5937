"""CPU FP64 oracle for the multilevel local-and-parallel eigen-correction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code with the GPU path: it assembles the finite element operators
element by element, builds nodal interpolation by point location, solves every
local problem with a sparse direct factorisation and every small eigenproblem
with a dense generalized symmetric eigensolver.

Modules
  fem     -- meshes, P1 element assembly, nodal interpolation (Section 2.1)
  fem_p2  -- the same for P2 elements (vertex and edge-midpoint nodes)
  mlc  -- the one correction step (Algorithm 4.1) and the multilevel driver
          (Algorithm 4.2), with the readings listed in the design notes.
"""
from .fem import Mesh, make_mesh, assemble, interpolation  # noqa: F401
from .mlc import Hierarchy, OracleResult, solve, direct_eigs  # noqa: F401
