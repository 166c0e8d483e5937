"""MI355X (gfx950) implementation of the multilevel local-and-parallel eigen-correction
(Li, Han, Xie, You, arXiv:1401.4969): a HIP library behind a C ABI (include/mlc.h) and a
thin ctypes binding.  PyTorch only supplies device memory and the HIP stream."""
from .binding import (BatchSolver, MLCError, Solver, batch_workspace_size, default_opts,  # noqa: F401
                      eigenvalue, load_library, make_desc, solve, workspace_size)


def __getattr__(name):
    if name == "MultilevelEigen":
        from .binding import _multilevel_eigen_cls
        return _multilevel_eigen_cls()
    raise AttributeError(name)
