"""MI355X (gfx950) DDG two-level PCG: HIP kernels behind a C ABI, Python binding.

``DDGSolver`` wraps a ``ddg_handle`` (see include/ddg.h).  Importing the
package does not load the shared library; the first solver does, and fails
loudly when ``libddg.so`` has not been built.
"""

from ._lib import DDGError  # noqa: F401


def __getattr__(name):
    if name in ("DDGSolver", "DDGBatchSolver", "tune_batched", "stencil_assemble", "stencil_coeff_grad"):
        from . import solver
        return getattr(solver, name)
    if name in ("DDGSolveFunction", "ddg_solve_fn", "DiffusionSolver"):
        from . import autograd
        return getattr(autograd, name)
    if name == "cc_pattern":
        from .stencil import cc_pattern
        return cc_pattern
    raise AttributeError(name)
