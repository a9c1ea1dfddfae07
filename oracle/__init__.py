"""Plain FP64 CPU oracle of the DDG two-level PCG method (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and it shares no code
with that path: only the seeded input generators in ``workloads`` feed both.
"""

from .ddg import (DDGOracle, OracleError, ThreeLevelOracle, cg_iteration_bound,  # noqa: F401
                  condition_estimate, fractional_iterations, lanczos_ritz, pcg)
from .gradient import coeff_grad_cc, assemble_cc  # noqa: F401
