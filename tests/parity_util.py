"""Shared parity bars of the GPU tests (FP64 and mixed modes against the oracle).

FP64 mode: the GPU's u within 1e-10 (relative, 2-norm) of the oracle's, with
iteration counts within one.  When the counts differ by one, both sides are
run again for exactly the smaller count (rtol 0, capped iterations), so u is
always compared at a common iteration.  Mixed modes: the true final residual
||f - A u|| / ||f||, computed on the CPU from the GPU's u, at most 1e-8, and
the iteration count within one of the FP64 oracle's at the same tolerance.
"""

from __future__ import annotations

import numpy as np

FP64_U_TOL = 1e-10
MIXED_RES_TOL = 1e-8


def rel(a, b) -> float:
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def fp64_u_error(u_gpu, it_gpu, x_or, it_or, rerun_gpu, rerun_oracle):
    """Relative error of the GPU's u against the oracle at a common iteration count.

    rerun_gpu(m) / rerun_oracle(m) return the iterate after exactly m
    iterations (rtol 0).  Returns (error, compared_at)."""
    assert abs(it_gpu - it_or) <= 1, f"iteration counts {it_gpu} vs {it_or} differ by more than one"
    if it_gpu == it_or:
        return rel(u_gpu, x_or), it_gpu
    m = min(it_gpu, it_or)
    return rel(rerun_gpu(m), rerun_oracle(m)), m


def true_rel_res(A, u, f) -> float:
    return float(np.linalg.norm(f - A @ u)) / float(np.linalg.norm(f))
