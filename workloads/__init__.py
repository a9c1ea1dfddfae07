"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This package builds problem *inputs* only: sparse SPD operators, right-hand
sides, coefficient fields, subdomain partitions and generating vectors.  It
contains none of the solver's arithmetic (no coarse basis, no Galerkin
product, no Schwarz sweep, no Krylov iteration), so both the oracle and the
HIP path can consume its output without sharing any method code.
"""

from .generators import *  # noqa: F401,F403
