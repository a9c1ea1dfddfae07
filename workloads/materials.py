"""Two-material diffusion inputs (the paper's Section 7 problem C), seeded and synthetic.

The paper's problem C is a finite-element annulus with D = S + 100 J, where
S = exp(1 + sin(pi (x + y))) is smooth and J = H(0.25 + cos(pi x) cos(2 pi y))
marks a second material.  Here the same coefficient sits on a structured
L x L cell-centred grid over [0, 1]^2 (the annulus mesh is not available),
with the 5-point harmonic-mean operator, zero-Dirichlet ghosts on all sides
and a box partition that does not follow the material boundary.

Generating vectors: degree-p monomials of the cell centres, or, material-aware,
the same monomials multiplied by J and by 1 - J (twice the columns: every
generating vector is a piecewise polynomial with respect to the materials).
Builds inputs only; none of the solver's arithmetic lives here.
"""

from __future__ import annotations

import numpy as np

from .generators import STREAM_F, Problem, box_partition, cell_coords, diffusion_cc, monomials, seed_rng

__all__ = ["two_material_coefficient", "material_problem"]


def two_material_coefficient(L: int):
    """(D, J) per cell, numpy shape (L, L), cell centres ((i + 1/2)/L, (j + 1/2)/L)."""
    t = (np.arange(L) + 0.5) / L
    y, x = np.meshgrid(t, t, indexing="ij")
    S = np.exp(1.0 + np.sin(np.pi * (x + y)))
    J = (0.25 + np.cos(np.pi * x) * np.cos(2.0 * np.pi * y) > 0.0).astype(np.float64)
    return S + 100.0 * J, J


def material_problem(L: int, boxes: int, overlap: int, p: int, aware: bool, cfg_id: int = 7,
                     rtol: float = 1e-9, name: str = "") -> Problem:
    """Two-material diffusion on L x L cells; ``aware`` doubles F as [F J, F (1 - J)]."""
    D, J = two_material_coefficient(L)
    A = diffusion_cc(D)
    part = box_partition((L, L), (boxes, boxes))
    F = monomials(cell_coords((L, L)), p)
    if aware:
        j = J.ravel()[:, None]
        F = np.asfortranarray(np.concatenate([F * j, F * (1.0 - j)], axis=1))
    f = seed_rng(cfg_id, STREAM_F).uniform(-1.0, 1.0, L * L)
    return Problem(A=A, F=F, part=part, n_parts=boxes * boxes, overlap=overlap, f=f, rtol=rtol,
                   name=name or f"two_material_{L}{'_aware' if aware else ''}",
                   meta={"grid": (L, L), "p": p, "aware": aware, "J": J})
