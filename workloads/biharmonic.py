"""Biharmonic inputs (the paper's Section 7 problem F), seeded and synthetic.

Builds the operator, partition, generating vectors and right-hand side only;
none of the solver's arithmetic lives here.

Operator: the 13-point finite-difference stencil of the biharmonic operator on
an m x m grid of interior nodes with unit spacing,

    20 u(i,j) - 8 [u(i+-1,j) + u(i,j+-1)] + 2 [u(i+-1,j+-1)] + [u(i+-2,j) + u(i,j+-2)],

with homogeneous Dirichlet and Neumann conditions on every side (a clamped
plate): the boundary nodes carry u = 0, and the node beyond each boundary
mirrors the first interior node (a central difference of du/dn = 0 at the
boundary node), so a row next to a side gains +1 on its diagonal per such side.
Node id i + m j (x fastest), coordinates ((i+1)/(m+1), (j+1)/(m+1)).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .generators import CSR, STREAM_F, Problem, box_partition, monomials, node_coords_2d, seed_rng

__all__ = ["biharmonic13", "biharmonic_problem"]

# (di, dj, coefficient) of the 13-point stencil
_STENCIL = [(0, 0, 20.0)]
_STENCIL += [(d, 0, -8.0) for d in (-1, 1)] + [(0, d, -8.0) for d in (-1, 1)]
_STENCIL += [(a, b, 2.0) for a in (-1, 1) for b in (-1, 1)]
_STENCIL += [(d, 0, 1.0) for d in (-2, 2)] + [(0, d, 1.0) for d in (-2, 2)]


def biharmonic13(m: int) -> CSR:
    """Clamped-plate 13-point biharmonic operator on m x m interior nodes."""
    if m < 1:
        raise ValueError("m must be positive")
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    row = i + m * j
    rows, cols, vals = [], [], []
    for di, dj, c in _STENCIL:
        ii, jj = i + di, j + dj
        inside = (ii >= 0) & (ii < m) & (jj >= 0) & (jj < m)
        rows.append(row[inside])
        cols.append((ii + m * jj)[inside])
        vals.append(np.full(int(inside.sum()), c))
    # mirrored nodes beyond the sides: +1 on the diagonal per adjacent side
    extra = (i == 0).astype(float) + (i == m - 1) + (j == 0) + (j == m - 1)
    rows.append(row)
    cols.append(row)
    vals.append(extra)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m * m, m * m))
    A.sum_duplicates()
    A.eliminate_zeros()
    return CSR.from_scipy(A)


def biharmonic_problem(m: int, boxes: int, overlap: int, p: int, cfg_id: int = 6, rtol: float = 1e-6,
                       name: str = "") -> Problem:
    """Biharmonic on m x m nodes, ``boxes`` x ``boxes`` box partition, degree-p monomials."""
    A = biharmonic13(m)
    part = box_partition((m, m), (boxes, boxes))
    F = monomials(node_coords_2d(m), p)
    f = seed_rng(cfg_id, STREAM_F).uniform(-1.0, 1.0, m * m)
    return Problem(A=A, F=F, part=part, n_parts=boxes * boxes, overlap=overlap, f=f, rtol=rtol,
                   name=name or f"biharmonic_{m}", meta={"grid": (m, m), "p": p, "boxes": (boxes, boxes)})
