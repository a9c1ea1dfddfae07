"""CSR pattern of the cell-centred diffusion operator assembled by ``ddg_stencil_assemble``.

Cells are numbered x-fastest on an nx x ny x nz grid (nz = 1 is 2D).  Row g
holds, in ascending column order, its existing neighbours z-1, y-1, x-1, the
diagonal, then x+1, y+1, z+1 -- the order in which the assembly kernel writes
the values.  Integer structure only.
"""

from __future__ import annotations

import numpy as np


def cc_pattern(dims):
    """(row_ptr int64[n+1], col_idx int32[nnz]) for grid dims (nx, ny, nz)."""
    nx, ny, nz = (int(d) for d in dims)
    n = nx * ny * nz
    g = np.arange(n, dtype=np.int64)
    x = g % nx
    y = (g // nx) % ny
    z = g // (nx * ny)
    offs = [(-nx * ny, z > 0), (-nx, y > 0), (-1, x > 0), (0, np.ones(n, dtype=bool)),
            (1, x < nx - 1), (nx, y < ny - 1), (nx * ny, z < nz - 1)]
    counts = np.zeros(n, dtype=np.int64)
    for _, m in offs:
        counts += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cols = np.empty(row_ptr[-1], dtype=np.int64)
    pos = row_ptr[:-1].copy()
    for off, m in offs:
        idx = np.flatnonzero(m)
        cols[pos[idx]] = g[idx] + off
        pos[idx] += 1
    return row_ptr, cols.astype(np.int32)
