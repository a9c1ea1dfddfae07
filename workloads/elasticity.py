"""3D linear elasticity on trilinear (Q1) hexahedra: a seeded vector-valued workload.

The unit cube is cut into nel^3 cubic elements (h = 1/nel) with
(nel+1)^3 nodes; the nodes of the face x = 0 are clamped (their three
displacement components are removed).  Young's modulus is log-normal per
element, E_e = exp(sigma z_e) with z_e iid N(0, 1); Poisson ratio nu.  The
element stiffness is the standard displacement formulation integrated by
2x2x2 Gauss quadrature; because all elements are the same cube, every
element matrix is E_e times one reference matrix.  The load vector is
f ~ U(-1, 1) per free degree of freedom.

Degrees of freedom are node-major: dof = 3 * (free node index) + component,
free nodes numbered x-fastest.  The generating vectors follow the paper's
per-component rule for elasticity (Section 7, problem E): for each
component c, the monomials {1, x, y, z} times the unit vector e_c, 12 in all.

The partition grows subdomains by breadth-first search over the 26-neighbour
node graph from the lowest-numbered unassigned node, each to a seeded target
size drawn uniformly from a dof range; fragments below the minimum are then
merged into their smallest neighbouring subdomain.  Subdomain ids are
renumbered in order of their lowest node.
"""

from __future__ import annotations

import numpy as np

from .generators import CSR, Problem, seed_rng

__all__ = ["q1_reference_stiffness", "elasticity_q1", "graph_grow_partition", "STREAM_E", "STREAM_PART"]

STREAM_E = 1
STREAM_PART = 5


def q1_reference_stiffness(h: float, nu: float) -> np.ndarray:
    """24 x 24 stiffness of a cube of edge h for E = 1 (dofs: 3 per local node, node a = i + 2j + 4k)."""
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2.0 * mu
    D[3:, 3:] = np.eye(3) * mu
    signs = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)]) * 2.0 - 1.0  # +-1
    g = 1.0 / np.sqrt(3.0)
    K = np.zeros((24, 24))
    for gx in (-g, g):
        for gy in (-g, g):
            for gz in (-g, g):
                xi = np.array([gx, gy, gz])
                # dN_a/dxi_d = s_ad/8 * prod_{e != d} (1 + s_ae xi_e)
                dN = np.empty((8, 3))
                for a in range(8):
                    t = 1.0 + signs[a] * xi
                    for d in range(3):
                        dN[a, d] = signs[a, d] / 8.0 * np.prod(np.delete(t, d))
                dN *= 2.0 / h  # d/dx = (2/h) d/dxi
                B = np.zeros((6, 24))
                for a in range(8):
                    bx, by, bz = dN[a]
                    c = 3 * a
                    B[0, c] = bx
                    B[1, c + 1] = by
                    B[2, c + 2] = bz
                    B[3, c + 1], B[3, c + 2] = bz, by   # gamma_yz
                    B[4, c], B[4, c + 2] = bz, bx       # gamma_xz
                    B[5, c], B[5, c + 1] = by, bx       # gamma_xy
                K += B.T @ D @ B * (h / 2.0) ** 3
    return 0.5 * (K + K.T)


def graph_grow_partition(dims, free: np.ndarray, rng: np.random.Generator, lo_dofs: int, hi_dofs: int,
                         min_dofs: int, dofs_per_node: int = 3) -> np.ndarray:
    """Subdomain id per free node (see the module docstring).

    dims = (nx, ny, nz) nodes, x fastest; free[node] marks nodes that carry dofs.
    """
    nx, ny, nz = dims
    nn = nx * ny * nz
    part = np.full(nn, -1, dtype=np.int64)
    part[~free] = -2  # never assigned
    xs = np.arange(nn) % nx
    ys = (np.arange(nn) // nx) % ny
    zs = np.arange(nn) // (nx * ny)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]

    def neighbours(nodes):
        out = []
        x, y, z = xs[nodes], ys[nodes], zs[nodes]
        for dx, dy, dz in offs:
            ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
            out.append(nodes[ok] + dx + nx * (dy + ny * dz))
        return np.unique(np.concatenate(out)) if out else np.empty(0, dtype=np.int64)

    pid = 0
    cursor = 0
    while True:
        while cursor < nn and part[cursor] != -1:
            cursor += 1
        if cursor >= nn:
            break
        target = int(rng.integers(lo_dofs, hi_dofs + 1)) // dofs_per_node
        part[cursor] = pid
        count = 1
        front = np.array([cursor], dtype=np.int64)
        while count < target and front.size:
            cand = neighbours(front)
            cand = cand[part[cand] == -1]
            if cand.size > target - count:
                cand = cand[:target - count]
            part[cand] = pid
            count += cand.size
            front = cand
        pid += 1
    # merge fragments below the minimum into the smallest neighbouring subdomain
    min_nodes = (min_dofs + dofs_per_node - 1) // dofs_per_node
    while True:
        sizes = np.bincount(part[part >= 0], minlength=pid)
        small = [p for p in range(pid) if 0 < sizes[p] < min_nodes]
        if not small:
            break
        merged = False
        for p in small:
            nodes = np.flatnonzero(part == p)
            nb = neighbours(nodes)
            nbp = np.unique(part[nb])
            nbp = nbp[(nbp >= 0) & (nbp != p)]
            if nbp.size == 0:
                continue
            q = nbp[np.argmin(sizes[nbp])]
            part[nodes] = q
            sizes[q] += sizes[p]
            sizes[p] = 0
            merged = True
        if not merged:
            break
    # renumber by lowest node
    ids = part[part >= 0]
    first = {}
    for node in np.flatnonzero(part >= 0):
        p = part[node]
        if p not in first:
            first[p] = len(first)
    remap = np.full(pid, -1, dtype=np.int64)
    for p, newp in first.items():
        remap[p] = newp
    out = np.full(nn, -1, dtype=np.int32)
    out[part >= 0] = remap[ids]
    return out


def elasticity_q1(nel: int = 64, nu: float = 0.3, sigma: float = 0.5, cfg_id: int = 2,
                  part_dofs=(2000, 8000), min_dofs: int = 2000, overlap: int = 1, rtol: float = 1e-8,
                  name: str = "") -> Problem:
    """Clamped Q1 elasticity on nel^3 elements (defaults: 64^3, 811,200 free dofs)."""
    nx = ny = nz = nel + 1
    nn = nx * ny * nz
    h = 1.0 / nel
    Kref = q1_reference_stiffness(h, nu)
    E = np.exp(sigma * seed_rng(cfg_id, STREAM_E).standard_normal((nel, nel, nel)))  # (ez, ey, ex)
    # node-pair blocks: val[node, offset(27), 3, 3], offset index (dx+1) + 3(dy+1) + 9(dz+1)
    blocks = np.zeros((nz, ny, nx, 27, 3, 3))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
            d = (bx - ax + 1) + 3 * (by - ay + 1) + 9 * (bz - az + 1)
            kab = Kref[3 * a:3 * a + 3, 3 * b:3 * b + 3]
            # element (ex, ey, ez) touches node (ex+ax, ey+ay, ez+az) as local node a
            blocks[az:az + nel, ay:ay + nel, ax:ax + nel, d] += E[..., None, None] * kab
    blocks = blocks.reshape(nn, 27, 3, 3)
    xs = np.arange(nn) % nx
    ys = (np.arange(nn) // nx) % ny
    zs = np.arange(nn) // (nx * ny)
    # exact symmetry: block (p, q) and block (q, p)^T are sums of the same terms in
    # different orders; average them so that A = A^T holds bit for bit
    for d in range(14):  # offsets with d < 13 mirror to 26 - d; d = 13 is the node itself
        dx, dy, dz = d % 3 - 1, (d // 3) % 3 - 1, d // 9 - 1
        if d == 13:
            blocks[:, 13] = 0.5 * (blocks[:, 13] + np.swapaxes(blocks[:, 13], 1, 2))
            continue
        x, y, z = xs + dx, ys + dy, zs + dz
        ok = np.flatnonzero((x >= 0) & (x < nx) & (y >= 0) & (y < ny) & (z >= 0) & (z < nz))
        q = x[ok] + nx * (y[ok] + ny * z[ok])
        avg = 0.5 * (blocks[ok, d] + np.swapaxes(blocks[q, 26 - d], 1, 2))
        blocks[ok, d] = avg
        blocks[q, 26 - d] = np.swapaxes(avg, 1, 2)
    free = xs > 0
    fidx = np.full(nn, -1, dtype=np.int64)
    fidx[free] = np.arange(int(free.sum()))
    nfree = int(free.sum())
    n = 3 * nfree
    # rows: free node p, component c; columns ascending = neighbours in ascending node order
    # (offsets ordered dz, dy, dx ascending), then component
    cols_per = []
    vals_per = []
    fnodes = np.flatnonzero(free)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                d = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                x, y, z = xs[fnodes] + dx, ys[fnodes] + dy, zs[fnodes] + dz
                ok = (x >= 1) & (x < nx) & (y >= 0) & (y < ny) & (z >= 0) & (z < nz)
                q = np.where(ok, x + nx * (y + ny * z), 0)
                cols_per.append(np.where(ok, fidx[q], -1))
                vals_per.append(blocks[fnodes, d])  # (nfree, 3, 3)
    nbr = np.stack(cols_per, axis=1)                # (nfree, 27) free-node column or -1
    vb = np.stack(vals_per, axis=1)                 # (nfree, 27, 3, 3)
    present = nbr >= 0
    cnt = present.sum(axis=1) * 3                   # entries per row (same for the 3 components)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.repeat(cnt, 3), out=row_ptr[1:])
    # column indices and values, row by row: for node p, component c: for each present neighbour q: 3 columns
    col = np.empty(row_ptr[-1], dtype=np.int32)
    val = np.empty(row_ptr[-1], dtype=np.float64)
    # slot position of neighbour j within the row: 3 * (number of present neighbours before j)
    before = np.cumsum(present, axis=1) - present
    for c in range(3):
        rows = 3 * np.arange(nfree) + c
        base = row_ptr[rows]
        for j in range(27):
            m = present[:, j]
            pos = base[m] + 3 * before[m, j]
            qn = nbr[m, j]
            for e in range(3):
                col[pos + e] = 3 * qn + e
                val[pos + e] = vb[m, j, c, e]
    A = CSR(n=n, row_ptr=row_ptr, col_idx=col, val=val)
    # generating vectors: per component, {1, x, y, z} e_c
    F = np.zeros((n, 12), order="F")
    coords = [xs[fnodes] * h, ys[fnodes] * h, zs[fnodes] * h]
    monos = [np.ones(nfree)] + coords
    for c in range(3):
        for m in range(4):
            F[c::3, 4 * c + m] = monos[m]
    npart = graph_grow_partition((nx, ny, nz), free, seed_rng(cfg_id, STREAM_PART), part_dofs[0], part_dofs[1],
                                 min_dofs)
    part_nodes = npart[fnodes]
    part = np.repeat(part_nodes, 3).astype(np.int32)
    n_parts = int(part.max()) + 1
    f = seed_rng(cfg_id, 0).uniform(-1.0, 1.0, n)
    return Problem(A=A, F=F, part=part, n_parts=n_parts, overlap=overlap, f=f, rtol=rtol,
                   name=name or f"elasticity_q1_{nel}", meta={"nel": nel, "E": E, "nu": nu})
