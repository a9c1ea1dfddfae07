"""Seeded synthetic problem generators (inputs only, no solver arithmetic).

Every workload is synthetic.  The paper's own test problems (Section 7,
problems A-F) use meshes and SCOTCH partitions that are not available, so
structured-grid problems of the same kind stand in for them:

* cfg1 -- 2D Poisson, 5-point finite differences on a 63x63 interior grid,
  zero Dirichlet boundary eliminated, 4x4 box subdomains, overlap 2,
  6 monomials of degree <= 2.
* cfg2 -- 3D variable-coefficient diffusion, 7-point cell-centred stencil on
  128^3 cells, kappa = exp(g) with g a Gaussian random field (correlation
  length 8 cells, sigma 1), 8^3 boxes of 16^3 cells, overlap 1, p = 2.
* cfg5 -- as cfg2 on 96^3 cells with 12^3-cell boxes (differentiation case).
* cfg4 -- batches of 2D variable-coefficient problems of uneven sizes.

Conventions
-----------
Grid arrays have numpy shape ``(nz, ny, nx)`` (or ``(ny, nx)`` in 2D) so that
the C-order flat index is ``x + nx*(y + ny*z)`` (x fastest).  Matrices are
full symmetric CSR with int64 row pointers, int32 sorted column indices and
float64 values.  Generating vectors ``F`` are n-by-k, column-major
(Fortran order), as the C ABI expects.

Seeds are ``numpy.random.default_rng([cfg_id, stream_id])`` with stream ids
f = 0, kappa/theta = 1, theta_obs = 2, instance sides = 3, sampled cells = 4.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

__all__ = [
    "CSR", "Problem", "seed_rng", "grf", "laplace5_nodes", "diffusion_cc",
    "box_partition", "box_groups", "monomials", "monomial_count", "node_coords_2d",
    "cell_coords", "cfg1", "poisson2d_nodes", "diffusion_problem", "cfg2",
    "cfg5", "cfg5_pair", "cfg4_sides", "cfg4_instance", "STREAM_F",
    "STREAM_KAPPA", "STREAM_KAPPA_OBS", "STREAM_SIDES", "STREAM_CELLS",
]

STREAM_F = 0
STREAM_KAPPA = 1
STREAM_KAPPA_OBS = 2
STREAM_SIDES = 3
STREAM_CELLS = 4


def seed_rng(cfg_id: int, stream_id: int) -> np.random.Generator:
    """Deterministic generator for (workload id, purpose stream)."""
    return np.random.default_rng([int(cfg_id), int(stream_id)])


@dataclass
class CSR:
    """Full symmetric CSR matrix (host arrays)."""

    n: int
    row_ptr: np.ndarray  # int64, n+1
    col_idx: np.ndarray  # int32, nnz, sorted within each row
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = sp.csr_matrix(m)
        m.sum_duplicates()
        m.sort_indices()
        return CSR(
            n=m.shape[0],
            row_ptr=np.ascontiguousarray(m.indptr, dtype=np.int64),
            col_idx=np.ascontiguousarray(m.indices, dtype=np.int32),
            val=np.ascontiguousarray(m.data, dtype=np.float64),
        )


@dataclass
class Problem:
    """One linear system with everything ``ddg_setup`` needs."""

    A: CSR
    F: np.ndarray          # n x k float64, Fortran order
    part: np.ndarray       # int32, n
    n_parts: int
    overlap: int
    f: np.ndarray          # float64, n
    rtol: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.n

    @property
    def k(self) -> int:
        return int(self.F.shape[1])


# ---------------------------------------------------------------------------
# Coefficient fields


def grf(shape, ell: float, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Periodic Gaussian random field with squared-exponential covariance.

    White N(0,1) noise is filtered in Fourier space by a Gaussian of spatial
    standard deviation ell/sqrt(2), which gives covariance exp(-r^2/(2 ell^2)).
    The result is standardised to mean 0 and standard deviation ``sigma``.
    ``shape`` is the numpy array shape (slowest axis first).
    """
    noise = rng.standard_normal(shape)
    s = ell / np.sqrt(2.0)
    spec = np.fft.fftn(noise)
    filt = np.ones(shape)
    for ax, m in enumerate(shape):
        w = 2.0 * np.pi * np.fft.fftfreq(m)
        g = np.exp(-0.5 * (s * w) ** 2)
        sh = [1] * len(shape)
        sh[ax] = m
        filt = filt * g.reshape(sh)
    g = np.real(np.fft.ifftn(spec * filt))
    g = (g - g.mean()) / g.std()
    return sigma * g


# ---------------------------------------------------------------------------
# Operators


def laplace5_nodes(m: int) -> CSR:
    """5-point Laplacian (4, -1) on an m x m interior node grid.

    Zero Dirichlet values on the boundary are eliminated, so boundary
    neighbours simply drop out.  Node id = i + m*j (i along x, fastest).
    """
    n = m * m
    idx = np.arange(n).reshape(m, m)  # [j, i]
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [np.full(n, 4.0)]
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        a = a.ravel(); b = b.ravel()
        rows += [a, b]; cols += [b, a]
        vals += [np.full(a.size, -1.0), np.full(a.size, -1.0)]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return CSR.from_scipy(A)


def diffusion_cc(kappa: np.ndarray, bc: str = "dirichlet") -> CSR:
    """Cell-centred finite-volume diffusion operator with harmonic-mean faces.

    ``kappa`` has shape (ny, nx) or (nz, ny, nx).  Interior face between cells
    L and R carries a_f = 2 kL kR / (kL + kR).  With ``bc="dirichlet"`` each
    boundary face of cell c is a zero-Dirichlet ghost face with coefficient
    2 kc; with ``bc="x0"`` only the faces on x = 0 are (the paper's problem A:
    one Dirichlet face, Neumann elsewhere).  Unit grid spacing.
    """
    if bc not in ("dirichlet", "x0"):
        raise ValueError("bc must be 'dirichlet' or 'x0'")
    kappa = np.asarray(kappa, dtype=np.float64)
    shape = kappa.shape
    n = kappa.size
    diag = np.zeros(shape)
    for ax in range(kappa.ndim):
        m = shape[ax]
        sl_l = [slice(None)] * kappa.ndim
        sl_r = [slice(None)] * kappa.ndim
        sl_l[ax] = slice(0, m - 1)
        sl_r[ax] = slice(1, m)
        kl = kappa[tuple(sl_l)]
        kr = kappa[tuple(sl_r)]
        a = 2.0 * kl * kr / (kl + kr)
        diag[tuple(sl_l)] += a
        diag[tuple(sl_r)] += a
        # ghost faces on both ends of this axis
        lo = [slice(None)] * kappa.ndim
        hi = [slice(None)] * kappa.ndim
        lo[ax] = 0
        hi[ax] = m - 1
        if bc == "dirichlet" or ax == kappa.ndim - 1:
            diag[tuple(lo)] += 2.0 * kappa[tuple(lo)]
        if bc == "dirichlet":
            diag[tuple(hi)] += 2.0 * kappa[tuple(hi)]
    # CSR rows directly, columns ascending: minus-neighbours along axes 0..d-1
    # (largest stride first), the diagonal, then plus-neighbours along d-1..0
    d = kappa.ndim
    strides = [int(np.prod(shape[ax + 1:])) for ax in range(d)]
    slots = []
    for ax in range(d):
        m = shape[ax]
        sl_l = [slice(None)] * d
        sl_r = [slice(None)] * d
        sl_l[ax] = slice(0, m - 1)
        sl_r[ax] = slice(1, m)
        a = 2.0 * kappa[tuple(sl_l)] * kappa[tuple(sl_r)] / (kappa[tuple(sl_l)] + kappa[tuple(sl_r)])
        minus = np.zeros(shape, dtype=bool)
        minus[tuple(sl_r)] = True
        mval = np.zeros(shape)
        mval[tuple(sl_r)] = -a
        plus = np.zeros(shape, dtype=bool)
        plus[tuple(sl_l)] = True
        pval = np.zeros(shape)
        pval[tuple(sl_l)] = -a
        slots.append(((-strides[ax], minus.ravel(), mval.ravel()), (strides[ax], plus.ravel(), pval.ravel())))
    order = [slots[ax][0] for ax in range(d)] + [(0, np.ones(n, dtype=bool), diag.ravel())] + \
            [slots[ax][1] for ax in reversed(range(d))]
    counts = np.zeros(n, dtype=np.int64)
    for _, msk, _ in order:
        counts += msk
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(row_ptr[-1], dtype=np.int32)
    val = np.empty(row_ptr[-1], dtype=np.float64)
    pos = row_ptr[:-1].copy()
    g = np.arange(n, dtype=np.int64)
    for off, msk, v in order:
        rows_ = np.flatnonzero(msk)
        col[pos[rows_]] = g[rows_] + off
        val[pos[rows_]] = v[rows_]
        pos[rows_] += 1
    return CSR(n=n, row_ptr=row_ptr, col_idx=col, val=val)


# ---------------------------------------------------------------------------
# Partitions and generating vectors


def _chunks(L: int, m: int) -> np.ndarray:
    """Chunk id of each of L positions for m near-equal chunks [floor(cL/m), floor((c+1)L/m))."""
    starts = (np.arange(m + 1) * L) // m
    out = np.empty(L, dtype=np.int64)
    for c in range(m):
        out[starts[c]:starts[c + 1]] = c
    return out


def box_partition(shape, boxes) -> np.ndarray:
    """Box partition of a grid of numpy shape ``shape`` (slowest first).

    ``boxes`` gives the number of boxes along each numpy axis.  Box id is
    x-fastest: bx + mx*(by + my*bz).
    """
    shape = tuple(shape)
    boxes = tuple(boxes)
    ids = np.zeros(shape, dtype=np.int64)
    mult = 1
    for ax in reversed(range(len(shape))):  # x axis is the last numpy axis
        c = _chunks(shape[ax], boxes[ax])
        sh = [1] * len(shape)
        sh[ax] = shape[ax]
        ids = ids + mult * c.reshape(sh)
        mult *= boxes[ax]
    return ids.ravel().astype(np.int32)


def box_groups(boxes, group):
    """Coarse partition of the boxes of ``box_partition`` (numpy axis order).

    Box (b_z, b_y, b_x) goes to coarse box (b_z // g_z, ...), numbered x-fastest
    like the boxes themselves; ``group`` gives g per numpy axis.  Returns the
    coarse id of every box and the number of coarse boxes.
    """
    boxes = tuple(boxes)
    group = tuple(group)
    cnt = tuple((m + g - 1) // g for m, g in zip(boxes, group))
    grids = np.meshgrid(*[np.arange(m) for m in boxes], indexing="ij")
    ids = np.zeros(boxes, dtype=np.int64)
    mult = 1
    for ax in reversed(range(len(boxes))):
        ids = ids + mult * (grids[ax] // group[ax])
        mult *= cnt[ax]
    return ids.ravel().astype(np.int32), int(np.prod(cnt))


def monomial_count(dim: int, p: int) -> int:
    from math import comb
    return comb(p + dim, dim)


def monomials(coords, p: int) -> np.ndarray:
    """Monomials of total degree <= p in graded-lex order, n x k Fortran array.

    ``coords`` is a list of 1-D coordinate arrays (x, y[, z]).  Order within a
    degree is lexicographic in the exponent tuple, descending on x first:
    degree 1 -> x, y, z; degree 2 -> x^2, xy, xz, y^2, yz, z^2.
    """
    d = len(coords)
    n = coords[0].size
    cols = []
    for deg in range(p + 1):
        exps = []

        def rec(prefix, remaining, dims_left):
            if dims_left == 1:
                exps.append(prefix + (remaining,))
                return
            for e in range(remaining, -1, -1):
                rec(prefix + (e,), remaining - e, dims_left - 1)

        rec((), deg, d)
        for e in exps:
            v = np.ones(n)
            for c, ei in zip(coords, e):
                if ei:
                    v = v * c ** ei
            cols.append(v)
    return np.asfortranarray(np.stack(cols, axis=1))


def node_coords_2d(m: int):
    """x = i/(m+1), y = j/(m+1) for interior nodes i, j = 1..m, x fastest."""
    t = np.arange(1, m + 1) / (m + 1.0)
    y, x = np.meshgrid(t, t, indexing="ij")
    return [x.ravel(), y.ravel()]


def cell_coords(shape):
    """Cell-centre coordinates (i + 1/2)/L per axis; returned x, y[, z]."""
    axes = [(np.arange(m) + 0.5) / m for m in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    return [g.ravel() for g in reversed(grids)]


# ---------------------------------------------------------------------------
# Workloads


def poisson2d_nodes(m: int, boxes: int, overlap: int, p: int, cfg_id: int = 0,
                    rtol: float = 1e-10, name: str = "") -> Problem:
    """2D node-centred Poisson (5-point), zero Dirichlet, ``boxes`` x ``boxes``."""
    A = laplace5_nodes(m)
    part = box_partition((m, m), (boxes, boxes))
    F = monomials(node_coords_2d(m), p)
    f = seed_rng(cfg_id, STREAM_F).uniform(-1.0, 1.0, m * m)
    return Problem(A=A, F=F, part=part, n_parts=boxes * boxes, overlap=overlap, f=f,
                   rtol=rtol, name=name or f"poisson2d_{m}", meta={"grid": (m, m), "p": p})


def cfg1() -> Problem:
    """2D Poisson, 63x63 interior nodes, 4x4 boxes, overlap 2, p = 2, rtol 1e-10."""
    return poisson2d_nodes(63, 4, 2, 2, cfg_id=0, rtol=1e-10, name="cfg1_poisson2d_63")


def diffusion_problem(shape, boxes, overlap: int, p: int, cfg_id: int, rtol: float,
                      ell: float = 8.0, sigma: float = 1.0, kappa: Optional[np.ndarray] = None,
                      stream: int = STREAM_KAPPA, name: str = "", bc: str = "dirichlet") -> Problem:
    """Cell-centred variable-coefficient diffusion on a box grid.

    kappa = exp(g) with g a GRF (``ell``, ``sigma``) unless ``kappa`` is given;
    sigma = 0 gives the constant-coefficient Poisson operator.
    """
    shape = tuple(shape)
    if kappa is None:
        if sigma == 0.0:
            kappa = np.ones(shape)
        else:
            kappa = np.exp(grf(shape, ell, sigma, seed_rng(cfg_id, stream)))
    A = diffusion_cc(kappa, bc=bc)
    part = box_partition(shape, boxes)
    F = monomials(cell_coords(shape), p)
    n = int(np.prod(shape))
    f = seed_rng(cfg_id, STREAM_F).uniform(-1.0, 1.0, n)
    nparts = int(np.prod(boxes))
    return Problem(A=A, F=F, part=part, n_parts=nparts, overlap=overlap, f=f, rtol=rtol,
                   name=name or f"diffusion_{'x'.join(map(str, shape))}",
                   meta={"grid": shape, "p": p, "kappa": kappa, "boxes": tuple(boxes), "bc": bc})


def cfg2(side: int = 128, box: int = 16) -> Problem:
    """3D variable-kappa diffusion 128^3, 16^3 boxes, overlap 1, p = 2, rtol 1e-8."""
    m = side // box
    return diffusion_problem((side,) * 3, (m,) * 3, 1, 2, cfg_id=1, rtol=1e-8,
                             name=f"cfg2_diffusion3d_{side}")


def cfg5(side: int = 96, box: int = 12) -> Problem:
    """3D diffusion 96^3 with kappa = exp(theta), 12^3 boxes, overlap 1, p = 2."""
    m = side // box
    return diffusion_problem((side,) * 3, (m,) * 3, 1, 2, cfg_id=4, rtol=1e-10,
                             name=f"cfg5_diffusion3d_{side}")


def cfg5_pair(side: int = 96, ell: float = 8.0, sigma: float = 1.0):
    """(theta, theta_obs) for the differentiation workload, numpy shape (s,s,s)."""
    shape = (side,) * 3
    th = grf(shape, ell, sigma, seed_rng(4, STREAM_KAPPA))
    th_obs = grf(shape, ell, sigma, seed_rng(4, STREAM_KAPPA_OBS))
    return th, th_obs


def cfg4_sides(count: int = 256, lo: int = 128, hi: int = 512) -> np.ndarray:
    """Side lengths of the batched 2D instances, uniform on {lo..hi}."""
    return seed_rng(3, STREAM_SIDES).integers(lo, hi + 1, size=count)


def cfg4_instance(i: int, L: int, overlap: int = 2, p: int = 3, cell: int = 32,
                  rtol: float = 1e-8) -> Problem:
    """Instance i of the batched workload: L x L cells, kappa = exp(z), z iid N(0,1).

    Boxes: m = max(1, round(L/cell)) near-equal chunks per axis.
    """
    rng_k = seed_rng(1000 + i, STREAM_KAPPA)
    kappa = np.exp(rng_k.standard_normal((L, L)))
    A = diffusion_cc(kappa)
    m = max(1, int(round(L / cell)))
    part = box_partition((L, L), (m, m))
    F = monomials(cell_coords((L, L)), p)
    f = seed_rng(1000 + i, STREAM_F).uniform(-1.0, 1.0, L * L)
    return Problem(A=A, F=F, part=part, n_parts=m * m, overlap=overlap, f=f, rtol=rtol,
                   name=f"cfg4_inst{i}_L{L}", meta={"grid": (L, L), "p": p, "kappa": kappa})
