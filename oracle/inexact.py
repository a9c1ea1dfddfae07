"""Inexact-solve variant of the DDG preconditioner, FP64 oracle (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

Section 7 describes the timed 3D runs: the subdomain problems were smoothed
with successive over-relaxation instead of being solved exactly, and the coarse
problem was solved by conjugate gradients preconditioned with incomplete
Cholesky.  The paper fixes neither the number of sweeps, the relaxation factor,
the order of the rows, nor the inner tolerance; the readings taken here:

* local smoother: symmetric SOR (a forward then a backward sweep, relaxation
  omega, ``sweeps`` such double sweeps from a zero start) on A_i, with the rows
  visited colour by colour in a greedy colouring of the graph of A_i (ascending
  local index, smallest free colour).  Rows of one colour are not coupled, so
  within a colour the order does not matter.  A symmetric smoother keeps the
  preconditioner symmetric under the reversed post-sweep;
* coarse solve: CG on A0 from zero, preconditioned by the zero-fill incomplete
  Cholesky factor of A0 on its block pattern (every entry of the blocks of coupled
  subdomains, a structural pattern: zero values inside it stay in it), stopped at
  a relative residual ``ic_tol`` or after ``ic_maxit`` iterations.  This makes
  the preconditioner depend on its input, so the outer CG uses the
  Polak-Ribiere direction update.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .ddg import DDGOracle, OracleError, subdomain_adjacency


def local_colouring(Ai: sp.csr_matrix) -> np.ndarray:
    """Greedy colouring of the graph of A_i in ascending local index."""
    n = Ai.shape[0]
    col = np.full(n, -1, dtype=np.int64)
    for r in range(n):
        nb = Ai.indices[Ai.indptr[r]:Ai.indptr[r + 1]]
        used = {int(col[c]) for c in nb if c < r}
        c = 0
        while c in used:
            c += 1
        col[r] = c
    return col


class SSORLocal:
    """``sweeps`` symmetric SOR double sweeps on A_i x = b from x = 0, rows by colour."""

    def __init__(self, Ai: sp.csr_matrix, omega: float, sweeps: int):
        if not (0.0 < omega < 2.0) or sweeps < 1:
            raise OracleError("INVALID_ARG", "SSOR needs 0 < omega < 2 and at least one sweep")
        self.A = sp.csr_matrix(Ai)
        self.A.sort_indices()
        self.d = self.A.diagonal()
        self.colour = local_colouring(self.A)
        nc = int(self.colour.max()) + 1 if self.colour.size else 0
        self.groups = [np.flatnonzero(self.colour == c) for c in range(nc)]
        self.omega = omega
        self.sweeps = sweeps

    def _relax(self, rows, b, x):
        # x_r += omega (b_r - (A x)_r) / a_rr for every row of one colour (no mutual couplings)
        x[rows] += self.omega * (b[rows] - self.A[rows] @ x) / self.d[rows]

    def solve(self, b: np.ndarray) -> np.ndarray:
        x = np.zeros_like(b)
        for _ in range(self.sweeps):
            for g in self.groups:
                self._relax(g, b, x)
            for g in reversed(self.groups):
                self._relax(g, b, x)
        return x


def ic0(A: sp.csr_matrix) -> sp.csr_matrix:
    """Zero-fill incomplete Cholesky L L^T ~ A on the lower pattern of A (row by row)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    rows = [dict() for _ in range(n)]   # L[i, j] for j <= i on the pattern
    for i in range(n):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        Li = rows[i]
        for j, a in zip(cols, vals):
            if j > i:
                continue
            s = a
            Lj = rows[j]
            # sum over k < j on both patterns
            for k, v in Li.items():
                if k < j and k in Lj:
                    s -= v * Lj[k]
            if j == i:
                if not s > 0.0:
                    raise OracleError("NOT_SPD", "incomplete Cholesky pivot not positive", i)
                Li[i] = np.sqrt(s)
            else:
                Li[j] = s / Lj[j]
    r, c, v = [], [], []
    for i in range(n):
        for j, x in rows[i].items():
            r.append(i)
            c.append(j)
            v.append(x)
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def ic_pcg(A: sp.csr_matrix, L: sp.csr_matrix, b: np.ndarray, tol: float, maxit: int) -> np.ndarray:
    """CG on A y = b from y = 0 with M = L L^T, stopped at ||r|| <= tol ||b|| or maxit."""
    from scipy.sparse.linalg import spsolve_triangular
    nb = float(np.linalg.norm(b))
    y = np.zeros_like(b)
    if nb == 0.0:
        return y
    Lt = sp.csr_matrix(L.T)

    def prec(r):
        w = spsolve_triangular(L, r, lower=True)
        return spsolve_triangular(Lt, w, lower=False)

    r = b.copy()
    z = prec(r)
    p = z.copy()
    rho = float(r @ z)
    for _ in range(maxit):
        q = A @ p
        alpha = rho / float(p @ q)
        y += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * nb:
            break
        z = prec(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return y


class InexactDDGOracle(DDGOracle):
    """The two-level DDG preconditioner with SSOR local smoothing and, optionally,
    an incomplete-Cholesky-preconditioned CG coarse solve (Section 7's timed 3D code)."""

    def __init__(self, A, F, part, n_parts: int, overlap: int, omega: float = 1.0, sweeps: int = 1,
                 coarse_solver: str = "exact", ic_tol: float = 1e-6, ic_maxit: int = 200, **kw):
        self.omega = omega
        self.sweeps = sweeps
        super().__init__(A, F, part, n_parts, overlap, **kw)
        if coarse_solver not in ("exact", "ic_cg"):
            raise OracleError("INVALID_ARG", "coarse_solver must be 'exact' or 'ic_cg'")
        self.coarse_solver = coarse_solver
        if self.coarse and coarse_solver == "ic_cg":
            adj = subdomain_adjacency(self.A, self.part, self.n_parts)
            # the block pattern of A0 (unknowns of coupled subdomains), kept structurally:
            # an entry of a coupled block belongs to the pattern even when its value is 0
            owner = np.repeat(np.arange(self.n_parts), self.k_counts)
            self.block_mask = adj[owner][:, owner].toarray() > 0
            r, c = np.nonzero(self.block_mask)
            self.A0s = sp.csr_matrix((self.A0[r, c], (r, c)), shape=self.A0.shape)
            self.L0 = ic0(self.A0s)
            self.ic_tol = ic_tol
            self.ic_maxit = ic_maxit

    def _make_local(self, Ai, i):
        return SSORLocal(Ai, self.omega, self.sweeps)

    def coarse_apply(self, v: np.ndarray) -> np.ndarray:
        if self.coarse_solver == "exact":
            return super().coarse_apply(v)
        b0 = self.R0 @ v
        return self.R0.T @ ic_pcg(self.A0s, self.L0, b0, self.ic_tol, self.ic_maxit)
