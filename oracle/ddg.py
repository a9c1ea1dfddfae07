"""FP64 CPU oracle: DDG coarse grid + two-level symmetric multiplicative Schwarz PCG.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``; never by the product path.

Each step follows the paper (Edwards and Bridson, "The Discretely-
Discontinuous Galerkin Coarse Grid for Domain Decomposition"):

* coarse basis: Section 4 -- restrict every generating vector to every
  non-overlapping subdomain, orthonormalise each subdomain's block
  independently, discard rank-deficient columns (Fig. 2 gives the column
  layout: subdomain-major, k slots per subdomain);
* coarse operator: Section 4 -- A0 = R0 A R0^T, coarse solve A0 u0 = R0 f;
* overlapping subdomains: Section 6 -- expand each partition set to graph
  distance Delta in the graph of A, local matrices A_i = R~_i A R~_i^T
  solved exactly;
* preconditioner: Section 6 -- multiplicative update over subdomains
  (the Section 6 update equation), one pass as pre-smoother, the coarse
  correction, one pass in reverse order as post-smoother;
* Krylov: CG with this preconditioner, x0 = 0 (Section 7 protocol),
  1000-iteration cap.

Readings where the paper is silent (each listed in the design notes):
rank tolerance |R_jj| <= 1e-10 |R_11| with column-pivoted Householder QR;
the graph of A is its stored pattern; the subdomain visiting order is the
greedy conflict colouring in increasing subdomain id, colour-major,
ascending id inside a colour (descending in the post-sweep); CG stops when
||r_k||_2 <= rtol ||f||_2 using the recurrence residual, and the iteration
count is the number of products A p.

Local solves use LAPACK banded Cholesky (dense Cholesky for small blocks);
the coarse solve uses a dense LAPACK Cholesky of A0.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class OracleError(Exception):
    """Error with a code name matching the C ABI's status codes."""

    def __init__(self, code: str, msg: str, where: int = -1):
        super().__init__(f"{code}: {msg}")
        self.code = code
        self.where = where


def _as_csr(A) -> sp.csr_matrix:
    if hasattr(A, "to_scipy"):
        A = A.to_scipy()
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    return A


# ---------------------------------------------------------------------------
# Setup steps


def validate(A: sp.csr_matrix, F: np.ndarray, part: np.ndarray, n_parts: int, overlap: int):
    """Input checks: square symmetric A with positive diagonal, valid partition, finite F."""
    n = A.shape[0]
    if A.shape[0] != A.shape[1]:
        raise OracleError("INVALID_ARG", "A is not square")
    d = A.diagonal()
    if not np.all(d > 0):
        raise OracleError("NOT_SPD", "non-positive diagonal entry", int(np.argmin(d)))
    asym = abs(A - A.T)
    scale = abs(A).max() if A.nnz else 1.0
    if asym.nnz and asym.max() > 1e-14 * scale:
        raise OracleError("INVALID_ARG", "A is not symmetric")
    part = np.asarray(part)
    if part.shape != (n,) or n_parts < 1 or part.min() < 0 or part.max() >= n_parts:
        raise OracleError("INVALID_ARG", "partition out of range")
    counts = np.bincount(part, minlength=n_parts)
    if np.any(counts == 0):
        raise OracleError("INVALID_ARG", "empty subdomain", int(np.argmin(counts)))
    if overlap < 0:
        raise OracleError("INVALID_ARG", "negative overlap")
    if F is not None and F.size and not np.all(np.isfinite(F)):
        raise OracleError("INVALID_ARG", "non-finite generating vectors")


def coarse_basis(F: np.ndarray, part: np.ndarray, n_parts: int, rank_tol: float):
    """DDG coarse restriction (Section 4, Fig. 2).

    For each subdomain i the block F[Omega_i, :] is orthonormalised with
    column-pivoted Householder QR; columns whose |R_jj| falls at or below
    rank_tol * |R_11| are discarded.  Returns (R0 as sparse N_c x n,
    per-subdomain kept counts, per-subdomain offsets, per-subdomain Q blocks,
    per-subdomain node lists).
    """
    n, k = F.shape
    rows, cols, vals = [], [], []
    counts = np.zeros(n_parts, dtype=np.int64)
    offsets = np.zeros(n_parts + 1, dtype=np.int64)
    Qs, nodes = [], []
    off = 0
    for i in range(n_parts):
        idx = np.flatnonzero(part == i)
        B = F[idx, :]
        Q, R, _piv = sla.qr(B, mode="economic", pivoting=True)
        diag = np.abs(np.diag(R))
        if diag.size == 0 or diag[0] == 0.0:
            raise OracleError("RANK", "every generating vector vanishes on a subdomain", i)
        keep = int(np.count_nonzero(diag > rank_tol * diag[0]))
        Qi = Q[:, :keep]
        Qs.append(Qi)
        nodes.append(idx)
        counts[i] = keep
        offsets[i] = off
        for j in range(keep):
            rows.append(np.full(idx.size, off + j))
            cols.append(idx)
            vals.append(Qi[:, j])
        off += keep
    offsets[n_parts] = off
    R0 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(off, n))
    return R0, counts, offsets, Qs, nodes


def galerkin(A: sp.csr_matrix, R0: sp.csr_matrix) -> np.ndarray:
    """A0 = R0 A R0^T (Section 4), dense and symmetrised."""
    A0 = (R0 @ A @ R0.T).toarray()
    return 0.5 * (A0 + A0.T)


def overlap_sets(A: sp.csr_matrix, part: np.ndarray, n_parts: int, delta: int):
    """Expanded subdomains (Section 6): graph distance <= delta from Omega_i, ascending."""
    sets = []
    for i in range(n_parts):
        S = np.flatnonzero(part == i)
        front = S
        for _ in range(delta):
            nb = np.unique(A[front].indices)
            new = np.setdiff1d(nb, S, assume_unique=True)
            S = np.union1d(S, new)
            front = new
        sets.append(S.astype(np.int64))
    return sets


def closed_neighbourhood(A: sp.csr_matrix, S: np.ndarray) -> np.ndarray:
    """N[S] = S plus every node coupled to S by a stored entry of A."""
    return np.union1d(S, np.unique(A[S].indices))


def conflict_lists(A: sp.csr_matrix, sets, n: int):
    """j conflicts with i when the expanded set of j meets N[expanded set of i]."""
    n_parts = len(sets)
    rows = np.concatenate([np.full(s.size, i) for i, s in enumerate(sets)])
    cols = np.concatenate(sets)
    member = sp.csc_matrix((np.ones(rows.size, dtype=np.int8), (rows, cols)), shape=(n_parts, n))
    out = []
    for i, s in enumerate(sets):
        N = closed_neighbourhood(A, s)
        js = np.unique(member[:, N].indices)
        out.append(js[js != i])
    return out


def greedy_colouring(conflicts):
    """colour(i) = smallest colour not used by a conflicting j < i, in increasing i."""
    colours = np.full(len(conflicts), -1, dtype=np.int64)
    for i, js in enumerate(conflicts):
        used = {int(colours[j]) for j in js if j < i}
        c = 0
        while c in used:
            c += 1
        colours[i] = c
    return colours


def _lower_bandwidth(M: sp.csr_matrix) -> int:
    bw = 0
    for j in range(M.shape[0]):
        cs = M.indices[M.indptr[j]:M.indptr[j + 1]]
        if cs.size:
            bw = max(bw, j - int(cs.min()))
    return bw


class _LocalSolver:
    """Exact solve with A_i = A[set, set] (Section 6): banded or dense LAPACK Cholesky."""

    def __init__(self, Ai: sp.csr_matrix, sub: int):
        n = Ai.shape[0]
        bw = _lower_bandwidth(Ai)
        self.n = n
        try:
            if n <= 256 or 2 * bw >= n:
                self.kind = "dense"
                self.fac = sla.cho_factor(Ai.toarray(), lower=True, check_finite=True)
            else:
                self.kind = "banded"
                ab = np.zeros((bw + 1, n))
                coo = sp.tril(Ai).tocoo()
                ab[coo.row - coo.col, coo.col] = coo.data
                self.fac = sla.cholesky_banded(ab, lower=True, check_finite=True)
        except np.linalg.LinAlgError as exc:
            raise OracleError("NOT_SPD", f"local Cholesky failed: {exc}", sub) from None
        if self.kind == "dense" and not np.all(np.diag(self.fac[0]) > 0):
            raise OracleError("NOT_SPD", "local Cholesky failed", sub)

    def solve(self, b: np.ndarray) -> np.ndarray:
        if self.kind == "dense":
            return sla.cho_solve(self.fac, b, check_finite=False)
        return sla.cho_solve_banded((self.fac, True), b, check_finite=False)


class DDGOracle:
    """Setup + application of the two-level DDG preconditioner, FP64.

    ``k = 0`` columns (F with no columns) or ``coarse=False`` disables the
    coarse step (a test switch used to check the one-level reductions).
    """

    def __init__(self, A, F, part, n_parts: int, overlap: int, rank_tol: float = 1e-10,
                 coarse: bool = True, colours=None):
        A = _as_csr(A)
        part = np.asarray(part, dtype=np.int64)
        F = np.zeros((A.shape[0], 0)) if F is None else np.asarray(F, dtype=np.float64)
        validate(A, F, part, n_parts, overlap)
        self.A = A
        self.n = A.shape[0]
        self.part = part
        self.n_parts = n_parts
        self.overlap = overlap
        self.coarse = bool(coarse and F.shape[1] > 0)
        if self.coarse:
            self.R0, self.k_counts, self.k_offsets, self.Qs, self.nodes = coarse_basis(
                F, part, n_parts, rank_tol)
            self.A0 = galerkin(A, self.R0)
            try:
                self.A0_fac = sla.cho_factor(self.A0, lower=True)
            except np.linalg.LinAlgError as exc:
                raise OracleError("NOT_SPD", f"coarse Cholesky failed: {exc}") from None
        else:
            self.R0 = None
            self.A0 = None
        self.sets = overlap_sets(A, part, n_parts, overlap)
        self.conflicts = conflict_lists(A, self.sets, self.n)
        self.colours = np.asarray(colours) if colours is not None else greedy_colouring(self.conflicts)
        self.n_colours = int(self.colours.max()) + 1
        self.order = [np.flatnonzero(self.colours == c) for c in range(self.n_colours)]
        self.rows = [A[s] for s in self.sets]
        self.local = [self._make_local(A[s][:, s], i) for i, s in enumerate(self.sets)]

    def _make_local(self, Ai, i):
        """Exact solver of the local problem A_i (Section 6: solved exactly)."""
        return _LocalSolver(Ai, i)

    # -- pieces ------------------------------------------------------------

    @property
    def n_coarse(self) -> int:
        return 0 if not self.coarse else int(self.R0.shape[0])

    def coarse_apply(self, v: np.ndarray) -> np.ndarray:
        """R0^T A0^{-1} R0 v (Section 4 coarse approximation)."""
        u0 = sla.cho_solve(self.A0_fac, self.R0 @ v)
        return self.R0.T @ u0

    def local_update(self, i: int, r: np.ndarray, e: np.ndarray, e_read=None):
        """e[set_i] += A_i^{-1} (r - A e)[set_i]  (Section 6 update equation)."""
        src = e if e_read is None else e_read
        s = self.sets[i]
        b = r[s] - self.rows[i] @ src
        return s, self.local[i].solve(b)

    def apply(self, r: np.ndarray, snapshot: bool = False, trace=None) -> np.ndarray:
        """M^{-1} r: pre-sweep (colour-major), coarse, reverse post-sweep (Section 6).

        ``snapshot=True`` evaluates every subdomain of a colour from the e
        before that colour (a check that same-colour subdomains are independent).
        ``trace`` (a list) receives (event, subdomain, e-copy) after each step.
        """
        r = np.asarray(r, dtype=np.float64)
        e = np.zeros(self.n)
        seq = [(c, list(self.order[c])) for c in range(self.n_colours)]
        for c, ids in seq:
            self._colour(ids, r, e, snapshot, trace)
        if self.coarse:
            e += self.coarse_apply(r - self.A @ e)
            if trace is not None:
                trace.append(("coarse", -1, e.copy()))
        for c, ids in reversed(seq):
            self._colour(list(reversed(ids)), r, e, snapshot, trace)
        return e

    def _colour(self, ids, r, e, snapshot, trace):
        if snapshot:
            e0 = e.copy()
            ups = [self.local_update(i, r, e, e_read=e0) for i in ids]
            for s, x in ups:
                e[s] += x
        else:
            for i in ids:
                s, x = self.local_update(i, r, e)
                e[s] += x
                if trace is not None:
                    trace.append(("local", i, e.copy()))

    def dense_operator(self) -> np.ndarray:
        """M^{-1} as a dense matrix (tiny problems only)."""
        I = np.eye(self.n)
        return np.stack([self.apply(I[:, j]) for j in range(self.n)], axis=1)

    def pcg(self, f, rtol: float, max_iter: int = 1000, variant: str = "fr", trace: bool = False):
        return pcg(self.A, self.apply, f, rtol, max_iter, variant=variant, trace=trace)


def pcg(A, apply_minv, f, rtol: float, max_iter: int = 1000, variant: str = "fr", trace: bool = False):
    """Preconditioned CG from x0 = 0 (Section 7 protocol).

    Stops at the first k with ||r_k|| <= rtol ||f|| (recurrence residual);
    the iteration count is the number of products A p.  Returns
    (x, iterations, info) with info holding status, residual history, the
    CG coefficients (alpha, beta) and the true relative residual.

    ``variant`` picks the direction update: "fr" (Fletcher-Reeves,
    beta = r_new^T z_new / r^T z) or "pr" (Polak-Ribiere,
    beta = z_new^T (r_new - r) / r^T z), which stays usable when the
    preconditioner is not exactly a fixed linear operator.  With
    ``trace`` the search directions are kept in info["p"].
    """
    if variant not in ("fr", "pr"):
        raise OracleError("INVALID_ARG", "variant must be 'fr' or 'pr'")
    A = _as_csr(A)
    f = np.asarray(f, dtype=np.float64)
    nf = float(np.linalg.norm(f))
    x = np.zeros_like(f)
    info = {"status": "ok", "alpha": [], "beta": [], "res": [1.0 if nf > 0 else 0.0]}
    if nf == 0.0:
        info.update(true_rel_res=0.0, rel_res=0.0)
        return x, 0, info
    if not np.all(np.isfinite(f)):
        raise OracleError("INVALID_ARG", "non-finite right-hand side")
    r = f.copy()
    z = apply_minv(r)
    p = z.copy()
    rho = float(r @ z)
    if trace:
        info["p"] = [p.copy()]
    it = 0
    while True:
        if it >= max_iter:
            info["status"] = "no_convergence"
            break
        q = A @ p
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0 or not np.isfinite(rho) or rho <= 0.0:
            info["status"] = "breakdown"
            break
        alpha = rho / pq
        x += alpha * p
        r_prev = r.copy() if variant == "pr" else None
        r -= alpha * q
        it += 1
        rn = float(np.linalg.norm(r))
        info["alpha"].append(alpha)
        info["res"].append(rn / nf)
        if rn <= rtol * nf:
            break
        z = apply_minv(r)
        rho_new = float(r @ z)
        if variant == "pr":
            beta = float(z @ (r - r_prev)) / rho
        else:
            beta = rho_new / rho
        info["beta"].append(beta)
        p = z + beta * p
        rho = rho_new
        if trace:
            info["p"].append(p.copy())
    info["rel_res"] = info["res"][-1]
    info["true_rel_res"] = float(np.linalg.norm(f - A @ x)) / nf
    return x, it, info


def lanczos_ritz(alphas, betas) -> np.ndarray:
    """Ritz values of the preconditioned operator from CG coefficients.

    The CG coefficients define the Lanczos tridiagonal T with
    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1} and
    T_{j,j+1} = sqrt(beta_j)/alpha_j (standard CG-Lanczos relation).
    """
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return np.linalg.eigvalsh(T)


def fractional_iterations(res, tol: float) -> float:
    """Fractional iteration count (Section 7 protocol).

    ``res[k]`` is the relative residual after k iterations (res[0] = 1).
    The log-residual is interpolated linearly between the last iterate
    above the tolerance and the first one at or below it; the fractional
    count is where that line meets log(tol).  Returns nan if no iterate
    reaches tol, and 0 if res[0] already does.
    """
    res = np.asarray(res, dtype=np.float64)
    hit = np.flatnonzero(res <= tol)
    if hit.size == 0:
        return float("nan")
    k = int(hit[0])
    if k == 0:
        return 0.0
    a, b = np.log(res[k - 1]), np.log(res[k])
    return (k - 1) + (np.log(tol) - a) / (b - a)


def condition_estimate(alphas, betas):
    """(lambda_min, lambda_max, kappa) of M^{-1} A from the extreme Ritz values (Section 7)."""
    ritz = lanczos_ritz(alphas, betas)
    lo, hi = float(ritz.min()), float(ritz.max())
    return lo, hi, hi / lo


def cg_iteration_bound(kappa: float, tol: float) -> int:
    """Smallest k with 2 ((sqrt(kappa) - 1) / (sqrt(kappa) + 1))^k <= tol.

    The classical CG bound on the A-norm error reduction, used with the
    Lanczos condition estimate as the iteration bound the paper reports
    for solves stopped at the iteration cap (Section 7).
    """
    if kappa <= 1.0:
        return 0 if tol >= 2.0 else 1
    q = (np.sqrt(kappa) - 1.0) / (np.sqrt(kappa) + 1.0)
    return max(0, int(np.ceil(np.log(tol / 2.0) / np.log(q))))


# ---------------------------------------------------------------------------
# Three-level V-cycle (Section 6, three-level paragraph)


def subdomain_adjacency(A: sp.csr_matrix, part: np.ndarray, n_parts: int) -> sp.csr_matrix:
    """Boolean n_parts x n_parts matrix: subdomains i, j coupled by a stored entry of A."""
    n = A.shape[0]
    P = sp.csr_matrix((np.ones(n), (np.asarray(part), np.arange(n))), shape=(n_parts, n))
    pat = A.copy()
    pat.data = np.ones_like(pat.data)
    adj = (P @ pat @ P.T).tocsr()
    adj.data = np.ones_like(adj.data)
    return adj


class ThreeLevelOracle:
    """Three-level DDG preconditioner, FP64 (Section 6, three-level paragraph).

    The two-level method is applied again to the coarse matrix A0: the coarse
    unknowns (the kept columns of subdomain i) are grouped into coarse
    subdomains by ``part0`` (coarse subdomain of each fine subdomain), the
    coarsened generating vectors are F0 = R0 F, and the same overlap Delta is
    used in the graph of A0.  The graph of A0 is its block pattern: unknowns of
    subdomains i and j are coupled when A couples Omega_i and Omega_j.  One
    preconditioner application is a V-cycle: the fine pre-sweep, then
    R0^T M0^{-1} R0 (r - A e) with M0^{-1} one application of the two-level
    preconditioner of A0 (its own pre-sweep, the coarsest correction
    R1^T A1^{-1} R1, its post-sweep), then the fine post-sweep.
    """

    def __init__(self, A, F, part, n_parts: int, overlap: int, part0, n_parts0: int,
                 rank_tol: float = 1e-10):
        self.fine = DDGOracle(A, F, part, n_parts, overlap, rank_tol=rank_tol)
        fine = self.fine
        if not fine.coarse:
            raise OracleError("INVALID_ARG", "the three-level method needs generating vectors")
        F = np.asarray(F, dtype=np.float64)
        part0 = np.asarray(part0, dtype=np.int64)
        if part0.shape != (n_parts,) or part0.min() < 0 or part0.max() >= n_parts0:
            raise OracleError("INVALID_ARG", "coarse partition out of range")
        # graph of A0: blocks of coupled subdomain pairs
        adj = subdomain_adjacency(fine.A, fine.part, n_parts).tocoo()
        owner = np.repeat(np.arange(n_parts), fine.k_counts)          # subdomain of each coarse unknown
        first = fine.k_offsets[:-1]
        rows, cols = [], []
        for i, j in zip(adj.row, adj.col):
            ri = first[i] + np.arange(fine.k_counts[i])
            cj = first[j] + np.arange(fine.k_counts[j])
            rows.append(np.repeat(ri, cj.size))
            cols.append(np.tile(cj, ri.size))
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        A0s = sp.csr_matrix((fine.A0[rows, cols], (rows, cols)), shape=fine.A0.shape)
        A0s.sort_indices()
        self.A0 = A0s
        self.F0 = np.asarray(fine.R0 @ F)
        self.part_c = part0[owner]
        self.coarse = DDGOracle(A0s, self.F0, self.part_c, n_parts0, overlap, rank_tol=rank_tol)
        self.A = fine.A
        self.n = fine.n

    def apply(self, r: np.ndarray) -> np.ndarray:
        """M^{-1} r: fine pre-sweep, R0^T M0^{-1} R0 (r - A e), fine post-sweep."""
        f = self.fine
        r = np.asarray(r, dtype=np.float64)
        e = np.zeros(self.n)
        seq = [list(f.order[c]) for c in range(f.n_colours)]
        for ids in seq:
            f._colour(ids, r, e, False, None)
        b0 = f.R0 @ (r - self.A @ e)
        e += f.R0.T @ self.coarse.apply(b0)
        for ids in reversed(seq):
            f._colour(list(reversed(ids)), r, e, False, None)
        return e

    def pcg(self, f, rtol: float, max_iter: int = 1000, variant: str = "fr", trace: bool = False):
        return pcg(self.A, self.apply, f, rtol, max_iter, variant=variant, trace=trace)
