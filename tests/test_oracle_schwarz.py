"""Pins for the oracle's overlapping Schwarz preconditioner and PCG (Sections 6 and 7)."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import (DDGOracle, OracleError, cg_iteration_bound, condition_estimate, fractional_iterations,
                    lanczos_ritz, pcg)
from workloads import (CSR, box_partition, cell_coords, diffusion_cc, laplace5_nodes, monomials,
                       node_coords_2d, poisson2d_nodes, seed_rng)


def tiny2d(m=9, boxes=3, overlap=1, p=1):
    P = poisson2d_nodes(m, boxes, overlap, p, cfg_id=21)
    return P


def tiny3d(side=6, boxes=2, overlap=1, p=1, seed=22):
    kappa = np.exp(seed_rng(seed, 1).standard_normal((side,) * 3))
    A = diffusion_cc(kappa)
    part = box_partition((side,) * 3, (boxes,) * 3)
    F = monomials(cell_coords((side,) * 3), p)
    return A, F, part, boxes ** 3


def test_overlap_is_graph_ball():
    """Expanded subdomains = nodes within graph distance Delta (Section 6): an L1 ball for 5-point."""
    m, boxes = 15, 3
    for delta in (0, 1, 2):
        P = poisson2d_nodes(m, boxes, delta, 1)
        o = DDGOracle(P.A, P.F, P.part, P.n_parts, delta)
        jj, ii = np.divmod(np.arange(m * m), m)
        for b in range(P.n_parts):
            inside = P.part == b
            bi, bj = ii[inside], jj[inside]
            dx = np.maximum(0, np.maximum(bi.min() - ii, ii - bi.max()))
            dy = np.maximum(0, np.maximum(bj.min() - jj, jj - bj.max()))
            expect = np.flatnonzero(dx + dy <= delta)
            assert np.array_equal(o.sets[b], expect)


def test_colouring_is_parity_and_conflict_free():
    """Greedy colouring in increasing id gives parity colours on box grids; no same-colour conflicts."""
    A, F, part, nparts = tiny3d(side=12, boxes=4, p=0)
    o = DDGOracle(A, F, part, nparts, 1)
    b = np.arange(nparts)
    bx, by, bz = b % 4, (b // 4) % 4, b // 16
    assert np.array_equal(o.colours, (bx % 2) + 2 * (by % 2) + 4 * (bz % 2))
    As = A.to_scipy()
    for i in range(nparts):
        N = np.union1d(o.sets[i], np.unique(As[o.sets[i]].indices))
        for j in range(nparts):
            if j != i and o.colours[j] == o.colours[i]:
                assert np.intersect1d(N, o.sets[j]).size == 0
    P = poisson2d_nodes(63, 4, 2, 2)
    o2 = DDGOracle(P.A, P.F, P.part, P.n_parts, 2)
    assert o2.n_colours == 4


def test_each_local_step_zeroes_its_residual():
    """Exact local solves (Section 6): after updating subdomain i, (r - A e) vanishes on its set."""
    A, F, part, nparts = tiny3d(side=8)
    o = DDGOracle(A, F, part, nparts, 1)
    r = seed_rng(23, 0).standard_normal(A.n)
    trace = []
    o.apply(r, trace=trace)
    As = A.to_scipy()
    for kind, i, e in trace:
        if kind == "local":
            res = (r - As @ e)[o.sets[i]]
            assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(r)
        else:
            # Galerkin orthogonality after the coarse correction: R0 (r - A e) = 0
            assert np.linalg.norm(o.R0 @ (r - As @ e)) <= 1e-12 * np.linalg.norm(r)


def test_snapshot_equals_sequential():
    A, F, part, nparts = tiny3d(side=8)
    o = DDGOracle(A, F, part, nparts, 1)
    r = seed_rng(24, 0).standard_normal(A.n)
    a = o.apply(r)
    b = o.apply(r, snapshot=True)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def _error_propagation_form(o: DDGOracle):
    """M^{-1} = (I - E) A^{-1}, E = S* (I - P0) S, S = prod (I - P_i) in sweep order."""
    Ad = o.A.toarray()
    n = o.n
    I = np.eye(n)
    Ps = []
    for i in range(o.n_parts):
        s = o.sets[i]
        R = I[s]
        Ps.append(R.T @ np.linalg.solve(Ad[np.ix_(s, s)], R @ Ad))
    order = [i for c in range(o.n_colours) for i in o.order[c]]
    S = I.copy()
    for i in order:
        S = (I - Ps[i]) @ S
    Sstar = I.copy()
    for i in order:
        Sstar = Sstar @ (I - Ps[i])
    if o.coarse:
        R0 = o.R0.toarray()
        P0 = R0.T @ np.linalg.solve(R0 @ Ad @ R0.T, R0 @ Ad)
    else:
        P0 = np.zeros((n, n))
    E = Sstar @ (I - P0) @ S
    return (I - E) @ np.linalg.inv(Ad)


@pytest.mark.parametrize("dim", [2, 3])
def test_preconditioner_closed_form(dim):
    if dim == 2:
        P = tiny2d()
        o = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
    else:
        A, F, part, nparts = tiny3d()
        o = DDGOracle(A, F, part, nparts, 1)
    M = o.dense_operator()
    ref = _error_propagation_form(o)
    assert np.abs(M - ref).max() <= 1e-11 * np.abs(ref).max()
    # symmetric, and spectrum of M^{-1} A inside (0, 1]
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    ev = np.linalg.eigvals(M @ o.A.toarray()).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-10


def test_single_subdomain_is_direct_solve():
    P = tiny2d(m=8, boxes=1, overlap=0)
    o = DDGOracle(P.A, P.F, np.zeros(P.n, dtype=np.int32), 1, 0)
    Ad = P.A.to_scipy().toarray()
    r = seed_rng(25, 0).standard_normal(P.n)
    assert np.linalg.norm(o.apply(r) - np.linalg.solve(Ad, r)) <= 1e-13 * np.linalg.norm(r)
    x, it, info = o.pcg(P.f, 1e-12)
    assert it == 1


def test_singletons_no_coarse_is_symmetric_gauss_seidel():
    """One node per subdomain, Delta = 0, no coarse: SGS in colour-major order, M = (D+L) D^-1 (D+L)^T."""
    m = 6
    A = laplace5_nodes(m)
    n = m * m
    part = np.arange(n, dtype=np.int32)
    o = DDGOracle(A, None, part, n, 0, coarse=False)
    order = np.array([i for c in range(o.n_colours) for i in o.order[c]])
    Ad = A.to_scipy().toarray()
    Ap = Ad[np.ix_(order, order)]
    D = np.diag(np.diag(Ap))
    L = np.tril(Ap, -1)
    Msgs = (D + L) @ np.linalg.solve(D, (D + L).T)
    Pm = np.eye(n)[order]
    ref = Pm.T @ np.linalg.inv(Msgs) @ Pm
    got = o.dense_operator()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert o.n_colours == 2  # red-black for the 5-point graph


@pytest.mark.parametrize("dim", [2, 3])
def test_pcg_matches_dense_solve(dim):
    if dim == 2:
        P = poisson2d_nodes(7, 2, 1, 1, cfg_id=26)
        A, F, part, nparts, f = P.A, P.F, P.part, P.n_parts, P.f
    else:
        A, F, part, nparts = tiny3d()
        f = seed_rng(26, 0).uniform(-1, 1, A.n)
    o = DDGOracle(A, F, part, nparts, 1)
    x, it, info = o.pcg(f, 1e-14)
    ref = np.linalg.solve(A.to_scipy().toarray(), f)
    assert info["status"] == "ok"
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert info["true_rel_res"] <= 1e-13


def test_lanczos_ritz_values_in_unit_interval():
    """CG coefficients give Ritz values of M^{-1} A, whose spectrum lies in (0, 1]."""
    A, F, part, nparts = tiny3d(side=8)
    o = DDGOracle(A, F, part, nparts, 0)
    f = seed_rng(27, 0).standard_normal(A.n)
    x, it, info = o.pcg(f, 1e-10)
    ritz = lanczos_ritz(info["alpha"], info["beta"])
    assert ritz.min() > 0 and ritz.max() <= 1 + 1e-8


def test_lanczos_extremes_equal_preconditioned_spectrum():
    """The extreme Ritz values from the CG coefficients converge to the extreme
    eigenvalues of M^{-1} A (Section 7: condition estimates from the Lanczos
    coefficients).  Reference: eigenvalues of L^T M^{-1} L with A = L L^T, from the
    dense preconditioner."""
    A, F, part, nparts = tiny3d(side=8)
    o = DDGOracle(A, F, part, nparts, 0)
    f = seed_rng(28, 0).standard_normal(A.n)
    x, it, info = o.pcg(f, 1e-13)
    assert info["status"] == "ok" and it >= 10
    Minv = o.dense_operator()
    L = np.linalg.cholesky(A.to_scipy().toarray())
    ev = np.linalg.eigvalsh(0.5 * ((L.T @ Minv @ L) + (L.T @ Minv @ L).T))
    lo, hi, kappa = condition_estimate(info["alpha"], info["beta"])
    # the smallest eigenvalue is isolated and converges first
    assert abs(lo - ev.min()) <= 1e-8 * ev.min()
    # the top of the spectrum is a cluster at 1: Ritz values interlace, so the largest
    # lies just below the largest eigenvalue
    assert ev.max() - 1e-4 <= hi <= ev.max() + 1e-12
    ritz = lanczos_ritz(info["alpha"], info["beta"])
    assert ritz.size == it and ritz.min() >= ev.min() - 1e-12


def test_fractional_iterations_closed_forms():
    """Log-linear interpolation of the residual history (Section 7 protocol): on an
    exactly geometric history res_k = q^k it meets tol at log(tol)/log(q)."""
    for q in (0.5, 0.1, 0.37):
        res = q ** np.arange(30)
        for tol in (1e-3, 1e-8, 2.5e-6):
            assert abs(fractional_iterations(res, tol) - np.log(tol) / np.log(q)) <= 1e-9
    res = np.array([1.0, 1e-2, 1e-4, 1e-9])
    assert fractional_iterations(res, 1e-4) == 2.0
    assert abs(fractional_iterations(res, 1e-6) - (2 + 2.0 / 5.0)) <= 1e-12
    assert fractional_iterations(res, 1e-12) != fractional_iterations(res, 1e-12)  # nan: never reached
    assert fractional_iterations(res, 1.0) == 0.0


def test_cg_iteration_bound_closed_forms():
    """k = ceil(log(tol/2) / log((sqrt(kappa)-1)/(sqrt(kappa)+1))): kappa = 9 gives q = 1/2."""
    assert cg_iteration_bound(9.0, 2.0 ** -10) == 11
    assert cg_iteration_bound(9.0, 2.0 ** -10 * 1.0001) == 11
    assert cg_iteration_bound(9.0, 2.0 ** -9 * 0.9999) == 11
    assert cg_iteration_bound(1.0, 1e-8) == 1
    # monotone in kappa and tol
    ks = [cg_iteration_bound(k, 1e-8) for k in (2.0, 10.0, 100.0, 1e4)]
    assert ks == sorted(ks) and ks[-1] > ks[0]
    # for large kappa about sqrt(kappa)/2 ln(2/tol)
    k = cg_iteration_bound(1e6, 1e-9)
    assert abs(k - 0.5 * 1e3 * np.log(2e9)) <= 2


def test_polak_ribiere_keeps_directions_conjugate():
    """With Polak-Ribiere beta = z+^T (r+ - r) / r^T z, consecutive directions stay
    A-conjugate (p+^T A p = 0) even when the preconditioner changes from one
    iteration to the next; Fletcher-Reeves loses this.  With the fixed two-level
    preconditioner both give the same iterates (exact arithmetic)."""
    A, F, part, nparts = tiny3d(side=6)
    As = A.to_scipy()
    rng = seed_rng(29, 0)
    n = A.n
    diags = [np.exp(rng.standard_normal(n)) for _ in range(40)]
    calls = {"k": 0}

    def varying(r):
        d = diags[calls["k"] % len(diags)]
        calls["k"] += 1
        return d * r

    f = rng.standard_normal(n)
    worst = {}
    for variant in ("pr", "fr"):
        calls["k"] = 0
        _, it, info = pcg(As, varying, f, 1e-10, max_iter=30, variant=variant, trace=True)
        ps = info["p"]
        worst[variant] = max(abs(ps[j + 1] @ (As @ ps[j])) / (np.linalg.norm(ps[j + 1]) * np.linalg.norm(As @ ps[j]))
                             for j in range(len(ps) - 1))
    assert worst["pr"] <= 1e-12
    assert worst["fr"] >= 1e-4
    o = DDGOracle(A, F, part, nparts, 1)
    x_fr, it_fr, _ = o.pcg(f, 1e-10)
    x_pr, it_pr, _ = o.pcg(f, 1e-10, variant="pr")
    assert it_fr == it_pr
    assert np.linalg.norm(x_fr - x_pr) <= 1e-9 * np.linalg.norm(x_fr)


def test_pcg_conventions():
    P = tiny2d()
    o = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
    x, it, info = o.pcg(np.zeros(P.n), 1e-8)
    assert it == 0 and not x.any()
    x, it, info = o.pcg(P.f, 1e-30, max_iter=3)
    assert it == 3 and info["status"] == "no_convergence"
    with pytest.raises(OracleError):
        bad = P.f.copy(); bad[0] = np.nan
        o.pcg(bad, 1e-8)


def test_breakdown_on_indefinite_operator():
    """PCG with an indefinite operator hits p^T q <= 0 and reports breakdown."""
    n = 4
    A = sp.csr_matrix(np.diag([1.0, -1.0, 1.0, -1.0]))
    x, it, info = pcg(A, lambda r: r.copy(), np.array([1.0, 1.0, 0.0, 0.0]), 1e-10)
    assert info["status"] == "breakdown"


def test_validation_errors():
    m = 5
    A = laplace5_nodes(m)
    F = monomials(node_coords_2d(m), 1)
    part = np.zeros(m * m, dtype=np.int32)
    with pytest.raises(OracleError) as ei:
        DDGOracle(A, F, part, 2, 0)  # subdomain 1 empty
    assert ei.value.code == "INVALID_ARG"
    bad = CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.val.copy())
    bad.val[bad.row_ptr[3]] = 0.5  # break symmetry
    with pytest.raises(OracleError):
        DDGOracle(bad, F, part, 1, 0)
    neg = CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), -A.val)
    with pytest.raises(OracleError) as ei:
        DDGOracle(neg, F, part, 1, 0)
    assert ei.value.code == "NOT_SPD"


def test_cfg1_reference_run():
    """cfg1: 63x63 Poisson, 4x4 boxes, overlap 2, p = 2 -> N_c = 96, 4 colours, converges."""
    from workloads import cfg1
    P = cfg1()
    o = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
    assert o.n_coarse == 96 and o.n_colours == 4
    assert sum(len(s) for s in o.sets) == 5517
    x, it, info = o.pcg(P.f, P.rtol)
    assert info["status"] == "ok" and info["true_rel_res"] <= 1e-9
    assert 3 <= it <= 30
