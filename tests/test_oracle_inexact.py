"""Pins of the inexact-solve oracle (Section 7's timed 3D variant; CPU only).

* SSOR local smoothing equals its dense closed form: one symmetric sweep from
  zero is x = omega (2 - omega) (D + omega U)^{-1} D (D + omega L)^{-1} b in the
  colour-sorted order, and s sweeps are s steps of x += B (b - A x);
* the greedy local colouring is a proper colouring (red-black on box sets of
  a 7-point stencil);
* the preconditioner stays symmetric with its spectrum of M^{-1} A in (0, 1];
* IC(0) reproduces A on its pattern, and is the exact Cholesky factor when
  the pattern admits no fill (a tridiagonal matrix);
* the IC-preconditioned CG coarse solve reaches A0^{-1} b at a tight tolerance.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import DDGOracle
from oracle.ddg import subdomain_adjacency
from oracle.inexact import InexactDDGOracle, SSORLocal, ic0, ic_pcg, local_colouring
from workloads import box_partition, cell_coords, diffusion_cc, monomials, seed_rng


def tiny3d(L=8, boxes=2, overlap=1, p=1, seed=61):
    kappa = np.exp(seed_rng(seed, 1).standard_normal((L, L, L)))
    A = diffusion_cc(kappa).to_scipy()
    return A, monomials(cell_coords((L, L, L)), p), box_partition((L, L, L), (boxes,) * 3), boxes ** 3, overlap


def ssor_closed_form(Ai, omega):
    S = SSORLocal(Ai, omega, 1)
    perm = np.concatenate(S.groups)
    Ap = Ai.toarray()[np.ix_(perm, perm)]
    D = np.diag(np.diag(Ap))
    Lw = np.tril(Ap, -1)
    Uw = np.triu(Ap, 1)
    Bp = omega * (2 - omega) * np.linalg.solve(D + omega * Uw, D @ np.linalg.inv(D + omega * Lw))
    B = np.zeros_like(Bp)
    B[np.ix_(perm, perm)] = Bp
    return B


@pytest.mark.parametrize("omega", [1.0, 1.4])
def test_ssor_matches_closed_form(omega):
    A, F, part, n_parts, overlap = tiny3d()
    o = DDGOracle(A, F, part, n_parts, overlap)
    s = o.sets[3]
    Ai = sp.csr_matrix(A[s][:, s])
    B = ssor_closed_form(Ai, omega)
    b = seed_rng(62, 0).standard_normal(len(s))
    assert np.allclose(SSORLocal(Ai, omega, 1).solve(b), B @ b, rtol=1e-12, atol=1e-12 * np.abs(B @ b).max())
    x = np.zeros_like(b)
    Ad = Ai.toarray()
    for _ in range(3):
        x = x + B @ (b - Ad @ x)
    assert np.allclose(SSORLocal(Ai, omega, 3).solve(b), x, rtol=1e-11, atol=1e-11 * np.abs(x).max())
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()


def test_local_colouring_is_proper_and_red_black_on_boxes():
    A, F, part, n_parts, overlap = tiny3d(L=8, boxes=2, overlap=0)
    o = DDGOracle(A, F, part, n_parts, overlap)
    Ai = sp.csr_matrix(A[o.sets[0]][:, o.sets[0]]).tocoo()
    col = local_colouring(sp.csr_matrix(A[o.sets[0]][:, o.sets[0]]))
    off = Ai.row != Ai.col
    assert np.all(col[Ai.row[off]] != col[Ai.col[off]])
    assert col.max() == 1


@pytest.mark.parametrize("omega,sweeps", [(1.0, 1), (1.5, 2)])
def test_inexact_preconditioner_symmetric_with_spectrum_in_unit_interval(omega, sweeps):
    A, F, part, n_parts, overlap = tiny3d()
    o = InexactDDGOracle(A, F, part, n_parts, overlap, omega=omega, sweeps=sweeps)
    M = o.dense_operator()
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    lam = np.linalg.eigvals(M @ A.toarray()).real
    assert lam.min() > 0 and lam.max() <= 1 + 1e-10


def test_ic0_properties_and_coarse_cg():
    n = 40
    T = sp.diags([-np.ones(n - 1), 2.5 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    L = ic0(T).toarray()
    assert np.allclose(L @ L.T, T.toarray(), rtol=0, atol=1e-14)
    A, F, part, n_parts, overlap = tiny3d(L=10, boxes=2, p=2)
    o = InexactDDGOracle(A, F, part, n_parts, overlap, coarse_solver="ic_cg", ic_tol=1e-13, ic_maxit=500)
    L0 = o.L0.toarray()
    # the pattern is the block pattern of coupled subdomains (structural)
    adj = subdomain_adjacency(A, part, n_parts).toarray() > 0
    owner = np.repeat(np.arange(n_parts), o.k_counts)
    pat = adj[owner][:, owner]
    assert np.array_equal(pat, o.block_mask) and not pat.all()
    # zero fill: L has entries only in the lower triangle of that pattern, and L L^T
    # reproduces A0 on it
    assert np.all((L0 != 0) <= np.tril(pat))
    LLt = L0 @ L0.T
    assert np.allclose(LLt[pat], o.A0[pat], rtol=0, atol=1e-12 * np.abs(o.A0).max())
    b = seed_rng(63, 0).standard_normal(o.A0.shape[0])
    y = ic_pcg(o.A0s, o.L0, b, 1e-13, 500)
    assert np.linalg.norm(y - np.linalg.solve(o.A0, b)) <= 1e-11 * np.linalg.norm(y)


def test_inexact_pcg_converges_with_more_iterations():
    A, F, part, n_parts, overlap = tiny3d(L=12, boxes=3, p=2)
    f = seed_rng(64, 0).uniform(-1, 1, A.shape[0])
    _, it_exact, _ = DDGOracle(A, F, part, n_parts, overlap).pcg(f, 1e-10)
    x, it, info = InexactDDGOracle(A, F, part, n_parts, overlap).pcg(f, 1e-10)
    assert info["status"] == "ok" and it >= it_exact
    x2, it2, info2 = InexactDDGOracle(A, F, part, n_parts, overlap, coarse_solver="ic_cg",
                                      ic_tol=1e-4).pcg(f, 1e-10, variant="pr")
    assert info2["status"] == "ok"
    assert np.linalg.norm(x2 - x) <= 1e-8 * np.linalg.norm(x)


def test_ic0_on_a_full_block_pattern_is_the_cholesky_factor():
    """Two coupled subdomains: the block pattern of A0 is the whole matrix, so the
    zero-fill incomplete factor is the complete Cholesky factor (numpy's)."""
    L = 6
    kappa = np.exp(seed_rng(65, 1).standard_normal((L, L, L)))
    A = diffusion_cc(kappa).to_scipy()
    part = box_partition((L, L, L), (2, 1, 1))
    o = InexactDDGOracle(A, monomials(cell_coords((L, L, L)), 2), part, 2, 1, coarse_solver="ic_cg")
    assert o.block_mask.all()
    C = np.linalg.cholesky(o.A0)
    assert np.allclose(o.L0.toarray(), C, rtol=0, atol=1e-13 * np.abs(C).max())
