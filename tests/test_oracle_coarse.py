"""Pins for the oracle's coarse grid (Section 4): basis, Galerkin operator, coarse solve.

Every check here compares the oracle against something other than itself:
exact rational arithmetic, closed forms, invariants the paper states, or a
hand-derived fixture.
"""

import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import DDGOracle, OracleError
from oracle.ddg import coarse_basis, galerkin
from workloads import (box_partition, cell_coords, diffusion_cc, laplace5_nodes, monomials,
                       node_coords_2d, poisson2d_nodes, seed_rng)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_2d(m=17, boxes=3, overlap=1, p=2):
    return poisson2d_nodes(m, boxes, overlap, p, cfg_id=7)


def small_3d(side=8, boxes=2, overlap=1, p=2, seed=3):
    rng = seed_rng(seed, 1)
    kappa = np.exp(rng.standard_normal((side,) * 3))
    A = diffusion_cc(kappa)
    part = box_partition((side,) * 3, (boxes,) * 3)
    F = monomials(cell_coords((side,) * 3), p)
    return A, F, part, boxes ** 3


def test_r0_orthonormal_and_spans_generating_vectors():
    P = small_2d()
    R0, counts, offs, _, _ = coarse_basis(P.F, P.part, P.n_parts, 1e-10)
    G = (R0 @ R0.T).toarray()
    assert np.abs(G - np.eye(G.shape[0])).max() <= 1e-13
    # every generating vector lies in range(R0^T): R0^T R0 F_j = F_j
    for j in range(P.F.shape[1]):
        Fj = P.F[:, j]
        back = R0.T @ (R0 @ Fj)
        assert np.linalg.norm(back - Fj) <= 1e-12 * np.linalg.norm(Fj)
    # subdomain-major layout (Fig. 2): coarse row offset_i + j is supported on Omega_i only
    R0c = R0.tocsr()
    for i in range(P.n_parts):
        for j in range(int(counts[i])):
            cols = R0c.indices[R0c.indptr[offs[i] + j]:R0c.indptr[offs[i] + j + 1]]
            assert np.all(P.part[cols] == i)


def test_projector_matches_hand_fixture():
    rows = []
    with open(os.path.join(GOLDEN, "r0_projector_1d.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(Fraction(t)) for t in line.split()])
    expected = np.array(rows)
    x = np.arange(6.0)
    F = np.stack([np.ones(6), x], axis=1)
    part = np.array([0, 0, 0, 1, 1, 1])
    R0, counts, _, _, _ = coarse_basis(F, part, 2, 1e-10)
    assert list(counts) == [2, 2]
    assert np.abs((R0.T @ R0).toarray() - expected).max() <= 1e-14


def test_coarse_solution_exact_rational_1d():
    """Coarse approximation R0^T u0 with A0 u0 = R0 f (Section 4), checked in exact arithmetic.

    The operator R0^T (R0 A R0^T)^{-1} R0 does not depend on which basis of
    the DDG space is used, so it equals Z (Z^T A Z)^{-1} Z^T for the raw
    restricted basis Z = [R_i^T R_i F], which is computed here with fractions.
    """
    n = 6
    A = np.diag([2.0] * n) + np.diag([-1.0] * (n - 1), 1) + np.diag([-1.0] * (n - 1), -1)
    x = np.arange(float(n))
    F = np.stack([np.ones(n), x], axis=1)
    part = np.array([0, 0, 0, 1, 1, 1])
    o = DDGOracle(sp.csr_matrix(A), F, part, 2, 0)
    f = np.array([3.0, -1.0, 2.0, 0.5, 4.0, -2.0])
    got = o.coarse_apply(f)
    # exact: Z (Z^T A Z)^{-1} Z^T f
    Z = [[Fraction(0)] * 4 for _ in range(n)]
    for v in range(n):
        b = 2 * int(part[v])
        Z[v][b] = Fraction(1)
        Z[v][b + 1] = Fraction(int(x[v]))
    Af = [[Fraction(int(A[i, j])) for j in range(n)] for i in range(n)]
    ff = [Fraction(f[i]).limit_denominator(1000) for i in range(n)]
    ZtA = [[sum(Z[v][a] * Af[v][w] for v in range(n)) for w in range(n)] for a in range(4)]
    M = [[sum(ZtA[a][w] * Z[w][b] for w in range(n)) for b in range(4)] for a in range(4)]
    rhs = [sum(Z[v][a] * ff[v] for v in range(n)) for a in range(4)]
    # Gauss elimination in fractions
    aug = [M[a][:] + [rhs[a]] for a in range(4)]
    for c in range(4):
        piv = next(r for r in range(c, 4) if aug[r][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        for r in range(4):
            if r != c and aug[r][c] != 0:
                fac = aug[r][c] / aug[c][c]
                aug[r] = [aug[r][t] - fac * aug[c][t] for t in range(5)]
    y = [aug[a][4] / aug[a][a] for a in range(4)]
    exact = np.array([float(sum(Z[v][a] * y[a] for a in range(4))) for v in range(n)])
    assert np.abs(got - exact).max() <= 1e-14 * np.abs(exact).max()


def test_a0_spd_symmetric_and_block_pattern():
    A, F, part, nparts = small_3d()
    o = DDGOracle(A, F, part, nparts, 1)
    A0 = o.A0
    assert np.abs(A0 - A0.T).max() <= 1e-13 * np.abs(A0).max()
    assert np.linalg.eigvalsh(A0).min() > 0
    # block sparsity = subdomain adjacency (Section 4)
    As = A.to_scipy().tocoo()
    adj = np.zeros((nparts, nparts), dtype=bool)
    adj[part[As.row], part[As.col]] = True
    offs = o.k_offsets
    for i in range(nparts):
        for j in range(nparts):
            blk = A0[offs[i]:offs[i + 1], offs[j]:offs[j + 1]]
            if adj[i, j]:
                assert np.abs(blk).max() > 0
            else:
                assert np.abs(blk).max() == 0.0


def test_coarse_operator_basis_invariant():
    """A change of basis of F leaves the coarse space and its projector unchanged."""
    A, F, part, nparts = small_3d()
    M = seed_rng(11, 0).standard_normal((F.shape[1], F.shape[1])) + 3 * np.eye(F.shape[1])
    o1 = DDGOracle(A, F, part, nparts, 1)
    o2 = DDGOracle(A, np.asfortranarray(F @ M), part, nparts, 1)
    assert np.allclose(np.sort(np.linalg.eigvalsh(o1.A0)), np.sort(np.linalg.eigvalsh(o2.A0)),
                       rtol=1e-10, atol=0)
    v = seed_rng(11, 1).standard_normal(A.n)
    a, b = o1.coarse_apply(v), o2.coarse_apply(v)
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)


@pytest.mark.parametrize("piecewise", [False, True])
def test_coarse_solve_reproduces_polynomials(piecewise):
    """Manufactured solution: u* in span(R0^T) is reproduced exactly by the Galerkin solve.

    R0^T A0^{-1} R0 A is the A-orthogonal projector onto the DDG space
    (Section 5.1), so any per-subdomain polynomial of degree <= p is fixed.
    """
    A, F, part, nparts = small_3d()
    o = DDGOracle(A, F, part, nparts, 1)
    rng = seed_rng(12, int(piecewise))
    if piecewise:
        u = np.zeros(A.n)
        for i in range(nparts):
            m = part == i
            u[m] = F[m] @ rng.standard_normal(F.shape[1])
    else:
        u = F @ rng.standard_normal(F.shape[1])
    f = A.to_scipy() @ u
    got = o.coarse_apply(f)
    assert np.linalg.norm(got - u) <= 1e-10 * np.linalg.norm(u)


def test_coarse_error_non_increasing_in_p():
    """Nested spaces + Galerkin optimality: the A-norm coarse error never grows with p (Section 5)."""
    side = 10
    rng = seed_rng(13, 1)
    kappa = np.exp(rng.standard_normal((side, side)))
    A = diffusion_cc(kappa)
    As = A.to_scipy()
    part = box_partition((side, side), (3, 3))
    f = seed_rng(13, 0).standard_normal(A.n)
    u = np.linalg.solve(As.toarray(), f)
    errs = []
    for p in range(4):
        F = monomials(cell_coords((side, side)), p)
        o = DDGOracle(A, F, part, 9, 0)
        d = o.coarse_apply(f) - u
        errs.append(float(np.sqrt(d @ (As @ d))))
    for a, b in zip(errs, errs[1:]):
        assert b <= a * (1 + 1e-12)
    assert errs[-1] < 0.5 * errs[0]


def test_constant_vector_reduces_to_aggregation():
    """F = constant vector gives non-smoothed aggregation (Section 2): Z (Z^T A Z)^{-1} Z^T."""
    A, _, part, nparts = small_3d(p=0)
    As = A.to_scipy().toarray()
    F = np.ones((A.n, 1))
    o = DDGOracle(A, F, part, nparts, 1)
    Z = np.zeros((A.n, nparts))
    Z[np.arange(A.n), part] = 1.0
    P = Z @ np.linalg.solve(Z.T @ As @ Z, Z.T)
    v = seed_rng(14, 0).standard_normal(A.n)
    assert np.linalg.norm(o.coarse_apply(v) - P @ v) <= 1e-13 * np.linalg.norm(P @ v)
    assert list(o.k_counts) == [1] * nparts


def test_rank_deficient_blocks_are_trimmed():
    """Section 4: columns are discarded when the restricted vectors are dependent.

    On a strip one node wide in x, the degree-2 monomials in (x, y) span only
    {1, y, y^2}: rank 3 of 6.  A strip two nodes wide has rank 5
    ({1, x, y, xy, y^2}; x^2 is affine in x on two points).
    """
    m = 12
    A = laplace5_nodes(m)
    F = monomials(node_coords_2d(m), 2)
    xs = np.arange(m * m) % m
    part = np.where(xs == 0, 0, np.where(xs < 3, 1, 2)).astype(np.int32)
    R0, counts, _, _, _ = coarse_basis(F, part, 3, 1e-10)
    assert list(counts) == [3, 5, 6]
    G = (R0 @ R0.T).toarray()
    assert np.abs(G - np.eye(G.shape[0])).max() <= 1e-12
    for j in range(F.shape[1]):
        assert np.linalg.norm(R0.T @ (R0 @ F[:, j]) - F[:, j]) <= 1e-10 * np.linalg.norm(F[:, j])


def test_zero_block_is_rank_error():
    m = 6
    A = laplace5_nodes(m)
    F = monomials(node_coords_2d(m), 1)
    F[:6, :] = 0.0
    part = np.zeros(m * m, dtype=np.int32)
    part[:6] = 1
    with pytest.raises(OracleError) as ei:
        coarse_basis(F, part, 2, 1e-10)
    assert ei.value.code == "RANK" and ei.value.where == 1


def test_galerkin_is_r0_a_r0t():
    """A0 entries equal q_a^T A q_b for the orthonormal basis vectors (definition, Section 4)."""
    A, F, part, nparts = small_3d(side=6, p=1)
    R0, _, _, _, _ = coarse_basis(F, part, nparts, 1e-10)
    A0 = galerkin(A.to_scipy(), R0)
    Rd = R0.toarray()
    Ad = A.to_scipy().toarray()
    rng = seed_rng(15, 0)
    for _ in range(20):
        a, b = rng.integers(0, Rd.shape[0], size=2)
        assert abs(A0[a, b] - Rd[a] @ Ad @ Rd[b]) <= 1e-13 * np.abs(A0).max()
