"""Pins of the three-level oracle (Section 6, three-level paragraph; CPU only).

The three-level V-cycle applies the two-level method again to A0 with the
coarsened generating vectors F0 = R0 F.  What the paper and the mathematics fix:

* F0 lies in the range of the coarsest basis R1^T (the coarsest space is built
  from it, restricted to coarse subdomains), and R0^T F0 = F because every
  generating vector lies in range(R0^T);
* A1 = R1 A0 R1^T is SPD;
* M^{-1} is symmetric and equals its dense error-propagation form
  (I - E) A^{-1}, E = S* (I - R0^T M0^{-1} R0 A) S with S the fine sweep's
  product of (I - P_i), and M0^{-1} = (I - E0) A0^{-1} built the same way
  on the coarse level: an independent code path;
* the spectrum of M^{-1} A lies in (0, 1];
* with one coarse subdomain and no further structure the coarse smoother
  solves A0 exactly, so the three-level preconditioner equals the two-level one;
* PCG with it reaches the dense solution on tiny grids.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import DDGOracle, ThreeLevelOracle
from workloads import box_groups, box_partition, cell_coords, diffusion_cc, monomials, seed_rng


def tiny2d(L=16, boxes=4, overlap=1, p=1, group=2, seed=51):
    kappa = np.exp(seed_rng(seed, 1).standard_normal((L, L)))
    A = diffusion_cc(kappa).to_scipy()
    part = box_partition((L, L), (boxes, boxes))
    F = monomials(cell_coords((L, L)), p)
    part0, n0 = box_groups((boxes, boxes), (group, group))
    return A, F, part, boxes * boxes, overlap, part0, n0


def tiny3d(L=8, boxes=4, overlap=1, p=1, group=2, seed=52):
    kappa = np.exp(seed_rng(seed, 1).standard_normal((L, L, L)))
    A = diffusion_cc(kappa).to_scipy()
    part = box_partition((L, L, L), (boxes,) * 3)
    F = monomials(cell_coords((L, L, L)), p)
    part0, n0 = box_groups((boxes,) * 3, (group,) * 3)
    return A, F, part, boxes ** 3, overlap, part0, n0


def sweep_product(o: DDGOracle) -> np.ndarray:
    """S = product of (I - P_i) over the pre-sweep order, P_i = R~_i^T A_i^{-1} R~_i A (dense)."""
    A = o.A.toarray()
    n = A.shape[0]
    S = np.eye(n)
    for c in range(o.n_colours):
        for i in o.order[c]:
            s = o.sets[i]
            Ai = A[np.ix_(s, s)]
            P = np.zeros((n, n))
            P[s, :] = np.linalg.solve(Ai, A[s, :])
            S = (np.eye(n) - P) @ S
    return S


def dense_two_level_inverse(o: DDGOracle) -> np.ndarray:
    A = o.A.toarray()
    n = A.shape[0]
    S = sweep_product(o)
    R0 = o.R0.toarray()
    A0 = R0 @ A @ R0.T
    P0 = R0.T @ np.linalg.solve(A0, R0 @ A)
    # post-sweep in reverse order = adjoint of S in the A inner product
    Sstar = np.linalg.solve(A, S.T @ A)
    E = Sstar @ (np.eye(n) - P0) @ S
    return (np.eye(n) - E) @ np.linalg.inv(A)


@pytest.mark.parametrize("make", [tiny2d, tiny3d], ids=["2d", "3d"])
def test_coarsened_vectors_and_coarsest_operator(make):
    A, F, part, n_parts, overlap, part0, n0 = make()
    t = ThreeLevelOracle(A, F, part, n_parts, overlap, part0, n0)
    F0 = t.F0
    R1 = t.coarse.R0.toarray()
    assert np.linalg.norm(R1.T @ (R1 @ F0) - F0) <= 1e-12 * np.linalg.norm(F0)
    R0 = t.fine.R0.toarray()
    assert np.linalg.norm(R0.T @ F0 - F) <= 1e-12 * np.linalg.norm(F)
    A1 = t.coarse.A0
    assert np.allclose(A1, A1.T, rtol=0, atol=1e-13 * np.abs(A1).max())
    assert np.linalg.eigvalsh(A1).min() > 0
    # coarse partition: coarse unknown (i, j) belongs to coarse subdomain part0[i]
    owner = np.repeat(np.arange(n_parts), t.fine.k_counts)
    assert np.array_equal(t.part_c, part0[owner])


@pytest.mark.parametrize("make", [tiny2d, tiny3d], ids=["2d", "3d"])
def test_three_level_closed_form_and_spectrum(make):
    A, F, part, n_parts, overlap, part0, n0 = make()
    t = ThreeLevelOracle(A, F, part, n_parts, overlap, part0, n0)
    n = A.shape[0]
    I = np.eye(n)
    M = np.stack([t.apply(I[:, j]) for j in range(n)], axis=1)
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    # closed form: the coarse solve of the two-level form replaced by M0^{-1}
    Ad = A.toarray()
    M0 = dense_two_level_inverse(t.coarse)
    S = sweep_product(t.fine)
    Sstar = np.linalg.solve(Ad, S.T @ Ad)
    R0 = t.fine.R0.toarray()
    E = Sstar @ (I - R0.T @ M0 @ R0 @ Ad) @ S
    Mc = (I - E) @ np.linalg.inv(Ad)
    assert np.abs(M - Mc).max() <= 1e-10 * np.abs(Mc).max()
    lam = np.linalg.eigvals(M @ Ad).real
    assert lam.min() > 0.0 and lam.max() <= 1.0 + 1e-10


def test_single_coarse_subdomain_reduces_to_two_level():
    A, F, part, n_parts, overlap, part0, n0 = tiny2d()
    t = ThreeLevelOracle(A, F, part, n_parts, overlap, np.zeros(n_parts, dtype=np.int64), 1)
    two = DDGOracle(A, F, part, n_parts, overlap)
    r = seed_rng(53, 0).standard_normal(A.shape[0])
    z3, z2 = t.apply(r), two.apply(r)
    assert np.linalg.norm(z3 - z2) <= 1e-12 * np.linalg.norm(z2)


def test_three_level_pcg_reaches_dense_solution():
    A, F, part, n_parts, overlap, part0, n0 = tiny3d(L=10, boxes=5, p=2, group=2)
    t = ThreeLevelOracle(A, F, part, n_parts, overlap, part0, n0)
    f = seed_rng(54, 0).uniform(-1, 1, A.shape[0])
    x, it, info = t.pcg(f, 1e-13)
    xd = np.linalg.solve(A.toarray(), f)
    assert info["status"] == "ok"
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)
    # a V-cycle needs at least as many iterations as the exact coarse solve
    _, it2, _ = DDGOracle(A, F, part, n_parts, overlap).pcg(f, 1e-13)
    assert it >= it2
