"""Material-aware generating vectors (Section 7 problem C) in the oracle (CPU).

With F_aware = [F J, F (1 - J)] every subdomain keeps the columns of both
materials it meets: the kept count equals rank(F on its J cells) + rank(F on
its other cells), so subdomains inside one material keep k columns and those
that straddle the boundary keep up to 2k (Section 7, problem C).  The aware
coarse space contains the plain one (F = F J + F (1 - J)), so its Galerkin
projection error in the energy norm is no larger (nested spaces), and with a
cubic basis CG needs fewer iterations (context: the paper reports close to
half; parity of the count itself is unpinned).
"""

import numpy as np

from oracle import DDGOracle
from workloads.materials import material_problem


def _rank(B):
    if B.shape[0] == 0:
        return 0
    s = np.linalg.svd(B, compute_uv=False)
    return int(np.count_nonzero(s > 1e-10 * s[0])) if s.size and s[0] > 0 else 0


def test_kept_columns_follow_the_materials():
    P = material_problem(64, 4, 1, 2, aware=True)
    Pp = material_problem(64, 4, 1, 2, aware=False)
    J = P.meta["J"].ravel() > 0.5
    o = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
    k = Pp.F.shape[1]
    straddle = 0
    for i in range(P.n_parts):
        idx = np.flatnonzero(P.part == i)
        want = _rank(Pp.F[idx][J[idx]]) + _rank(Pp.F[idx][~J[idx]])
        assert o.k_counts[i] == want
        straddle += int(J[idx].any() and (~J[idx]).any())
        if not (J[idx].any() and (~J[idx]).any()):
            assert o.k_counts[i] == k
    assert 0 < straddle < P.n_parts


def test_aware_space_contains_plain_space():
    P = material_problem(48, 4, 1, 3, aware=True)
    Pp = material_problem(48, 4, 1, 3, aware=False)
    oa = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
    op = DDGOracle(Pp.A, Pp.F, Pp.part, Pp.n_parts, Pp.overlap)
    Ra, Rp = oa.R0.toarray(), op.R0.toarray()
    # every plain coarse basis vector lies in the aware coarse space
    assert np.linalg.norm(Ra.T @ (Ra @ Rp.T) - Rp.T) <= 1e-10 * np.linalg.norm(Rp)
    A = P.A.to_scipy()
    u = np.random.default_rng(5).standard_normal(P.n)
    f = A @ u

    def energy_err(o):
        e = u - o.coarse_apply(f)
        return float(e @ (A @ e))

    assert energy_err(oa) <= energy_err(op) * (1 + 1e-12)


def test_aware_cubic_basis_needs_fewer_iterations():
    P = material_problem(96, 6, 1, 3, aware=True)
    Pp = material_problem(96, 6, 1, 3, aware=False)
    _, it_a, _ = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap).pcg(P.f, 1e-9)
    _, it_p, _ = DDGOracle(Pp.A, Pp.F, Pp.part, Pp.n_parts, Pp.overlap).pcg(Pp.f, 1e-9)
    assert it_a < it_p
