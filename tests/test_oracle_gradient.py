"""Pins for the oracle's coefficient gradient (adjoint method on the cell-centred operator)."""

import numpy as np
import scipy.sparse.linalg as spla

from oracle import DDGOracle, assemble_cc, coeff_grad_cc
from workloads import box_partition, cell_coords, diffusion_cc, grf, monomials, seed_rng


def test_oracle_assembly_matches_generator():
    """Two independent assemblies of the harmonic-mean operator agree."""
    for shape in ((5, 7), (4, 5, 6)):
        kappa = np.exp(seed_rng(31, 1).standard_normal(shape))
        for bc in ("dirichlet", "x0"):
            a = assemble_cc(kappa, bc=bc)
            b = diffusion_cc(kappa, bc=bc).to_scipy()
            assert abs(a - b).max() <= 1e-14 * abs(b).max()


def test_coeff_grad_matches_assembly_difference():
    """g_c = -lam^T (dA/dtheta_c) u against a central difference of the assembly only."""
    shape = (4, 5, 6)
    rng = seed_rng(32, 1)
    theta = rng.standard_normal(shape)
    u = rng.standard_normal(theta.size)
    lam = rng.standard_normal(theta.size)
    g = coeff_grad_cc(np.exp(theta), u, lam)
    h = 1e-5
    for c in rng.choice(theta.size, size=25, replace=False):
        tp = theta.copy().ravel(); tp[c] += h
        tm = theta.copy().ravel(); tm[c] -= h
        dA = (assemble_cc(np.exp(tp.reshape(shape))) - assemble_cc(np.exp(tm.reshape(shape)))) / (2 * h)
        fd = -lam @ (dA @ u)
        assert abs(g.ravel()[c] - fd) <= 1e-8 * max(1.0, abs(fd))


def test_adjoint_gradient_vs_central_difference():
    """dL/dtheta for L = ||u(theta) - u_obs||^2 with u from DDG-PCG, vs FD of exact solves."""
    shape = (8, 8, 8)
    theta = grf(shape, 3.0, 1.0, seed_rng(33, 1))
    theta_obs = grf(shape, 3.0, 1.0, seed_rng(33, 2))
    f = seed_rng(33, 0).uniform(-1, 1, theta.size)
    part = box_partition(shape, (2, 2, 2))
    F = monomials(cell_coords(shape), 1)

    def solve(th, rhs, tol=1e-13):
        A = assemble_cc(np.exp(th))
        o = DDGOracle(A, F, part, 8, 1)
        x, it, info = o.pcg(rhs, tol)
        return x, A

    u_obs, _ = solve(theta_obs, f)
    u, A = solve(theta, f)
    lam, _ = solve(theta, 2 * (u - u_obs))
    # adjoint identity for the symmetric solve: lam^T f = (dL/du)^T u
    assert abs(lam @ f - 2 * (u - u_obs) @ u) <= 1e-10 * abs(lam @ f)
    g = coeff_grad_cc(np.exp(theta), u, lam).ravel()
    h = 1e-4
    rng = seed_rng(33, 4)
    for c in rng.choice(theta.size, size=8, replace=False):
        vals = []
        for s in (+1, -1):
            t = theta.copy().ravel(); t[c] += s * h
            Ap = assemble_cc(np.exp(t.reshape(shape))).tocsc()
            up = spla.spsolve(Ap, f)
            vals.append(float(np.sum((up - u_obs) ** 2)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[c] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_x0_boundary_closed_form():
    """Problem A boundary conditions (Section 7): with Dirichlet only on x = 0 the
    constant vector is annihilated everywhere except in the x = 0 cells, where
    A 1 = 2 kappa_c (the ghost face); with Dirichlet on every face each boundary
    face adds 2 kappa_c."""
    for shape in ((6, 7), (3, 4, 5)):
        kappa = np.exp(seed_rng(34, 1).standard_normal(shape))
        one = np.ones(kappa.size)
        r = (assemble_cc(kappa, bc="x0") @ one).reshape(shape)
        expect = np.zeros(shape)
        expect[..., 0] = 2.0 * kappa[..., 0]
        assert np.abs(r - expect).max() <= 1e-13 * kappa.max()
        r = (assemble_cc(kappa) @ one).reshape(shape)
        faces = np.zeros(shape)
        for ax in range(len(shape)):
            m = np.moveaxis(faces, ax, 0)
            m[0] += 1.0
            m[-1] += 1.0
        assert np.abs(r - 2.0 * kappa * faces).max() <= 1e-13 * kappa.max()
        # still SPD: one Dirichlet face makes the Neumann operator non-singular
        ev = np.linalg.eigvalsh(assemble_cc(kappa, bc="x0").toarray())
        assert ev.min() > 0


def test_coeff_grad_x0_matches_assembly_difference():
    """The gradient formula with the x = 0 boundary, against a central difference of the assembly."""
    shape = (4, 5, 6)
    rng = seed_rng(35, 1)
    theta = rng.standard_normal(shape)
    u = rng.standard_normal(theta.size)
    lam = rng.standard_normal(theta.size)
    g = coeff_grad_cc(np.exp(theta), u, lam, bc="x0")
    h = 1e-5
    for c in rng.choice(theta.size, size=25, replace=False):
        tp = theta.copy().ravel(); tp[c] += h
        tm = theta.copy().ravel(); tm[c] -= h
        dA = (assemble_cc(np.exp(tp.reshape(shape)), bc="x0") - assemble_cc(np.exp(tm.reshape(shape)), bc="x0")) / (2 * h)
        fd = -lam @ (dA @ u)
        assert abs(g.ravel()[c] - fd) <= 1e-8 * max(1.0, abs(fd))
