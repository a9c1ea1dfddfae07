"""Differentiation through the DDG solve on the GPU, against the FP64 oracle.

Loss L(theta) = ||u(theta) - u_obs||^2 with A(exp(theta)) u = f on the
cell-centred diffusion operator.  Checks, in this order:
  * device assembly of A(exp(theta)) against the oracle's own assembly
    (entry-wise, 1e-14 relative: only the exponential's rounding differs);
  * the coefficient-gradient kernel against the oracle formula on the same
    u and lambda (1e-12 relative in norm);
  * the autograd gradient (forward solve + adjoint solve with the same
    handle + kernel) against the oracle gradient (oracle PCG for u, u_obs and
    lambda, oracle formula): 1e-8 relative in norm with both solves at 1e-12;
  * central finite differences of the exact perturbed solves, computed by
    residual correction u+- = u0 + A+-^{-1}(f - A+- u0) (each correction
    solved to 1e-12 relative): per sampled cell |FD - g| <= 1e-5 |g| for
    cells with |g| >= 1e-3 max|g| and <= 1e-8 max|g| otherwise.
At full size (96^3, 12^3 boxes) the oracle's own u, lambda and gradient are
computed once (about a minute of CPU) and compared with the FP64 handle's
(1e-10 / 1e-8 / 1e-8) and with the benchmarked FP32 configuration's (gradient
error stated, at most 1e-6), the latter also checked by finite differences on
32 seeded cells.
"""

import sys
import time

import numpy as np
import pytest

from oracle import DDGOracle
from oracle.gradient import assemble_cc, coeff_grad_cc
from workloads import CSR, box_partition, cell_coords, grf, monomials, seed_rng

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STREAM_F, STREAM_KAPPA, STREAM_KAPPA_OBS = 0, 1, 2


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64).ravel()).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


class Case:
    def __init__(self, shape, boxes, cfg_id, p=2, overlap=1, ell=4.0, sigma=1.0):
        self.shape = tuple(shape)
        self.dims = tuple(reversed(self.shape)) + (1,) * (3 - len(self.shape))
        self.boxes = tuple(boxes)
        self.n = int(np.prod(self.shape))
        self.theta = grf(self.shape, ell, sigma, seed_rng(cfg_id, STREAM_KAPPA))
        self.theta_obs = grf(self.shape, ell, sigma, seed_rng(cfg_id, STREAM_KAPPA_OBS))
        self.f = seed_rng(cfg_id, STREAM_F).uniform(-1.0, 1.0, self.n)
        self.part = box_partition(self.shape, self.boxes)
        self.n_parts = int(np.prod(self.boxes))
        self.F = monomials(cell_coords(self.shape), p)
        self.overlap = overlap

    def solver(self, **kw):
        from paper_1504_00907_amd import DiffusionSolver
        say(f"[setup] grid {self.shape} boxes {self.boxes} {kw}")
        return DiffusionSolver(self.dims, self.F, self.part, self.n_parts, self.overlap, dev(self.theta), **kw)

    def oracle(self, theta):
        A = CSR.from_scipy(assemble_cc(np.exp(theta)))
        return A, DDGOracle(A, self.F, self.part, self.n_parts, self.overlap)


SMALL = {
    "3d16_b2": lambda: Case((16, 16, 16), (2, 2, 2), cfg_id=71),
    "3d_ragged": lambda: Case((10, 14, 18), (2, 2, 3), cfg_id=72),
    "2d40_b4": lambda: Case((40, 40), (4, 4), cfg_id=73, p=3, overlap=2),
}


def loss_and_grad(ds, theta, f, u_obs):
    from paper_1504_00907_amd import ddg_solve_fn
    th = dev(theta).requires_grad_(True)
    fd = dev(f).requires_grad_(True)
    u = ddg_solve_fn(th, fd, ds)
    L = ((u - u_obs) ** 2).sum()
    L.backward()
    return float(L.detach()), u.detach(), host(th.grad), host(fd.grad)


def fd_residual_correction(ds, theta, f, u0, u_obs, cell, h):
    """Central difference of L at the exact perturbed solves (residual correction)."""
    deltas = []
    for sgn in (1.0, -1.0):
        th = theta.copy()
        th.flat[cell] += sgn * h
        ds.refactor(dev(th))
        r = f - ds.solver.spmv(u0)
        deltas.append(ds.solve(r))
    dp, dm = deltas
    dL = torch.dot(dp - dm, 2.0 * u0 + dp + dm - 2.0 * u_obs)
    return float(dL) / (2.0 * h)


def check_fd(fd, g):
    gmax = np.abs(g).max()
    bad = []
    for c, (a, b) in enumerate(zip(fd, g)):
        if abs(b) >= 1e-3 * gmax:
            ok = abs(a - b) <= 1e-5 * abs(b)
        else:
            ok = abs(a - b) <= 1e-8 * gmax
        if not ok:
            bad.append((c, a, b))
    return bad


@pytest.mark.parametrize("bc", ["dirichlet", "x0"])
@pytest.mark.parametrize("name", list(SMALL))
def test_assembly_matches_oracle(name, bc):
    from paper_1504_00907_amd import cc_pattern, stencil_assemble
    c = SMALL[name]()
    rp, ci = cc_pattern(c.dims)
    val = torch.empty(int(rp[-1]), dtype=torch.float64, device="cuda")
    stencil_assemble(c.dims, dev(c.theta), val, bc=bc)
    M = assemble_cc(np.exp(c.theta), bc=bc)
    assert np.array_equal(rp, M.indptr) and np.array_equal(ci, M.indices)
    v = host(val)
    assert np.all(np.abs(v - M.data) <= 1e-14 * np.abs(M.data))


@pytest.mark.parametrize("bc", ["dirichlet", "x0"])
@pytest.mark.parametrize("name", list(SMALL))
def test_coeff_grad_kernel_matches_oracle(name, bc):
    from paper_1504_00907_amd import stencil_coeff_grad
    c = SMALL[name]()
    rng = seed_rng(74, 0)
    u, lam = rng.standard_normal(c.n), rng.standard_normal(c.n)
    g = host(stencil_coeff_grad(c.dims, dev(c.theta), dev(u), dev(lam), bc=bc))
    ref = coeff_grad_cc(np.exp(c.theta), u, lam, bc=bc).ravel()
    assert np.linalg.norm(g - ref) <= 1e-12 * np.linalg.norm(ref)


def test_stencil_rejects_unknown_bc():
    from paper_1504_00907_amd import DDGError, _lib
    import ctypes as C
    lib = _lib.load()
    d = (C.c_int32 * 3)(4, 4, 4)
    th = torch.zeros(64, dtype=torch.float64, device="cuda")
    val = torch.zeros(64 * 7, dtype=torch.float64, device="cuda")
    assert lib.ddg_stencil_assemble(d, th.data_ptr(), 7, val.data_ptr(), None) == -1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_autograd_matches_oracle_gradient(name, precision):
    c = SMALL[name]()
    tol = 1e-12
    ds = c.solver(rtol=tol, precision=precision)
    A, o = c.oracle(c.theta)
    _, o_obs = c.oracle(c.theta_obs)
    u_ref, _, _ = o.pcg(c.f, tol)
    uobs_ref, _, _ = o_obs.pcg(c.f, tol)
    lam_ref, _, _ = o.pcg(2.0 * (u_ref - uobs_ref), tol)
    g_ref = coeff_grad_cc(np.exp(c.theta), u_ref, lam_ref).ravel()

    ds.refactor(dev(c.theta_obs))
    u_obs = ds.solve(dev(c.f)).clone()
    say(f"[u_obs] iters {ds.last_info['iters']}")
    L, u, g, gf = loss_and_grad(ds, c.theta, c.f, u_obs)
    err_u = np.linalg.norm(host(u) - u_ref) / np.linalg.norm(u_ref)
    err_g = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    err_f = np.linalg.norm(gf - lam_ref) / np.linalg.norm(lam_ref)
    say(f"   {name} {precision}: |u-u_ref| {err_u:.2e} |g-g_ref| {err_g:.2e} |dL/df-lam| {err_f:.2e}")
    assert err_u <= 1e-10
    assert err_g <= 1e-8
    assert err_f <= 1e-8
    Lref = float(np.sum((u_ref - uobs_ref) ** 2))
    assert abs(L - Lref) <= 1e-9 * Lref
    ds.solver.close()


@pytest.mark.parametrize("name", ["3d16_b2", "2d40_b4"])
def test_autograd_matches_finite_differences(name):
    c = SMALL[name]()
    ds = c.solver(rtol=1e-12)
    ds.refactor(dev(c.theta_obs))
    u_obs = ds.solve(dev(c.f)).clone()
    _, u0, g, _ = loss_and_grad(ds, c.theta, c.f, u_obs)
    cells = seed_rng(75, 0).choice(c.n, size=16, replace=False)
    fd = np.array([fd_residual_correction(ds, c.theta, dev(c.f), u0, u_obs, int(k), 1e-6) for k in cells])
    rel = np.abs(fd - g[cells]) / np.abs(g[cells])
    say(f"   {name}: FD max rel err {rel.max():.2e}")
    assert not check_fd(fd, g[cells])
    ds.solver.close()


_ORACLE96 = {}


def oracle96(c, tol=1e-11):
    """Oracle u_obs, u, lambda and dL/dtheta at 96^3 (two setups, three PCG solves; about a minute)."""
    if "g" not in _ORACLE96:
        t0 = time.time()
        _, o_obs = c.oracle(c.theta_obs)
        uobs, it_obs, _ = o_obs.pcg(c.f, tol)
        del o_obs
        _, o = c.oracle(c.theta)
        u, it_u, _ = o.pcg(c.f, tol)
        lam, it_l, _ = o.pcg(2.0 * (u - uobs), tol)
        g = coeff_grad_cc(np.exp(c.theta), u, lam).ravel()
        say(f"[oracle 96^3] iters u_obs {it_obs} u {it_u} lambda {it_l}, {time.time() - t0:.1f} s")
        _ORACLE96.update(uobs=uobs, u=u, lam=lam, g=g, L=float(np.sum((u - uobs) ** 2)))
    return _ORACLE96


def case96():
    return Case((96, 96, 96), (8, 8, 8), cfg_id=4, ell=8.0)


def forward_adjoint(c, ds):
    """u_obs, then u(theta), dL/dtheta and lambda (= dL/df) through autograd."""
    from paper_1504_00907_amd import ddg_solve_fn
    ds.refactor(dev(c.theta_obs))
    u_obs = ds.solve(dev(c.f)).clone()
    th = dev(c.theta).requires_grad_(True)
    fd_ = dev(c.f).requires_grad_(True)
    u = ddg_solve_fn(th, fd_, ds)
    fwd_iters = ds.last_info["iters"]
    L = ((u - u_obs) ** 2).sum()
    L.backward()
    say(f"   forward iters {fwd_iters}, adjoint iters {ds.last_info['iters']}")
    return u_obs, u.detach(), host(th.grad), host(fd_.grad), float(L.detach())


def test_full_size_96_fp64_against_oracle():
    """96^3 cells, 8^3 boxes of 12^3, overlap 1, p = 2, FP64 factors, rtol 1e-12: u, lambda
    and dL/dtheta against the oracle's (which solves at 1e-11): u within 1e-10, lambda and
    the gradient within 1e-8 (norm-wise); assembled values and the gradient kernel on the
    GPU's own u and lambda against the oracle formulas."""
    c = case96()
    ref = oracle96(c)
    t0 = time.time()
    ds = c.solver(rtol=1e-12)
    say(f"   setup {time.time() - t0:.1f} s")
    u_obs, u0, g, lam, L = forward_adjoint(c, ds)
    err_u = np.linalg.norm(host(u0) - ref["u"]) / np.linalg.norm(ref["u"])
    err_l = np.linalg.norm(lam - ref["lam"]) / np.linalg.norm(ref["lam"])
    err_g = np.linalg.norm(g - ref["g"]) / np.linalg.norm(ref["g"])
    say(f"   fp64: |u-u_or| {err_u:.2e} |lam-lam_or| {err_l:.2e} |g-g_or| {err_g:.2e}")
    assert err_u <= 1e-10 and err_l <= 1e-8 and err_g <= 1e-8
    assert abs(L - ref["L"]) <= 1e-8 * ref["L"]
    val = host(ds.val)
    M = assemble_cc(np.exp(c.theta))
    assert np.all(np.abs(val - M.data) <= 1e-14 * np.abs(M.data))
    kern = coeff_grad_cc(np.exp(c.theta), host(u0), lam).ravel()
    assert np.linalg.norm(g - kern) <= 1e-10 * np.linalg.norm(kern)
    assert np.linalg.norm(c.f - M @ host(u0)) <= 1e-11 * np.linalg.norm(c.f)
    ds.solver.close()


def test_full_size_96_fp32_bench_configuration():
    """The configuration the benchmark times (FP32 factors, rtol 1e-10): the gradient
    against the oracle's (stated, bounded by 1e-6), and central finite differences by
    residual correction on 32 seeded cells within 1e-5 per cell."""
    c = case96()
    ref = oracle96(c)
    ds = c.solver(rtol=1e-10, precision="fp32")
    u_obs, u0, g, lam, L = forward_adjoint(c, ds)
    err_g = np.linalg.norm(g - ref["g"]) / np.linalg.norm(ref["g"])
    err_u = np.linalg.norm(host(u0) - ref["u"]) / np.linalg.norm(ref["u"])
    say(f"   fp32 rtol 1e-10: |u-u_or| {err_u:.2e} |g-g_or| {err_g:.2e}")
    assert err_g <= 1e-6
    cells = seed_rng(4, 5).choice(c.n, size=32, replace=False)
    t0 = time.time()
    fd = np.array([fd_residual_correction(ds, c.theta, dev(c.f), u0, u_obs, int(k), 1e-6) for k in cells])
    rel = np.abs(fd - g[cells]) / np.abs(g[cells])
    say(f"   FD over 32 cells: max rel err {rel.max():.2e} ({time.time() - t0:.1f} s)")
    assert not check_fd(fd, g[cells])
    ds.solver.close()


def test_backward_after_another_forward():
    """Two forwards on one handle, then the backwards in reverse order: each gradient
    equals the one from its own forward/backward pair (the handle is refactored back)."""
    from paper_1504_00907_amd import ddg_solve_fn
    c = SMALL["3d16_b2"]()
    ds = c.solver(rtol=1e-12)
    ds.refactor(dev(c.theta_obs))
    u_obs = ds.solve(dev(c.f)).clone()
    th1 = dev(c.theta)
    th2 = dev(c.theta + 0.3 * np.sin(np.arange(c.n)).reshape(c.theta.shape))
    ref = []
    for th in (th1, th2):
        _, _, g, _ = loss_and_grad(ds, host(th).reshape(c.theta.shape), c.f, u_obs)
        ref.append(g)
    t1 = th1.clone().requires_grad_(True)
    t2 = th2.clone().requires_grad_(True)
    L1 = ((ddg_solve_fn(t1, dev(c.f), ds) - u_obs) ** 2).sum()
    L2 = ((ddg_solve_fn(t2, dev(c.f), ds) - u_obs) ** 2).sum()
    L2.backward()
    L1.backward()
    for t, g in ((t1, ref[0]), (t2, ref[1])):
        err = np.linalg.norm(host(t.grad) - g) / np.linalg.norm(g)
        say(f"   reordered backward: rel diff {err:.2e}")
        assert err <= 1e-12
    ds.solver.close()
