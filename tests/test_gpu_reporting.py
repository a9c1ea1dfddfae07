"""CG reporting, direction-update variants, boundary option and launch accounting
on the GPU, through the C ABI, against the FP64 oracle.

* The CG coefficients and residual history of an FP64 solve equal the
  oracle's (1e-9 relative per entry, same iteration count); the fractional
  iteration count, the Lanczos extremes and the CG iteration bound computed by
  the library equal the oracle's functions applied to the oracle's own history
  (Section 7 protocol).
* Polak-Ribiere CG: FP64 u within 1e-10 of the oracle's Polak-Ribiere PCG at a
  common iteration count; FP32 factors reach a true residual <= 1e-8.
* Problem A boundary conditions (one Dirichlet face, Neumann elsewhere): FP64
  solve against the oracle, FP32 factors to 1e-8.
* Profiling credits only launches that ran: a solve of k iterations runs k
  preconditioner applications (2C local-solve launches each); launches
  enqueued after convergence are counted apart as idle.
"""

import sys

import numpy as np
import pytest

from oracle import DDGOracle, cg_iteration_bound, condition_estimate, fractional_iterations
from parity_util import FP64_U_TOL, MIXED_RES_TOL, fp64_u_error, true_rel_res
from workloads import cfg1, diffusion_problem, seed_rng

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = {
    "cfg1": lambda: cfg1(),
    "3d20": lambda: diffusion_problem((20,) * 3, (2,) * 3, 1, 2, cfg_id=51, rtol=1e-10, ell=4.0, name="3d20"),
    "3d16_x0": lambda: diffusion_problem((16,) * 3, (2,) * 3, 1, 2, cfg_id=54, rtol=1e-10, ell=4.0, bc="x0",
                                         name="3d16_x0"),
}
_cache = {}


def problem(name):
    if name not in _cache:
        P = CASES[name]()
        _cache[name] = (P, DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap))
    return _cache[name]


def make_solver(P, **kw):
    from paper_1504_00907_amd import DDGSolver
    say(f"[setup] {P.name} n={P.n} parts={P.n_parts} {kw}")
    return DDGSolver.from_problem(P, **kw)


def rerun_gpu(P, m, **kw):
    s = make_solver(P, rtol=0.0, max_iter=m, **kw)
    u, info = s.solve(dev(P.f), raise_on_error=False)
    assert info["iters"] == m
    u = host(u)
    s.close()
    return u


@pytest.mark.parametrize("name", ["cfg1", "3d20", "3d16_x0"])
def test_cg_history_and_report_match_oracle(name):
    P, o = problem(name)
    s = make_solver(P, rtol=P.rtol)
    u, info = s.solve(dev(P.f))
    x, it, oi = o.pcg(P.f, P.rtol)
    say(f"   {name}: iters gpu {info['iters']} oracle {it}")
    assert info["iters"] == it
    a, b, r = s.cg_history()
    assert a.size == it and b.size == it - 1 and r.size == it + 1
    assert np.all(np.abs(a - np.array(oi["alpha"])) <= 1e-9 * np.abs(oi["alpha"]))
    assert np.all(np.abs(b - np.array(oi["beta"])) <= 1e-9 * np.abs(oi["beta"]))
    assert np.all(np.abs(r - np.array(oi["res"])) <= 1e-9 * np.array(oi["res"]))
    rep = s.cg_report()
    frac = fractional_iterations(oi["res"], P.rtol)
    lo, hi, kappa = condition_estimate(oi["alpha"], oi["beta"])
    say(f"   report {rep}; oracle frac {frac:.6f} lambda [{lo:.6f}, {hi:.6f}]")
    assert rep["iters"] == it
    assert abs(rep["frac_iters"] - frac) <= 1e-6
    assert it - 1 < rep["frac_iters"] <= it
    assert abs(rep["lambda_min"] - lo) <= 1e-8 * lo and abs(rep["lambda_max"] - hi) <= 1e-8 * hi
    assert 0.0 < rep["lambda_min"] <= rep["lambda_max"] <= 1.0 + 1e-10
    assert rep["iter_bound"] == cg_iteration_bound(rep["kappa"], P.rtol)
    s.close()


@pytest.mark.parametrize("name", ["cfg1", "3d20", "3d16_x0"])
def test_polak_ribiere_fp64_matches_oracle(name):
    P, o = problem(name)
    s = make_solver(P, rtol=P.rtol, cg_variant="pr")
    u, info = s.solve(dev(P.f))
    u = host(u)
    s.close()
    x, it, _ = o.pcg(P.f, P.rtol, variant="pr")
    err, at = fp64_u_error(u, info["iters"], x, it, lambda m: rerun_gpu(P, m, cg_variant="pr"),
                           lambda m: o.pcg(P.f, 0.0, m, variant="pr")[0])
    say(f"   {name} PR: iters gpu {info['iters']} oracle {it} err {err:.2e} (at {at})")
    assert info["status"] == 0 and err <= FP64_U_TOL


@pytest.mark.parametrize("name", ["cfg1", "3d20", "3d16_x0"])
def test_mixed_modes_each_variant(name):
    P, o = problem(name)
    _, it, _ = o.pcg(P.f, 1e-8)
    for variant in ("fr", "pr"):
        s = make_solver(P, rtol=1e-8, precision="fp32", cg_variant=variant)
        u, info = s.solve(dev(P.f))
        u = host(u)
        s.close()
        res = true_rel_res(P.A.to_scipy(), u, P.f)
        say(f"   {name} fp32 {variant}: iters {info['iters']} (oracle fp64 {it}) true res {res:.2e}")
        assert info["status"] == 0 and res <= MIXED_RES_TOL and abs(info["iters"] - it) <= 1


def test_x0_boundary_fp64_matches_oracle():
    P, o = problem("3d16_x0")
    s = make_solver(P, rtol=P.rtol)
    r = seed_rng(91, 0).standard_normal(P.n)
    z = host(s.apply_precond(dev(r)))
    ref = o.apply(r)
    assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)
    u, info = s.solve(dev(P.f))
    u = host(u)
    s.close()
    x, it, _ = o.pcg(P.f, P.rtol)
    err, at = fp64_u_error(u, info["iters"], x, it, lambda m: rerun_gpu(P, m), lambda m: o.pcg(P.f, 0.0, m)[0])
    say(f"   x0 bc: iters gpu {info['iters']} oracle {it} err {err:.2e}")
    assert err <= FP64_U_TOL


@pytest.mark.parametrize("schedule", ["colours", "queue"])
def test_profile_credits_only_launches_that_ran(schedule):
    P, o = problem("3d20")
    s = make_solver(P, rtol=1e-8, precision="fp32", schedule=schedule)
    info0 = s.info()
    C = info0["n_colours"]
    s.profile_enable(True)
    s.profile_read()
    u, info = s.solve(dev(P.f))
    pr = s.profile_read()
    k = info["iters"]
    per_app = 2 * C if schedule == "colours" else 2
    enq = 4 * ((k + 3) // 4)
    say(f"   {schedule}: iters {k}, launches {pr['launches']} idle {pr['idle_launches']}")
    assert pr["launches"] == per_app * k
    assert pr["idle_launches"] == per_app * (enq - k + 1)
    # the credited bytes are k applications' worth
    z = s.apply_precond(dev(P.f))
    one = s.profile_read()
    assert one["launches"] == per_app and one["idle_launches"] == 0
    assert pr["bytes"] == k * one["bytes"]
    s.close()
