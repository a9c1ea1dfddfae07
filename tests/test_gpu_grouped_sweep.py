"""Grouped local-solve launches: several workgroups share one chain of a
subdomain's local solve, and every level of at least a set number of tile rounds
is split between them (each sums the slots of its own rounds; the partial sums go
through global memory and are added in workgroup order, so every workgroup of the
chain holds the same level result).

Forced on the small Q1 elasticity case with tile edge 16 (levels of 1 to 11
rounds; with 8 workgroups and levels split from 2 rounds, some workgroups of a
split level have no round and add zeros): preconditioner applications match the
oracle's M^{-1} r (1e-12 in FP64)
and the one-workgroup launches (1e-13 in FP64: only the order of the level sums
differs), three applications in a row (the barrier counts return to zero after
each launch), in both the two-chain and the one-chain schedule; solves keep the
one-workgroup iteration counts and are repeatable bit for bit.
"""

import sys

import numpy as np
import pytest

from oracle import DDGOracle
from workloads import seed_rng
from workloads.elasticity import elasticity_q1

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

_cache = {}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def problem():
    if "p" not in _cache:
        P = elasticity_q1(nel=10, part_dofs=(200, 500), min_dofs=200, sigma=1.0, rtol=1e-10)
        _cache["p"] = (P, DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap))
    return _cache["p"]


def solver(P, groups, monkeypatch, split=None, **kw):
    from paper_1504_00907_amd import DDGSolver
    monkeypatch.setenv("DDG_SWEEP_GROUPS", str(groups))
    monkeypatch.setenv("DDG_SWEEP_SPLIT_ROUNDS", str(split or max(2, groups)))
    say(f"[setup] groups {groups} {kw}")
    s = DDGSolver.from_problem(P, tile=16, **kw)
    assert s.info()["tile"] == 16
    return s


@pytest.mark.parametrize("twist", [True, False], ids=["two_chains", "one_chain"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("groups,split", [(2, 2), (3, 3), (4, 4), (8, 2)], ids=["g2", "g3", "g4", "g8s2"])
def test_grouped_preconditioner(groups, split, precision, twist, monkeypatch):
    if not twist:
        monkeypatch.setenv("DDG_NO_TWIST", "1")
    P, o = problem()
    rs = [seed_rng(93, j).standard_normal(P.n) for j in range(3)]
    s1 = solver(P, 1, monkeypatch, precision=precision)
    z1 = [host(s1.apply_precond(dev(r))) for r in rs]
    assert s1.info()["sweep_groups"] == 1
    s1.close()
    s = solver(P, groups, monkeypatch, split, precision=precision)
    zg = [host(s.apply_precond(dev(r))) for r in rs]
    assert s.info()["sweep_groups"] == groups
    s.close()
    tol = 1e-12 if precision == "fp64" else 1e-5
    for r, a, b in zip(rs, zg, z1):
        assert np.isfinite(a).all()
        ref = o.apply(r)
        err = np.linalg.norm(a - ref) / np.linalg.norm(ref)
        diff = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(f"   groups {groups} split {split} {precision} twist {twist}: vs oracle {err:.2e}, vs one workgroup {diff:.2e}")
        assert err <= tol
        assert diff <= (1e-13 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grouped_solve(precision, monkeypatch):
    P, o = problem()
    rtol = 1e-10 if precision == "fp64" else 1e-8
    res = {}
    for groups in (1, 4):
        s = solver(P, groups, monkeypatch, precision=precision, rtol=rtol)
        u, info = s.solve(dev(P.f))
        u = host(u)
        u2, info2 = s.solve(dev(P.f))
        assert np.array_equal(u, host(u2)) and info2["iters"] == info["iters"]
        assert s.info()["sweep_groups"] == groups
        res[groups] = (u, info)
        s.close()
    (u1, i1), (u4, i4) = res[1], res[4]
    true_res = np.linalg.norm(P.f - P.A.to_scipy() @ u4) / np.linalg.norm(P.f)
    diff = np.linalg.norm(u4 - u1) / np.linalg.norm(u1)
    say(f"   {precision}: iters {i4['iters']} (one workgroup {i1['iters']}), true res {true_res:.2e}, "
        f"u vs one workgroup {diff:.2e}")
    assert i4["status"] == 0 and i4["iters"] == i1["iters"]
    assert true_res <= (1e-9 if precision == "fp64" else 1e-8)
    assert diff <= (1e-10 if precision == "fp64" else 1e-6)
