"""Bounded waits of the local-solve launches, forced to give up from the host.

DDG_SPIN_LIMIT shortens every wait of the sweep kernels; DDG_SWEEP_FAULT leaves
waits unsatisfied (bit 0: the two chains of a subdomain never hand over; bit 1:
the first workgroup of a group never counts itself at a barrier).  The waits give
up, so every kernel ends; the solve reports the timeout; and once the switch is
cleared the same handle solves exactly as before the failure, bit for bit (the
handoff flags and the barrier counts were cleared with the error).
"""

import sys

import numpy as np
import pytest

from workloads import cfg1
from workloads.elasticity import elasticity_q1

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def solve_fail_recover(s, f, monkeypatch, fault, message):
    from paper_1504_00907_amd import DDGError
    u0, i0 = s.solve(f)
    u0 = host(u0)
    monkeypatch.setenv("DDG_SPIN_LIMIT", "256")
    monkeypatch.setenv("DDG_SWEEP_FAULT", str(fault))
    with pytest.raises(DDGError, match=message):
        s.solve(f)
    monkeypatch.delenv("DDG_SWEEP_FAULT")
    monkeypatch.delenv("DDG_SPIN_LIMIT")
    u1, i1 = s.solve(f)
    say(f"   fault {fault}: iters before {i0['iters']}, after {i1['iters']}")
    assert i1["status"] == 0 and i1["iters"] == i0["iters"]
    assert np.array_equal(host(u1), u0)


def test_chain_handoff_timeout(monkeypatch):
    """Two-chain launches on the 2D Poisson workload: the handoff is never signalled."""
    from paper_1504_00907_amd import DDGSolver
    monkeypatch.delenv("DDG_NO_TWIST", raising=False)
    P = cfg1()
    s = DDGSolver.from_problem(P, rtol=P.rtol)
    solve_fail_recover(s, dev(P.f), monkeypatch, 1, "handoff timed out")
    s.close()


def test_grouped_barrier_timeout(monkeypatch):
    """Grouped launches (four workgroups per chain, one chain per subdomain) on the
    small elasticity case: the first workgroup of each group never arrives."""
    from paper_1504_00907_amd import DDGSolver
    monkeypatch.setenv("DDG_NO_TWIST", "1")
    monkeypatch.setenv("DDG_SWEEP_GROUPS", "4")
    monkeypatch.setenv("DDG_SWEEP_SPLIT_ROUNDS", "4")
    P = elasticity_q1(nel=10, part_dofs=(200, 500), min_dofs=200, sigma=1.0, rtol=1e-10)
    s = DDGSolver.from_problem(P, rtol=P.rtol, tile=16)
    solve_fail_recover(s, dev(P.f), monkeypatch, 2, "grouped sweep barrier timed out")
    assert s.info()["sweep_groups"] == 4
    s.close()
