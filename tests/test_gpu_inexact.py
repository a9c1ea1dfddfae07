"""SSOR local smoothing (Section 7's inexact variant) on the GPU against the oracle.

The subdomain problems are smoothed by symmetric SOR sweeps instead of being
solved exactly (DDG_LOCAL_SSOR); the coarse solve stays exact.  Preconditioner
applications must match the inexact oracle's to 1e-12 and FP64 solves to
1e-10 at a common iteration count (iterations within one).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.inexact import InexactDDGOracle  # noqa: E402
from parity_util import FP64_U_TOL, fp64_u_error, rel  # noqa: E402
from paper_1504_00907_amd import DDGSolver  # noqa: E402
from workloads import cfg1, diffusion_problem  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [("cfg1", 1.0, 1), ("3d12", 1.0, 1), ("3d12", 1.5, 2), ("3d14x10x12", 1.2, 1)]


def problem(name):
    if name == "cfg1":
        return cfg1()
    if name == "3d12":
        return diffusion_problem((12, 12, 12), (3, 3, 3), 1, 2, cfg_id=71, rtol=1e-10)
    return diffusion_problem((14, 10, 12), (2, 2, 3), 1, 2, cfg_id=72, rtol=1e-10)


@pytest.mark.parametrize("name,omega,sweeps", CASES, ids=[f"{c[0]}_w{c[1]}_s{c[2]}" for c in CASES])
def test_ssor_matches_oracle(name, omega, sweeps):
    P = problem(name)
    o = InexactDDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap, omega=omega, sweeps=sweeps)
    kw = dict(local_solver="ssor", ssor_omega=omega, ssor_sweeps=sweeps)
    s = DDGSolver.from_problem(P, rtol=P.rtol, **kw)
    assert s.info()["factor_bytes"] == 0
    r = np.random.default_rng(9).standard_normal(P.n)
    assert rel(host(s.apply_precond(dev(r))), o.apply(r)) <= 1e-12
    u, inf = s.solve(dev(P.f))
    x, it, _ = o.pcg(P.f, P.rtol)

    def rerun(m):
        t = DDGSolver.from_problem(P, rtol=0.0, max_iter=m, **kw)
        v, _ = t.solve(dev(P.f), raise_on_error=False)
        v = host(v)
        t.close()
        return v

    err, at = fp64_u_error(host(u), inf["iters"], x, it, rerun, lambda m: o.pcg(P.f, 0.0, m)[0])
    print(f"ssor {name} omega {omega} sweeps {sweeps}: iters gpu {inf['iters']} oracle {it}, err {err:.2e}", flush=True)
    assert err <= FP64_U_TOL
    s.close()


def test_ssor_option_errors():
    P = cfg1()
    for kw in (dict(ssor_omega=2.0), dict(ssor_omega=0.0), dict(ssor_sweeps=0)):
        with pytest.raises(Exception, match="INVALID_ARG"):
            DDGSolver.from_problem(P, local_solver="ssor", **kw)
    with pytest.raises(Exception, match="UNSUPPORTED"):
        DDGSolver.from_problem(P, local_solver="ssor", schedule="queue")
