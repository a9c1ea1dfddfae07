"""Material-aware generating vectors (Section 7 problem C) on the GPU.

The two-material coefficient S + 100 J on a structured grid whose boxes do
not follow the material boundary; generating vectors plain (degree-p
monomials) or material-aware (the monomials times J and times 1 - J).  The
GPU keeps the same columns per subdomain as the oracle, its FP64 solves match
the oracle's, and with the cubic basis the material-aware space needs fewer
iterations (the paper reports close to half; the count is context).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import DDGOracle  # noqa: E402
from parity_util import FP64_U_TOL, fp64_u_error  # noqa: E402
from paper_1504_00907_amd import DDGSolver  # noqa: E402
from workloads.materials import material_problem  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("aware", [False, True], ids=["plain", "aware"])
def test_material_fp64_matches_oracle(aware):
    P = material_problem(96, 6, 1, 3, aware)
    o = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
    s = DDGSolver.from_problem(P, rtol=P.rtol)
    assert np.array_equal(s.kcounts(), o.k_counts)
    u, inf = s.solve(dev(P.f))
    x, it, _ = o.pcg(P.f, P.rtol)

    def rerun(m):
        t = DDGSolver.from_problem(P, rtol=0.0, max_iter=m)
        v, _ = t.solve(dev(P.f), raise_on_error=False)
        v = host(v)
        t.close()
        return v

    err, at = fp64_u_error(host(u), inf["iters"], x, it, rerun, lambda m: o.pcg(P.f, 0.0, m)[0])
    print(f"material {'aware' if aware else 'plain'}: iters gpu {inf['iters']} oracle {it}, err {err:.2e}", flush=True)
    assert err <= FP64_U_TOL
    s.close()


def test_material_aware_cubic_basis_needs_fewer_iterations_on_gpu():
    its = {}
    for aware in (False, True):
        P = material_problem(256, 8, 1, 3, aware)
        s = DDGSolver.from_problem(P, rtol=1e-9, precision="fp32")
        _, inf = s.solve(dev(P.f))
        its[aware] = inf["iters"]
        s.close()
    print(f"material 256^2 p=3: plain {its[False]} aware {its[True]} iterations", flush=True)
    assert its[True] < its[False]
