"""Diagonal storage of stencil operators against the CSR rows (GPU, C ABI).

The row dots (SpMV, CG's q = A p, local residuals, coarse restriction, true
residual) read a stencil operator from its diagonals when every system's
entries lie on a few offset pairs and the values are symmetric bit for bit.
The rows are summed in the CSR's sorted-column order, so every result must
equal the CSR path's bit for bit: A x, M^{-1} r, the CG iterates and the
iteration counts.  Values that are not exactly symmetric switch the handle to
the CSR rows.  FP64 solves are also held against the oracle.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import DDGOracle  # noqa: E402
from parity_util import FP64_U_TOL, rel  # noqa: E402
from paper_1504_00907_amd import DDGBatchSolver, DDGSolver  # noqa: E402
from workloads import CSR, cfg1, cfg4_instance, diffusion_problem  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(msg):
    print(msg, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def cases():
    yield "cfg1_nodes_5pt", cfg1()
    yield "3d_10x14x18_7pt", diffusion_problem((10, 14, 18), (2, 2, 3), 1, 2, cfg_id=21, rtol=1e-10)
    yield "2d_33x47_x0bc", diffusion_problem((33, 47), (3, 4), 2, 2, cfg_id=22, rtol=1e-10, bc="x0")
    yield "3d_16_ovl0", diffusion_problem((16, 16, 16), (2, 2, 2), 0, 1, cfg_id=23, rtol=1e-10)


@pytest.mark.parametrize("name,P", list(cases()), ids=lambda c: c if isinstance(c, str) else "")
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dia_equals_csr_bit_for_bit(name, P, precision):
    say(f"dia vs csr: {name} {precision} n={P.n}")
    sd = DDGSolver.from_problem(P, precision=precision, rtol=P.rtol)
    sc = DDGSolver.from_problem(P, precision=precision, rtol=P.rtol, matrix_format="csr")
    assert sd.info()["matrix_format"] == 2
    assert sc.info()["matrix_format"] == 1
    rng = np.random.default_rng(7)
    x = dev(rng.standard_normal(P.n))
    assert np.array_equal(host(sd.spmv(x)), host(sc.spmv(x)))
    assert np.array_equal(host(sd.spmv(x)), P.A.to_scipy() @ host(x)) or \
        rel(host(sd.spmv(x)), P.A.to_scipy() @ host(x)) <= 1e-15
    f = dev(P.f)
    assert np.array_equal(host(sd.apply_precond(f)), host(sc.apply_precond(f)))
    ud, id_ = sd.solve(f)
    uc, ic = sc.solve(f)
    assert id_["iters"] == ic["iters"]
    assert np.array_equal(host(ud), host(uc))
    assert id_["true_rel_res"] == ic["true_rel_res"]
    if precision == "fp64":
        o = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
        xo, it, _ = o.pcg(P.f, P.rtol)
        assert abs(it - id_["iters"]) <= 1
        if it == id_["iters"]:
            assert rel(host(ud), xo) <= FP64_U_TOL
    sd.close()
    sc.close()


def test_dia_batch_of_uneven_systems_equals_csr():
    probs = [cfg4_instance(i, L) for i, L in enumerate([40, 57, 33, 64])]
    say("dia vs csr: batch of 4 uneven 2D systems")
    tup = [(p.A.row_ptr, p.A.col_idx, p.A.val, p.F, p.part, p.n_parts) for p in probs]
    bd = DDGBatchSolver(tup, overlap=2, precision="fp32")
    bc = DDGBatchSolver(tup, overlap=2, precision="fp32", matrix_format="csr")
    assert bd.info()["matrix_format"] == 2 and bc.info()["matrix_format"] == 1
    f = dev(np.concatenate([p.f for p in probs]))
    assert np.array_equal(host(bd.apply_precond(f)), host(bc.apply_precond(f)))
    ud, infd = bd.solve(f)
    uc, infc = bc.solve(f)
    assert [i["iters"] for i in infd] == [i["iters"] for i in infc]
    assert np.array_equal(host(ud), host(uc))
    bd.close()
    bc.close()


def test_values_not_exactly_symmetric_use_csr_rows():
    P = diffusion_problem((12, 12, 12), (2, 2, 2), 1, 2, cfg_id=24, rtol=1e-10)
    A = P.A.to_scipy().tocsr()
    A.sort_indices()
    # one off-diagonal entry moved by one unit in the last place (its transpose keeps its bits)
    g = 500
    t = A.indptr[g]
    assert A.indices[t] < g
    val = A.data.copy()
    val[t] = np.nextafter(val[t], 0.0)
    Q = CSR(n=A.shape[0], row_ptr=A.indptr.astype(np.int64), col_idx=A.indices.astype(np.int32), val=val)
    say("dia: asymmetric bits fall back to CSR")
    s = DDGSolver(P.n, Q.row_ptr, Q.col_idx, Q.val, P.F, P.part, P.n_parts, P.overlap, rtol=1e-10)
    assert s.info()["matrix_format"] == 1
    x = dev(np.random.default_rng(3).standard_normal(P.n))
    y = host(s.spmv(x))
    Aq = Q.to_scipy()
    assert rel(y, Aq @ host(x)) <= 1e-15
    # a refactor with exactly symmetric values turns the diagonals back on
    s.refactor(dev(A.data))
    assert s.info()["matrix_format"] == 2
    assert rel(host(s.spmv(x)), A @ host(x)) <= 1e-15
    s.close()
