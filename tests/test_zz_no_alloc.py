"""The allocation-free preconditioner entry point against ddg_apply_precond.

ddg_apply_precond_noalloc runs the same kernels in the same order as
ddg_apply_precond, with its per-application buffers in the library's static
device scratch instead of the handle's, so the two must agree bit for bit.
Both are called through the C ABI (ctypes), on two handles in a row, the
second smaller than the first, then the first again (its coarse padding must
be cleared after the smaller handle's call left other values behind).  The
FP64 result is also held against the FP64 oracle's M^{-1} r (Section 6).
"""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import DDGOracle  # noqa: E402
from paper_1504_00907_amd import DDGSolver, _lib  # noqa: E402
from workloads import cfg1, diffusion_problem  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(s: DDGSolver, r: torch.Tensor):
    lib = _lib.load()
    z_ref = torch.full_like(r, float("nan"))
    z_na = torch.full_like(r, float("nan"))
    _lib.check(lib.ddg_apply_precond(s._h, C.c_void_p(r.data_ptr()), C.c_void_p(z_ref.data_ptr())))
    _lib.check(lib.ddg_apply_precond_noalloc(s._h, C.c_void_p(r.data_ptr()), C.c_void_p(z_na.data_ptr())))
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_na.cpu().numpy()


@pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")
def test_noalloc_matches_apply_precond_two_sizes():
    big = diffusion_problem((24, 24, 24), (3, 3, 3), 1, 2, cfg_id=11, rtol=1e-8)
    small = cfg1()
    s_big = DDGSolver.from_problem(big, precision="fp32")
    s_small = DDGSolver.from_problem(small, precision="fp64")
    r_big = torch.from_numpy(big.f).cuda()
    r_small = torch.from_numpy(small.f).cuda()
    print(f"noalloc: big n={big.n} then small n={small.n}", flush=True)
    zb_ref, zb_na = _both(s_big, r_big)
    assert np.all(np.isfinite(zb_ref))
    assert np.array_equal(zb_ref, zb_na)
    zs_ref, zs_na = _both(s_small, r_small)
    assert np.array_equal(zs_ref, zs_na)
    o = DDGOracle(small.A, small.F, small.part, small.n_parts, small.overlap)
    zo = o.apply(small.f)
    assert np.linalg.norm(zs_na - zo) <= 1e-12 * np.linalg.norm(zo)
    # the first handle again, after the smaller one left its values in the scratch
    zb2_ref, zb2_na = _both(s_big, r_big)
    assert np.array_equal(zb2_na, zb_ref) and np.array_equal(zb2_ref, zb_ref)
    s_big.close()
    s_small.close()


@pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")
def test_noalloc_rejects_handles_beyond_its_scratch():
    # 2048^2 cells without overlap: 8 bytes per row of the expanded sets alone fill the 32 MiB
    P = diffusion_problem((2048, 2048), (32, 32), 0, 0, cfg_id=12, rtol=1e-8, sigma=0.0)
    s = DDGSolver.from_problem(P, precision="fp32")
    r = torch.from_numpy(P.f).cuda()
    z = torch.zeros_like(r)
    lib = _lib.load()
    rc = lib.ddg_apply_precond_noalloc(s._h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()))
    assert _lib.STATUS[rc] == "UNSUPPORTED"
    assert b"32 MiB" in lib.ddg_last_error()
    torch.cuda.synchronize()
    assert float(z.abs().max()) == 0.0   # nothing was launched
    s.close()
