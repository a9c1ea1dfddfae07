"""Python binding of the C ABI: argument marshalling only.

Host numpy arrays go to ``ddg_setup``; device vectors are torch float64
tensors on the current HIP device and all work runs on the handle's stream
(by default torch's current stream at construction time).
"""

from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import CgReport, DDGError, Info, Options, Problem, TuneEntry, check


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dev(t: torch.Tensor, n: int, name: str) -> int:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous float64 device tensor of length {n}")
    return t.data_ptr()


def _options(lib, precision, rtol, max_iter, rank_tol, tile, block_target, check_every, stream,
             schedule="auto", cg_variant="fr", matrix_format="auto", local_solver="exact", ssor_omega=1.0,
             ssor_sweeps=1, coarse_solver="inverse", ic_tol=1e-6, ic_maxit=200):
    opt = Options()
    lib.ddg_default_options(C.byref(opt))
    opt.precision = _lib.PRECISION[precision]
    opt.rtol = rtol
    opt.max_iter = max_iter
    opt.rank_tol = rank_tol
    opt.tile = tile
    opt.block_target = block_target
    opt.check_every = check_every
    opt.schedule = _lib.SCHEDULE[schedule]
    opt.cg_variant = _lib.CG_VARIANT[cg_variant]
    opt.matrix_format = _lib.MATRIX_FORMAT[matrix_format]
    opt.local_solver = _lib.LOCAL_SOLVER[local_solver]
    opt.ssor_omega = float(ssor_omega)
    opt.ssor_sweeps = int(ssor_sweeps)
    opt.coarse_solver = _lib.COARSE_SOLVER[coarse_solver]
    opt.ic_tol = float(ic_tol)
    opt.ic_maxit = int(ic_maxit)
    opt.stream = C.c_void_p(stream.cuda_stream)
    return opt


class DDGSolver:
    """DDG two-level PCG handle (see include/ddg.h for the semantics)."""

    def __init__(self, n: int, row_ptr, col_idx, val, F: Optional[np.ndarray], part, n_parts: int,
                 overlap: int, precision: str = "fp64", rtol: float = 1e-8, max_iter: int = 1000,
                 rank_tol: float = 1e-10, tile: int = 0, block_target: int = 0, check_every: int = 4,
                 stream: Optional[torch.cuda.Stream] = None, schedule: str = "auto", cg_variant: str = "fr",
                 matrix_format: str = "auto", part0=None, n_parts0: int = 0, local_solver: str = "exact",
                 ssor_omega: float = 1.0, ssor_sweeps: int = 1, coarse_solver: str = "inverse",
                 ic_tol: float = 1e-6, ic_maxit: int = 200):
        """``part0`` (coarse subdomain of every subdomain, ``n_parts0`` of them) selects
        the three-level V-cycle (``ddg_setup_three_level``)."""
        lib = _lib.load()
        self._lib = lib
        self.n = int(n)
        self.max_iter = int(max_iter)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        vv = np.ascontiguousarray(val, dtype=np.float64)
        pp = np.ascontiguousarray(part, dtype=np.int32)
        if F is None or F.size == 0:
            k, Fp, Fh = 0, None, None
        else:
            Fh = np.asfortranarray(F, dtype=np.float64)
            k = Fh.shape[1]
            Fp = _ptr(Fh)
        if rp.shape != (self.n + 1,) or pp.shape != (self.n,):
            raise ValueError("row_ptr must have n+1 entries and part n entries")
        if ci.shape[0] != int(rp[-1]) or vv.shape[0] != int(rp[-1]):
            raise ValueError("col_idx/val length must equal row_ptr[-1]")
        if Fh is not None and Fh.shape[0] != self.n:
            raise ValueError("F must have n rows")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opt = _options(lib, precision, rtol, max_iter, rank_tol, tile, block_target, check_every, self.stream,
                       schedule, cg_variant, matrix_format, local_solver, ssor_omega, ssor_sweeps,
                       coarse_solver, ic_tol, ic_maxit)
        self.precision = precision
        h = C.c_void_p()
        if part0 is None:
            check(lib.ddg_setup(C.byref(h), self.n, _ptr(rp), _ptr(ci), _ptr(vv), k, Fp, _ptr(pp),
                                int(n_parts), int(overlap), C.byref(opt)))
        else:
            p0 = np.ascontiguousarray(part0, dtype=np.int32)
            if p0.shape != (int(n_parts),):
                raise ValueError("part0 must have n_parts entries")
            check(lib.ddg_setup_three_level(C.byref(h), self.n, _ptr(rp), _ptr(ci), _ptr(vv), k, Fp, _ptr(pp),
                                            int(n_parts), int(overlap), _ptr(p0), int(n_parts0), C.byref(opt)))
        self._h = h
        self.nnz = int(rp[-1])
        self.k = k

    @classmethod
    def from_problem(cls, P, **kw):
        """Build from a ``workloads.Problem``."""
        return cls(P.n, P.A.row_ptr, P.A.col_idx, P.A.val, P.F, P.part, P.n_parts, P.overlap, **kw)

    # -- device operations ------------------------------------------------

    def solve(self, f: torch.Tensor, u: Optional[torch.Tensor] = None, raise_on_error: bool = True):
        if u is None:
            u = torch.empty_like(f)
        info = Info()
        rc = self._lib.ddg_solve(self._h, _dev(f, self.n, "f"), _dev(u, self.n, "u"), C.byref(info))
        if rc != 0 and raise_on_error:
            check(rc)
        return u, info.as_dict()

    def apply_precond(self, r: torch.Tensor, z: Optional[torch.Tensor] = None) -> torch.Tensor:
        z = torch.empty_like(r) if z is None else z
        check(self._lib.ddg_apply_precond(self._h, _dev(r, self.n, "r"), _dev(z, self.n, "z")))
        return z

    def apply_stages(self, r: torch.Tensor, stages: int, e: Optional[torch.Tensor] = None) -> torch.Tensor:
        e = torch.empty_like(r) if e is None else e
        check(self._lib.ddg_apply_precond_stages(self._h, _dev(r, self.n, "r"), _dev(e, self.n, "e"), int(stages)))
        return e

    def spmv(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        y = torch.empty_like(x) if y is None else y
        check(self._lib.ddg_spmv(self._h, _dev(x, self.n, "x"), _dev(y, self.n, "y")))
        return y

    def refactor(self, val: torch.Tensor):
        check(self._lib.ddg_refactor(self._h, _dev(val, self.nnz, "val")))

    # -- host queries -------------------------------------------------------

    def info(self) -> dict:
        info = Info()
        check(self._lib.ddg_get_info(self._h, C.byref(info)))
        return info.as_dict()

    def cg_history(self, system: int = 0):
        """(alpha, beta, rel_res) of the last solve (numpy float64 arrays)."""
        cap = self.max_iter + 1
        a, b, r = (np.zeros(cap) for _ in range(3))
        cnt = C.c_int32()
        check(self._lib.ddg_cg_history(self._h, int(system), _ptr(a), _ptr(b), _ptr(r), cap, C.byref(cnt)))
        it = cnt.value
        return a[:it], b[:max(it - 1, 0)], r[:it + 1]

    def cg_report(self, system: int = 0) -> dict:
        """Fractional iteration count, Lanczos extremes, condition estimate and CG bound of the last solve."""
        rep = CgReport()
        check(self._lib.ddg_cg_report_get(self._h, int(system), C.byref(rep)))
        return rep.as_dict()

    def export(self, what: int) -> np.ndarray:
        need = C.c_int64()
        check(self._lib.ddg_export(self._h, what, None, 0, C.byref(need)))
        dtype = {_lib.EXPORT_COLOURS: np.int32, _lib.EXPORT_SET_PTR: np.int64, _lib.EXPORT_SET_IDX: np.int32,
                 _lib.EXPORT_KCOUNTS: np.int32, _lib.EXPORT_A0: np.float64, _lib.EXPORT_Q: np.float64,
                 _lib.EXPORT_BLOCKS: np.int32}[what]
        out = np.empty(need.value // np.dtype(dtype).itemsize, dtype=dtype)
        check(self._lib.ddg_export(self._h, what, _ptr(out), need.value, None))
        return out

    def colours(self) -> np.ndarray:
        return self.export(_lib.EXPORT_COLOURS)

    def sets(self):
        ptr = self.export(_lib.EXPORT_SET_PTR)
        idx = self.export(_lib.EXPORT_SET_IDX)
        return [idx[ptr[i]:ptr[i + 1]] for i in range(len(ptr) - 1)]

    def kcounts(self) -> np.ndarray:
        return self.export(_lib.EXPORT_KCOUNTS)

    def A0(self) -> np.ndarray:
        a = self.export(_lib.EXPORT_A0)
        m = int(round(np.sqrt(a.size)))
        return a.reshape(m, m)

    def Q(self) -> np.ndarray:
        return self.export(_lib.EXPORT_Q).reshape(self.n, -1)

    def blocks(self) -> np.ndarray:
        return self.export(_lib.EXPORT_BLOCKS).reshape(-1, 3)

    def profile_enable(self, on: bool = True):
        check(self._lib.ddg_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, reset: bool = True):
        ims, ila = C.c_double(), C.c_int64()
        check(self._lib.ddg_profile_read_idle(self._h, C.byref(ims), C.byref(ila)))
        ms, la, by = C.c_double(), C.c_int64(), C.c_int64()
        check(self._lib.ddg_profile_read(self._h, C.byref(ms), C.byref(la), C.byref(by), 1 if reset else 0))
        return {"ms": ms.value, "launches": la.value, "bytes": by.value, "idle_ms": ims.value,
                "idle_launches": ila.value}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ddg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_array(problems):
    """ctypes array of ddg_problem plus the host arrays it points into (keep them alive)."""
    keep = []
    arr = (Problem * len(problems))()
    for b, (rp, ci, vv, F, pp, nparts) in enumerate(problems):
        rp = np.ascontiguousarray(rp, dtype=np.int64)
        ci = np.ascontiguousarray(ci, dtype=np.int32)
        vv = np.ascontiguousarray(vv, dtype=np.float64)
        pp = np.ascontiguousarray(pp, dtype=np.int32)
        Fh = np.asfortranarray(F, dtype=np.float64) if F is not None and F.size else None
        n = rp.shape[0] - 1
        if ci.shape[0] != rp[-1] or vv.shape[0] != rp[-1] or pp.shape[0] != n:
            raise ValueError(f"system {b}: inconsistent array lengths")
        if Fh is not None and Fh.shape[0] != n:
            raise ValueError(f"system {b}: F must have n rows")
        keep += [rp, ci, vv, pp, Fh]
        arr[b].n = n
        arr[b].row_ptr = rp.ctypes.data
        arr[b].col_idx = ci.ctypes.data
        arr[b].val = vv.ctypes.data
        arr[b].k = 0 if Fh is None else Fh.shape[1]
        arr[b].F = None if Fh is None else Fh.ctypes.data
        arr[b].part = pp.ctypes.data
        arr[b].n_parts = int(nparts)
    return arr, keep


def tune_batched(problems, overlap: int, precision: str = "fp64", max_sample: int = 8,
                 cache: Optional[str] = None, stream: Optional[torch.cuda.Stream] = None):
    """Pick (tile, block_target) for a batch with the library's autotuner.

    Returns (tile, block_target, candidates) where candidates lists the
    measured (tile, block_target, precond_ms, factor_bytes) -- empty on a
    cache hit.
    """
    lib = _lib.load()
    arr, keep = _problem_array(problems)
    stream = stream if stream is not None else torch.cuda.current_stream()
    base = _options(lib, precision, 1e-8, 1000, 1e-10, 0, 0, 4, stream)
    best = Options()
    rep = (TuneEntry * 16)()
    nrep = C.c_int32()
    path = cache.encode() if cache else None
    check(lib.ddg_tune_batched(len(problems), arr, int(overlap), C.byref(base), int(max_sample), path,
                               C.byref(best), rep, 16, C.byref(nrep)))
    del keep
    cands = [(rep[i].tile, rep[i].block_target, rep[i].precond_ms, rep[i].factor_bytes) for i in range(nrep.value)]
    return best.tile, best.block_target, cands


class DDGBatchSolver(DDGSolver):
    """Many independent systems in one handle (``ddg_setup_batched``).

    ``problems`` is a sequence of (row_ptr, col_idx, val, F, part, n_parts)
    with host arrays; device vectors are the concatenation of the systems'
    vectors (``row_off`` gives the offsets).
    """

    def __init__(self, problems, overlap: int, precision: str = "fp64", rtol: float = 1e-8,
                 max_iter: int = 1000, rank_tol: float = 1e-10, tile: int = 0, block_target: int = 0,
                 check_every: int = 4, stream: Optional[torch.cuda.Stream] = None, schedule: str = "auto",
                 cg_variant: str = "fr", matrix_format: str = "auto", coarse_solver: str = "inverse",
                 ic_tol: float = 1e-6, ic_maxit: int = 200):
        lib = _lib.load()
        self._lib = lib
        self.max_iter = int(max_iter)
        arr, keep = _problem_array(problems)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opt = _options(lib, precision, rtol, max_iter, rank_tol, tile, block_target, check_every, self.stream,
                       schedule, cg_variant, matrix_format, coarse_solver=coarse_solver, ic_tol=ic_tol,
                       ic_maxit=ic_maxit)
        self.precision = precision
        h = C.c_void_p()
        check(lib.ddg_setup_batched(C.byref(h), len(problems), arr, int(overlap), C.byref(opt)))
        del keep
        self._h = h
        nb = C.c_int32()
        check(lib.ddg_batch_layout(h, C.byref(nb), None, None))
        self.nb = nb.value
        self.row_off = np.zeros(self.nb + 1, dtype=np.int64)
        self.sub_off = np.zeros(self.nb + 1, dtype=np.int32)
        check(lib.ddg_batch_layout(h, None, _ptr(self.row_off), _ptr(self.sub_off)))
        self.n = int(self.row_off[-1])
        self.nnz = int(sum(int(np.asarray(p[0])[-1]) for p in problems))
        self.k = max((0 if p[3] is None else np.asarray(p[3]).shape[1]) for p in problems)

    def solve(self, f: torch.Tensor, u: Optional[torch.Tensor] = None, raise_on_error: bool = True):
        """Solve all systems; returns (u, [info per system])."""
        if u is None:
            u = torch.empty_like(f)
        infos = (Info * self.nb)()
        rc = self._lib.ddg_solve_batched(self._h, _dev(f, self.n, "f"), _dev(u, self.n, "u"), infos)
        if rc != 0 and raise_on_error:
            check(rc)
        return u, [i.as_dict() for i in infos]

    def split(self, x: torch.Tensor):
        return [x[self.row_off[b]:self.row_off[b + 1]] for b in range(self.nb)]


def stencil_assemble(dims, theta: torch.Tensor, val: torch.Tensor, stream=None, bc: str = "dirichlet"):
    """CSR values of the cell-centred harmonic-mean operator for kappa = exp(theta)."""
    lib = _lib.load()
    d = (C.c_int32 * 3)(*[int(x) for x in dims])
    s = (stream or torch.cuda.current_stream()).cuda_stream
    n = int(np.prod(dims))
    check(lib.ddg_stencil_assemble(d, _dev(theta, n, "theta"), _lib.BC[bc], val.data_ptr(), C.c_void_p(s)))
    return val


def stencil_coeff_grad(dims, theta, u, lam, grad=None, stream=None, bc: str = "dirichlet"):
    """Per-cell dL/dtheta = -kappa lam^T (dA/dkappa) u."""
    lib = _lib.load()
    n = int(np.prod(dims))
    grad = torch.empty_like(theta) if grad is None else grad
    d = (C.c_int32 * 3)(*[int(x) for x in dims])
    s = (stream or torch.cuda.current_stream()).cuda_stream
    check(lib.ddg_stencil_coeff_grad(d, _dev(theta, n, "theta"), _dev(u, n, "u"), _dev(lam, n, "lam"),
                                     _lib.BC[bc], _dev(grad, n, "grad"), C.c_void_p(s)))
    return grad
