"""ctypes declarations of libddg.so (the C ABI in include/ddg.h).

The library is loaded from this package directory.  There is no fallback:
if the shared library is missing or fails to load, every entry point raises.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddg.so")

DDG_OK = 0
STATUS = {
    0: "OK", -1: "INVALID_ARG", -2: "NOT_SPD", -3: "RANK", -4: "BREAKDOWN",
    -5: "NO_CONVERGENCE", -6: "HIP", -7: "OOM", -8: "UNSUPPORTED",
}
PRECISION = {"fp64": 0, "fp32": 1, "mixed": 1, "bf16": 2}

EXPORT_COLOURS, EXPORT_SET_PTR, EXPORT_SET_IDX, EXPORT_KCOUNTS, EXPORT_A0, EXPORT_Q, EXPORT_BLOCKS = range(7)


SCHEDULE = {"auto": 0, "colours": 1, "queue": 2, "persistent": 3}
BC = {"dirichlet": 0, "x0": 1}
CG_VARIANT = {"fr": 0, "pr": 1}
MATRIX_FORMAT = {"auto": 0, "csr": 1}
LOCAL_SOLVER = {"exact": 0, "ssor": 1}
COARSE_SOLVER = {"inverse": 0, "ic_cg": 1}
MATRIX_FORMAT_NAME = {1: "csr", 2: "dia"}


class Options(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("max_iter", C.c_int32), ("rtol", C.c_double),
        ("rank_tol", C.c_double), ("tile", C.c_int32), ("block_target", C.c_int32),
        ("check_every", C.c_int32), ("schedule", C.c_int32), ("cg_variant", C.c_int32),
        ("stream", C.c_void_p), ("matrix_format", C.c_int32), ("local_solver", C.c_int32),
        ("ssor_omega", C.c_double), ("ssor_sweeps", C.c_int32), ("coarse_solver", C.c_int32),
        ("ic_tol", C.c_double), ("ic_maxit", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iters", C.c_int32), ("rel_res", C.c_double),
        ("true_rel_res", C.c_double), ("n_coarse", C.c_int32), ("n_colours", C.c_int32),
        ("n_parts", C.c_int32), ("n_blocks", C.c_int32), ("setup_ms", C.c_double),
        ("solve_ms", C.c_double), ("factor_bytes", C.c_int64), ("coarse_bytes", C.c_int64),
        ("sweep_bytes", C.c_int64), ("iter_bytes", C.c_int64), ("tile", C.c_int32), ("schedule", C.c_int32),
        ("envelope_elems", C.c_int64), ("set_rows", C.c_int64), ("nbhd_rows", C.c_int64),
        ("matrix_format", C.c_int32), ("levels", C.c_int32), ("n_coarsest", C.c_int32),
        ("coarse_refine", C.c_int32), ("coarse_inverse_err", C.c_double), ("coarse_solver", C.c_int32),
        ("coarse_iters", C.c_int32), ("sweep_groups", C.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class CgReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("iter_bound", C.c_int32), ("frac_iters", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("kappa", C.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
        ("k", C.c_int32), ("F", C.c_void_p), ("part", C.c_void_p), ("n_parts", C.c_int32),
    ]


class TuneEntry(C.Structure):
    _fields_ = [("tile", C.c_int32), ("block_target", C.c_int32), ("precond_ms", C.c_double),
                ("factor_bytes", C.c_int64)]


class DDGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("ddg_default_options", None, [C.POINTER(Options)]),
    ("ddg_setup", C.c_int, [C.POINTER(C.c_void_p), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Options)]),
    ("ddg_setup_three_level", C.c_int, [C.POINTER(C.c_void_p), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                        C.c_int32, C.POINTER(Options)]),
    ("ddg_refactor", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ddg_solve", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Info)]),
    ("ddg_setup_batched", C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Problem), C.c_int32,
                                    C.POINTER(Options)]),
    ("ddg_solve_batched", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Info)]),
    ("ddg_tune_batched", C.c_int, [C.c_int32, C.POINTER(Problem), C.c_int32, C.POINTER(Options), C.c_int32,
                                   C.c_char_p, C.POINTER(Options), C.POINTER(TuneEntry), C.c_int32,
                                   C.POINTER(C.c_int32)]),
    ("ddg_batch_layout", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p, C.c_void_p]),
    ("ddg_apply_precond", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ddg_apply_precond_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ddg_apply_precond_stages", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("ddg_spmv", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ddg_get_info", C.c_int, [C.c_void_p, C.POINTER(Info)]),
    ("ddg_cg_history", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.POINTER(C.c_int32)]),
    ("ddg_cg_report_get", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(CgReport)]),
    ("ddg_export", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    ("ddg_profile_enable", C.c_int, [C.c_void_p, C.c_int32]),
    ("ddg_profile_read", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.c_int32]),
    ("ddg_profile_read_idle", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("ddg_analyze", C.c_int, [C.POINTER(C.c_void_p), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_int32, C.c_int32, C.POINTER(Options)]),
    ("ddg_destroy", None, [C.c_void_p]),
    ("ddg_last_error", C.c_char_p, []),
    ("ddg_stencil_assemble", C.c_int, [C.POINTER(C.c_int32), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    ("ddg_stencil_coeff_grad", C.c_int, [C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_int32, C.c_void_p, C.c_void_p]),
]

SYMBOLS = [s[0] for s in _SIGS]


def load(path: str = LIB_PATH):
    """Load libddg.so once; raise if it is absent (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libddg.so not found at {path}; build it with "
                           "`python -m paper_1504_00907_amd.build` (there is no fallback path)")
    lib = C.CDLL(path)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != DDG_OK:
        msg = load().ddg_last_error()
        raise DDGError(rc, msg.decode() if msg else "")
