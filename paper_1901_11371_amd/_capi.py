"""ctypes declarations of the hbf C ABI (include/hbf.h).  Argument
marshalling only; every computation happens in the shared library."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libhbf.so")

HBF_OK, HBF_NOCONV, HBF_EINVAL, HBF_ENOMEM, HBF_EHIP, HBF_ESINGULAR, HBF_ESTATE = 0, 1, -1, -2, -3, -4, -5
HBF_C64, HBF_C128 = 0, 1
HBF_PREC_BLOCK_LU, HBF_PREC_PAPER_TRI, HBF_PREC_NONE = 0, 1, 2
HBF_GMRES, HBF_TFQMR = 0, 1


class Curve(C.Structure):
    _fields_ = [("ncurves", C.c_int32), ("node_off", C.POINTER(C.c_int64)), ("xy", C.POINTER(C.c_double))]


class BuildOpts(C.Structure):
    _fields_ = [("dtype", C.c_int), ("prec", C.c_int), ("eta0", C.c_double), ("z", C.POINTER(C.c_double)),
                ("max_nrhs", C.c_int32), ("restart", C.c_int32), ("device", C.c_int32), ("nthreads", C.c_int32),
                ("cache_plan", C.c_int32), ("superleaf", C.c_int32), ("verbose", C.c_int32),
                ("host_entries", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iters", C.c_int32),
                ("max_refine", C.c_int32), ("mixed", C.c_int32), ("x0_given", C.c_int32),
                ("inner_tol", C.c_double), ("method", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refinements", C.c_int32), ("converged", C.c_int32),
                ("relres", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("leaf", C.c_int64), ("levels", C.c_int64), ("n_blocks", C.c_int64),
                ("n_units", C.c_int64), ("max_rank", C.c_int32), ("mean_rank", C.c_double),
                ("bytes_butterfly", C.c_int64), ("bytes_dense", C.c_int64), ("bytes_index", C.c_int64),
                ("bytes_precond", C.c_int64), ("bytes_workspace", C.c_int64), ("build_seconds", C.c_double),
                ("scale_re", C.c_double), ("scale_im", C.c_double), ("apply_bytes_matvec", C.c_int64),
                ("apply_bytes_precond", C.c_int64), ("launches_matvec", C.c_int64),
                ("arena_rows", C.c_int64), ("launches_precond", C.c_int64), ("steps_precond", C.c_int64),
                ("n_internal", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes)
SIGNATURES = {
    "hbf_build": (C.c_int, [C.POINTER(Curve), C.c_double, C.c_int32, C.c_double, C.POINTER(BuildOpts),
                            C.POINTER(C.c_void_p)]),
    "hbf_set_impedance": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "hbf_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int, C.c_int32, C.c_void_p]),
    "hbf_matvec_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int, C.c_int32,
                                     C.c_void_p]),
    "hbf_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int, C.c_int32,
                                    C.c_void_p]),
    "hbf_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int, C.POINTER(SolveOpts),
                            C.POINTER(SolveInfo), C.c_void_p]),
    "hbf_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int,
                                    C.POINTER(SolveOpts), C.POINTER(SolveInfo), C.c_void_p]),
    "hbf_impedance_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int, C.c_void_p,
                                     C.c_void_p]),
    "hbf_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "hbf_tune": (C.c_int, [C.c_void_p, C.c_char_p, C.c_int64]),
    "hbf_size": (C.c_int64, [C.c_void_p]),
    "hbf_free": (None, [C.c_void_p]),
    "hbf_last_error": (C.c_char_p, []),
    "hbf_plan_build": (C.c_int, [C.POINTER(Curve), C.c_double, C.c_int32, C.c_double, C.POINTER(BuildOpts),
                                 C.POINTER(C.c_void_p)]),
    "hbf_plan_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "hbf_plan_precond": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "hbf_plan_entries": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int64, C.POINTER(C.c_int64),
                                   C.c_int64, C.c_void_p]),
    "hbf_plan_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "hbf_plan_free": (None, [C.c_void_p]),
    "hbf_hankel2_0": (None, [C.c_void_p, C.c_int64, C.c_void_p]),
}

_lib = None


def load(path: str | None = None):
    """Load the shared library (raises if it was not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"hbf native library not built: {p} (run __graft_entry__.build())")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name, None)
        if f is None:
            if path is None:
                raise RuntimeError(f"hbf native library lacks symbol {name}")
            continue
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


class HbfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hbf status {status}: {msg}")
        self.status = status


def check(lib, status):
    if status < 0:
        raise HbfError(status, lib.hbf_last_error().decode())
    return status
