"""ctypes loader for libeofa.so (the C ABI declared in include/eofa.h).

The library must have been built in-tree (``__graft_entry__.build()`` or
``python paper_1611_00298_amd/build.py``).  There is no fallback: a missing
library raises at first use.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.environ.get("EOFA_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libeofa.so")

EOFA_OK, EOFA_EINVAL, EOFA_ENOMEM, EOFA_ENOCONV, EOFA_ENAN, EOFA_EDEVICE = 0, -1, -2, -3, -4, -5
PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}

EXPORTS = [
    "eofa_ctx_create", "eofa_ctx_destroy", "eofa_ctx_update_gauge", "dwf_apply", "eofa_solve", "eofa_solve_dense",
    "eofa_force", "eofa_md_update", "eofa_md_update_noalloc", "eofa_rational_inv_sqrt", "eofa_heatbath", "eofa_meofa_bounds", "eofa_chrono",
    "eofa_gauge_action", "eofa_gauge_force", "eofa_timing_enable",
    "eofa_timing_query", "eofa_last_error",
]


class Geom(C.Structure):
    _fields_ = [("L", C.c_int * 4), ("Ls", C.c_int), ("M5", C.c_double), ("alpha", C.c_double),
                ("antiperiodic_t", C.c_int)]


class Solver(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("inner", C.c_int),
                ("reliable_delta", C.c_double), ("fused_fp64", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int * 2), ("reliable_updates", C.c_int * 2),
                ("true_resid", C.c_double * 2), ("seconds", C.c_double), ("flops", C.c_double),
                ("inner_used", C.c_int * 2)]

    def as_dict(self):
        names = {v: k for k, v in PREC.items()}
        return {"iters": list(self.iters), "reliable_updates": list(self.reliable_updates),
                "true_resid": list(self.true_resid), "seconds": self.seconds, "flops": self.flops,
                "inner_used": [names.get(v, str(v)) for v in self.inner_used]}


class EOFAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P, D, I_ = C.c_void_p, C.c_double, C.c_int
    sigs = {
        "eofa_ctx_create": (I_, [C.POINTER(C.c_void_p), C.POINTER(Geom), P, P]),
        "eofa_ctx_destroy": (None, [P]),
        "eofa_ctx_update_gauge": (I_, [P, P]),
        "dwf_apply": (I_, [P, D, D, I_, I_, I_, P, P]),
        "eofa_solve": (I_, [P, D, D, P, P, P, P, P, P, C.POINTER(C.c_double), C.POINTER(Solver),
                            C.POINTER(Stats)]),
        "eofa_solve_dense": (I_, [P, D, D, P, P, P, P, C.POINTER(C.c_double), C.POINTER(Solver),
                                  C.POINTER(Stats)]),
        "eofa_force": (I_, [P, D, D, P, P, P, P, P, C.POINTER(Solver), C.POINTER(Stats)]),
        "eofa_md_update": (I_, [P, P, P, P, D, D, C.POINTER(C.c_double)]),
        "eofa_md_update_noalloc": (I_, [P, P, P, P, D, D, P]),
        "eofa_rational_inv_sqrt": (I_, [D, D, I_, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "eofa_heatbath": (I_, [P, D, D, P, I_, D, C.POINTER(C.c_double), C.POINTER(C.c_double), I_, P,
                               C.POINTER(Solver), C.POINTER(Stats)]),
        "eofa_chrono": (I_, [P, I_]),
        "eofa_meofa_bounds": (I_, [P, D, D, P, I_, C.POINTER(Solver), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(Stats)]),
        "eofa_gauge_action": (I_, [P, P, D, D, C.POINTER(C.c_double)]),
        "eofa_gauge_force": (I_, [P, P, D, D, P, I_]),
        "eofa_timing_enable": (I_, [P, I_]),
        "eofa_timing_query": (I_, [P, C.c_char_p, C.POINTER(C.c_long), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
        "eofa_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int, allow_noconv: bool = False) -> int:
    if rc == EOFA_OK or (allow_noconv and rc == EOFA_ENOCONV):
        return rc
    msg = load().eofa_last_error().decode()
    raise EOFAError(rc, msg or "eofa call failed")
