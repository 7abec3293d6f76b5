"""ctypes binding of ``libcoarse.so`` (the C ABI declared in include/coarse.h).

Argument marshalling only. Loading fails loudly when the library is missing:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoarse.so")

CG_OK = 0
CG_NOT_CONVERGED = 1
CG_INVALID_ARG = -1
CG_UNSUPPORTED = -2
CG_HIP_ERROR = -3
CG_BREAKDOWN = -4
CG_NONFINITE = -5
CG_WORKSPACE_TOO_SMALL = -6

C64, C128, BF16, FP16, C64_3M = 0, 1, 2, 3, 4
LINK_DTYPES = {"c64": C64, "bf16": BF16, "fp16": FP16, "c64_3m": C64_3M}

EXPORTED = [
    "coarse_packed_bytes", "coarse_pack_links", "coarse_apply", "coarse_apply_adjoint", "coarse_link_grad",
    "coarse_bcg_workspace_bytes", "coarse_bcg_solve", "coarse_batched_workspace_bytes", "coarse_apply_batched",
    "cg_status_string", "cg_last_error",
]


class CoarseGeom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("nbasis", ctypes.c_int32), ("npoint", ctypes.c_int32),
                ("offsets", ctypes.POINTER(ctypes.c_int8))]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("max_inner", ctypes.c_int32), ("check_every", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("outer_dtype", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cycles", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("relres_max", ctypes.c_double), ("relres", ctypes.c_double * 32),
                ("seconds_total", ctypes.c_double), ("seconds_inner", ctypes.c_double),
                ("seconds_outer", ctypes.c_double)]


class ChebPrec(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double), ("order", ctypes.c_int32)]


class CoarseSystem(ctypes.Structure):
    _fields_ = [("geom", CoarseGeom), ("nrhs", ctypes.c_int32), ("packed", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class CoarseSolveSystem(ctypes.Structure):
    _fields_ = [("geom", CoarseGeom), ("nrhs", ctypes.c_int32), ("packed_outer", ctypes.c_void_p),
                ("packed_inner", ctypes.c_void_p), ("inner_dtype", ctypes.c_int32), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p)]


class CoarseError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2409_03904_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    G = ctypes.POINTER(CoarseGeom)
    lib.coarse_packed_bytes.argtypes = [G, i32, ctypes.POINTER(sz)]
    lib.coarse_pack_links.argtypes = [G, vp, i32, vp, vp]
    lib.coarse_apply.argtypes = [G, vp, i32, vp, vp, i32, i32, vp]
    lib.coarse_apply_adjoint.argtypes = [G, vp, i32, vp, vp, i32, i32, vp]
    lib.coarse_apply_generic.argtypes = [G, vp, i32, vp, vp, i32, i32, vp]
    lib.coarse_apply_adjoint_generic.argtypes = [G, vp, i32, vp, vp, i32, i32, vp]
    lib.coarse_link_grad.argtypes = [G, vp, vp, vp, ctypes.c_float, i32, i32, vp]
    lib.coarse_bcg_workspace_bytes.argtypes = [G, i32, ctypes.POINTER(SolveParams), ctypes.POINTER(sz)]
    lib.coarse_bcg_solve.argtypes = [G, vp, vp, i32, vp, vp, i32, ctypes.POINTER(SolveParams),
                                     ctypes.POINTER(SolveStats), vp, sz, vp]
    lib.coarse_batched_workspace_bytes.argtypes = [ctypes.POINTER(CoarseSystem), i32, ctypes.POINTER(sz)]
    lib.coarse_apply_batched.argtypes = [ctypes.POINTER(CoarseSystem), i32, vp, sz, vp]
    lib.coarse_batched_set_occupancy.argtypes = [i32]
    lib.coarse_tune_apply.argtypes = [G, vp, i32, vp, vp, i32, i32, i32, vp, ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.c_float)]
    lib.coarse_set_apply_variant.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.coarse_apply_variant_count.argtypes = [i32]
    lib.coarse_apply_workspace_bytes.argtypes = [G, i32, i32, ctypes.POINTER(sz)]
    SS = ctypes.POINTER(CoarseSolveSystem)
    lib.coarse_bcg_batched_workspace_bytes.argtypes = [SS, i32, ctypes.POINTER(SolveParams), ctypes.POINTER(sz)]
    lib.coarse_bcg_solve_batched.argtypes = [SS, i32, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveStats), vp,
                                             sz, vp]
    lib.coarse_apply_ws.argtypes = [G, vp, i32, vp, vp, i32, i32, vp, sz, vp]
    lib.coarse_apply_noalloc.argtypes = [G, vp, i32, vp, vp, i32, i32, vp]
    lib.coarse_apply_gram_workspace_bytes.argtypes = [G, i32, i32, ctypes.POINTER(sz)]
    lib.coarse_apply_gram.argtypes = [G, vp, i32, vp, vp, i32, vp, vp, sz, vp]
    dbl = ctypes.c_double
    lib.coarse_chebyshev_coefficients.argtypes = [dbl, dbl, i32, ctypes.POINTER(dbl)]
    lib.coarse_chebyshev_workspace_bytes.argtypes = [G, i32, i32, ctypes.POINTER(sz)]
    lib.coarse_chebyshev_apply.argtypes = [G, vp, i32, vp, vp, i32, dbl, dbl, i32, vp, sz, vp]
    lib.coarse_deflation_workspace_bytes.argtypes = [G, i32, i32, ctypes.POINTER(sz)]
    lib.coarse_deflate.argtypes = [G, vp, i32, vp, vp, vp, vp, i32, vp, sz, vp]
    lib.coarse_deflated_chebyshev_workspace_bytes.argtypes = [G, i32, i32, i32, ctypes.POINTER(sz)]
    lib.coarse_deflated_chebyshev_apply.argtypes = [G, vp, i32, vp, i32, vp, vp, vp, i32, dbl, dbl, i32, vp, sz, vp]
    lib.coarse_block_lanczos_workspace_bytes.argtypes = [G, i32, i32, i32, i32, ctypes.POINTER(sz)]
    lib.coarse_block_lanczos.argtypes = [G, vp, i32, vp, i32, i32, i32, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                         ctypes.POINTER(i32), vp, sz, vp]
    lib.coarse_adjoint_links.argtypes = [G, vp, vp, vp]
    lib.coarse_hermitian_eigh.argtypes = [i32, vp, vp, vp]
    lib.coarse_block_project.argtypes = [G, i32, vp, vp, vp, i32, vp]
    lib.coarse_block_promote.argtypes = [G, i32, vp, vp, vp, i32, vp]
    lib.coarse_pbcg_workspace_bytes.argtypes = [G, i32, ctypes.POINTER(SolveParams), ctypes.POINTER(ChebPrec),
                                                ctypes.POINTER(sz)]
    lib.coarse_pbcg_solve.argtypes = [G, vp, vp, i32, vp, vp, i32, ctypes.POINTER(SolveParams),
                                      ctypes.POINTER(ChebPrec), ctypes.POINTER(SolveStats), vp, sz, vp]
    for name in ["coarse_packed_bytes", "coarse_pack_links", "coarse_apply", "coarse_apply_adjoint",
                 "coarse_apply_generic", "coarse_apply_adjoint_generic", "coarse_link_grad", "coarse_bcg_workspace_bytes", "coarse_bcg_solve",
                 "coarse_batched_workspace_bytes", "coarse_apply_batched", "coarse_batched_set_occupancy",
                 "coarse_tune_apply", "coarse_set_apply_variant", "coarse_apply_variant_count",
                 "coarse_apply_workspace_bytes", "coarse_apply_ws", "coarse_apply_noalloc",
                 "coarse_apply_gram_workspace_bytes", "coarse_apply_gram",
                 "coarse_bcg_batched_workspace_bytes",
                 "coarse_bcg_solve_batched", "coarse_chebyshev_coefficients", "coarse_chebyshev_workspace_bytes",
                 "coarse_chebyshev_apply", "coarse_pbcg_workspace_bytes", "coarse_pbcg_solve",
                 "coarse_deflation_workspace_bytes", "coarse_deflate", "coarse_deflated_chebyshev_workspace_bytes",
                 "coarse_deflated_chebyshev_apply", "coarse_block_project", "coarse_block_promote",
                 "coarse_block_lanczos_workspace_bytes", "coarse_block_lanczos", "coarse_adjoint_links",
                 "coarse_hermitian_eigh"]:
        getattr(lib, name).restype = i32
    lib.cg_status_string.argtypes = [i32]
    lib.cg_status_string.restype = ctypes.c_char_p
    lib.cg_last_error.argtypes = []
    lib.cg_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(code: int, allow=(CG_OK,)) -> int:
    if code in allow:
        return code
    lib = load()
    msg = lib.cg_last_error().decode() or lib.cg_status_string(code).decode()
    raise CoarseError(code, msg)
