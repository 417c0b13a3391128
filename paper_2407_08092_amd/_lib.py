"""ctypes loader of libddq.so (the HIP library declared in include/ddq.h).

There is no fallback: if the library is missing or cannot be loaded, importing
the binding raises.  ``ensure_built()`` compiles it in-tree when it is absent.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# DDQ_LIBRARY selects an alternative build of the same library (tuning runs)
LIB_PATH = os.environ.get("DDQ_LIBRARY") or os.path.join(PKG, "libddq.so")

DDQ_F64, DDQ_F32, DDQ_F16, DDQ_BF16 = 0, 1, 2, 3
DDQ_STORE_F64, DDQ_STORE_F32, DDQ_STORE_F32_LINK12, DDQ_STORE_F16, DDQ_STORE_BF16 = 1, 2, 4, 8, 16
DDQ_RESERVE_SOLVE, DDQ_RESERVE_FULL, DDQ_RESERVE_SAP, DDQ_RESERVE_FORCE = 1, 2, 4, 8
STATUS = {
    0: "DDQ_OK", 1: "DDQ_NOT_CONVERGED", -1: "DDQ_ERR_ARG", -2: "DDQ_ERR_STATE", -3: "DDQ_ERR_HIP",
    -4: "DDQ_ERR_OOM", -5: "DDQ_ERR_NOT_PD", -6: "DDQ_ERR_NONFINITE",
}


class DDQError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        self.status = status
        super().__init__(f"{fn} returned {STATUS.get(status, status)}: {msg}")


class GmresParams(C.Structure):
    _fields_ = [("m", C.c_int), ("max_cycles", C.c_int), ("tol", C.c_double), ("inner_prec", C.c_int),
                ("smoother_sweeps", C.c_int), ("omega", C.c_double), ("inner_reduction", C.c_double),
                ("smoother_prec", C.c_int), ("orth_passes", C.c_int), ("cycle_graph", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("cycles", C.c_int), ("iters", C.c_int), ("applies_f64", C.c_int), ("applies_lo", C.c_int),
                ("true_relres", C.c_double), ("t_total_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MrTile(C.Structure):
    _fields_ = [("nb", C.c_int), ("waves", C.c_int), ("xcd_map", C.c_int), ("ms", C.c_double),
                ("passes", C.c_int), ("lds_kb", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStats(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int), ("total_ms", C.c_double),
                ("bytes_per_launch", C.c_double)]


_P = C.c_void_p
_SIGNATURES = {
    "ddq_create_lattice": [C.POINTER(C.c_int), C.c_int, _P, C.POINTER(_P)],
    "ddq_destroy_lattice": [_P],
    "ddq_set_stream": [_P, _P],
    "ddq_lattice_size": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "ddq_set_gauge": [_P, _P, C.c_int, C.c_uint],
    "ddq_set_clover": [_P, C.c_double, C.c_double],
    "ddq_get_clover": [_P, _P, _P],
    "ddq_pack_parity": [_P, C.c_int, C.c_int, C.c_int, _P, _P],
    "ddq_unpack_parity": [_P, C.c_int, C.c_int, C.c_int, _P, _P],
    "ddq_convert_parity": [_P, C.c_int, C.c_int, _P, C.c_int, _P],
    "ddq_apply_schur": [_P, C.c_int, C.c_int, _P, _P, C.c_int],
    "ddq_apply_schur_noalloc": [_P, C.c_int, C.c_int, _P, _P, C.c_int],
    "ddq_set_h16_clover": [_P, C.c_int],
    "ddq_set_sweep_chunks": [_P, C.c_int],
    "ddq_mrhs_pack": [_P, C.c_int, _P, _P],
    "ddq_mrhs_unpack": [_P, C.c_int, _P, _P],
    "ddq_mrhs_apply_schur": [_P, C.c_int, _P, _P, C.c_int],
    "ddq_mrhs_richardson_smooth": [_P, C.c_int, _P, _P, C.c_int, C.c_double, C.c_int],
    "ddq_mrhs_set_launch": [_P, C.c_int, C.c_int, C.c_int, C.c_int],
    "ddq_richardson_smooth": [_P, C.c_int, C.c_int, _P, _P, C.c_int, C.c_double],
    "ddq_estimate_lambda_max": [_P, C.c_int, _P, C.POINTER(C.c_double)],
    "ddq_set_multi_rhs_tile": [_P, C.c_int, C.POINTER(MrTile)],
    "ddq_tune_multi_rhs": [_P, C.c_int, C.c_int, C.POINTER(MrTile), C.c_int, C.POINTER(C.c_int), C.POINTER(MrTile)],
    "ddq_oe_prepare": [_P, C.c_int, _P, _P],
    "ddq_oe_reconstruct": [_P, C.c_int, _P, _P, _P],
    "ddq_oe_gmres_solve": [_P, C.c_int, _P, _P, C.POINTER(GmresParams), C.POINTER(SolveInfo)],
    "ddq_reserve": [_P, C.c_int, C.c_int, C.c_uint],
    "ddq_autotune": [_P, C.c_char_p],
    "ddq_batch_reserve": [_P, C.c_int, C.c_int],
    "ddq_batch_create": [C.POINTER(_P), C.POINTER(C.c_int), C.c_int, _P, C.POINTER(_P)],
    "ddq_batch_solve": [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(GmresParams), C.POINTER(C.c_double),
                        C.POINTER(SolveInfo)],
    "ddq_batch_destroy": [_P],
    "ddq_backward_apply": [_P, C.c_int, C.c_int, _P, _P],
    "ddq_backward_link_force": [_P, _P, _P, _P, _P, C.c_int],
    "ddq_stream_copy": [_P, _P, C.c_int64, C.c_int, _P],
    "ddq_stencil_stream": [_P, C.c_int, C.c_int, _P, _P, _P, _P],
    "ddq_apply_dirac": [_P, C.c_int, _P, _P],
    "ddq_oe_smoother": [_P, C.c_int, _P, _P, C.c_int, C.c_double, C.c_int],
    "ddq_fgmres_solve": [_P, _P, _P, _P, _P],
    "ddq_sap_smooth": [_P, C.c_int, _P, _P, C.c_int, C.c_int],
    "ddq_fgmres_sap_solve": [_P, _P, _P, _P, C.c_int, C.c_int, _P],
    "ddq_coarse_packed_bytes": [C.POINTER(C.c_int), C.c_int, C.c_int, C.POINTER(C.c_int64)],
    "ddq_coarse_pack_blocks": [C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int, _P, _P, _P],
    "ddq_coarse_apply": [C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int, _P, _P, _P, C.c_int, C.c_int, _P],
    "ddq_profile_begin": [_P],
    "ddq_profile_end": [_P, C.POINTER(KernelStats), C.c_int, C.POINTER(C.c_int)],
    "ddq_last_error": [],
}

_lib = None


def ensure_built() -> str:
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    return LIB_PATH


def lib():
    """The loaded library (compiled first if absent)."""
    global _lib
    if _lib is None:
        ensure_built()
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_char_p if name == "ddq_last_error" else C.c_int
        _lib = L
    return _lib


def check(status: int, fn: str, allow=(0,)) -> int:
    if status in allow:
        return status
    msg = lib().ddq_last_error().decode(errors="replace")
    raise DDQError(status, fn, msg)
