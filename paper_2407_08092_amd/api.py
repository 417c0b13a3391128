"""Python binding of the C ABI in include/ddq.h: same names, torch tensors for
device memory and streams, argument marshalling only.  Every step of the path
runs in the HIP library; nothing here computes.

Tensor layouts (see include/ddq.h):
  gauge links   complex128 [Lt, Lz, Ly, Lx, 4, 3, 3]
  full vector   complex128 / complex64 [Lt, Lz, Ly, Lx, 4, 3]   (or [nrhs, ...])
  parity vector complex128 [12, V/2] (or [nrhs, 12, V/2]);
                complex64 [6, V/2, 2] (or [nrhs, 6, V/2, 2]): rows 2k, 2k+1 paired per site;
                float16 / bfloat16 [3, V/2, 4, 2] (or [nrhs, ...]): rows 4k..4k+3 per
                site, (re, im) in the last axis (16-bit storage, FP32 arithmetic)
The arithmetic of a call follows the dtype: complex128 -> FP64, complex64 -> FP32,
float16 / bfloat16 -> 16-bit storage with FP32 arithmetic.

Work space: the library allocates only in its set-up and reservation calls.  The
helpers below call ``reserve`` with what the call needs before making it (a no-op
once the lattice holds that much), so Python users need not; callers of the C ABI
reserve themselves.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import (DDQ_BF16, DDQ_F16, DDQ_F32, DDQ_F64, DDQ_RESERVE_FORCE, DDQ_RESERVE_FULL, DDQ_RESERVE_SAP,
                   DDQ_RESERVE_SOLVE, DDQ_STORE_BF16, DDQ_STORE_F16, DDQ_STORE_F32, DDQ_STORE_F32_LINK12,
                   DDQ_STORE_F64, DDQError, GmresParams, SolveInfo, check, lib)

__all__ = [
    "Lattice", "DDQError", "create_lattice", "destroy_lattice", "set_gauge", "set_clover", "get_clover",
    "pack_parity", "unpack_parity", "apply_schur", "richardson_smooth", "estimate_lambda_max",
    "oe_prepare", "oe_reconstruct", "oe_gmres_solve", "parity_vector", "profile_begin", "profile_end",
    "stream_copy", "stencil_stream", "apply_dirac", "oe_smoother", "sap_smooth", "fgmres_solve", "fgmres_sap_solve", "backward_apply", "backward_link_force", "convert_parity",
    "CoarseOperator",
    "Batch", "batch_create", "batch_reserve", "batch_solve", "batch_destroy", "set_multi_rhs_tile",
    "tune_multi_rhs", "autotune", "reserve", "DDQ_RESERVE_SOLVE", "DDQ_RESERVE_FULL", "DDQ_RESERVE_SAP",
    "DDQ_RESERVE_FORCE",
    "DDQ_F64", "DDQ_F32", "DDQ_F16", "DDQ_BF16",
]


_PREC_OF = {torch.complex128: DDQ_F64, torch.complex64: DDQ_F32, torch.float16: DDQ_F16, torch.bfloat16: DDQ_BF16}
_DTYPE_OF = {v: k for k, v in _PREC_OF.items()}


def _prec(t: torch.Tensor) -> int:
    if t.dtype not in _PREC_OF:
        raise TypeError(f"expected complex128, complex64, float16 or bfloat16, got {t.dtype}")
    return _PREC_OF[t.dtype]


def _dev(t: torch.Tensor, name: str) -> C.c_void_p:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class Lattice:
    """Handle of a ddq_lattice; owns nothing on the Python side but the handle."""

    def __init__(self, handle: C.c_void_p, dims, t_antiperiodic: bool, device: torch.device):
        self.handle = handle
        self.dims = tuple(dims)
        self.t_antiperiodic = t_antiperiodic
        self.device = device
        V, Vh = C.c_int64(), C.c_int64()
        check(lib().ddq_lattice_size(handle, C.byref(V), C.byref(Vh)), "ddq_lattice_size")
        self.V, self.Vh = V.value, Vh.value
        self._stream = None

    def sync_stream(self):
        """Enqueue the next calls on torch's current stream of the lattice's device."""
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            check(lib().ddq_set_stream(self.handle, C.c_void_p(s)), "ddq_set_stream")
            self._stream = s

    @property
    def full_shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx, 4, 3)

    def __del__(self):
        h = getattr(self, "handle", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None  # None at interpreter exit
        if h is not None and L is not None:
            try:
                L.ddq_destroy_lattice(h)
            except Exception:  # pragma: no cover
                pass
            self.handle = None


def create_lattice(dims, t_antiperiodic: bool = True, device=None) -> Lattice:
    dims = [int(d) for d in dims]
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    arr = (C.c_int * 4)(*dims)
    h = C.c_void_p()
    with torch.cuda.device(device):
        s = torch.cuda.current_stream(device).cuda_stream
        check(lib().ddq_create_lattice(arr, int(bool(t_antiperiodic)), C.c_void_p(s), C.byref(h)),
              "ddq_create_lattice")
    lat = Lattice(h, dims, t_antiperiodic, device)
    lat._stream = s
    return lat


def destroy_lattice(lat: Lattice) -> None:
    if lat.handle is not None:
        check(lib().ddq_destroy_lattice(lat.handle), "ddq_destroy_lattice")
        lat.handle = None


def set_gauge(lat: Lattice, U: torch.Tensor, store=(DDQ_F64, DDQ_F32), link12: bool = False) -> None:
    """Links U (complex128, canonical).  store: the precisions to keep (DDQ_F64 always,
    DDQ_F32, DDQ_F16, DDQ_BF16).  link12: keep the FP32 links as two rows (third
    rebuilt from unitarity in the kernels); 16-bit links are always 12-real."""
    if U.dtype != torch.complex128 or tuple(U.shape) != lat.full_shape[:4] + (4, 3, 3):
        raise ValueError(f"U must be complex128 of shape {lat.full_shape[:4] + (4, 3, 3)}")
    U = U.contiguous()
    flags = (DDQ_STORE_F64 if DDQ_F64 in store else 0) | (DDQ_STORE_F32 if DDQ_F32 in store else 0)
    flags |= (DDQ_STORE_F16 if DDQ_F16 in store else 0) | (DDQ_STORE_BF16 if DDQ_BF16 in store else 0)
    if link12:
        flags |= DDQ_STORE_F32_LINK12
    lat.sync_stream()
    check(lib().ddq_set_gauge(lat.handle, C.c_void_p(U.data_ptr()), int(U.is_cuda), flags), "ddq_set_gauge")
    if not U.is_cuda:
        torch.cuda.current_stream(lat.device).synchronize()


def reserve(lat: Lattice, max_nrhs: int = 1, max_m: int = 0, what: int = 0) -> None:
    """Work space for later calls (grown, never shrunk): max_nrhs right-hand sides,
    cycle length max_m, what = DDQ_RESERVE_* flags."""
    check(lib().ddq_reserve(lat.handle, int(max_nrhs), int(max_m), int(what)), "ddq_reserve")


def autotune(lat: Lattice, cache_json_path: str) -> None:
    """Load the cached multi-right-hand-side tiles of this lattice and device, then
    save the lattice's tiles (see ddq_autotune)."""
    check(lib().ddq_autotune(lat.handle, str(cache_json_path).encode()), "ddq_autotune")


def set_clover(lat: Lattice, c_sw: float, m0: float) -> None:
    lat.sync_stream()
    check(lib().ddq_set_clover(lat.handle, float(c_sw), float(m0)), "ddq_set_clover")


def get_clover(lat: Lattice):
    """(A_ee, A_oo^-1) as complex128 device tensors [V/2, 2, 6, 6]."""
    a = torch.empty((lat.Vh, 2, 6, 6), dtype=torch.complex128, device=lat.device)
    b = torch.empty_like(a)
    lat.sync_stream()
    check(lib().ddq_get_clover(lat.handle, _dev(a, "A_ee"), _dev(b, "A_oo_inv")), "ddq_get_clover")
    return a, b


def _parity_shape(lat, dtype):
    if dtype == torch.complex128:
        return (12, lat.Vh)
    if dtype == torch.complex64:
        return (6, lat.Vh, 2)
    return (3, lat.Vh, 4, 2)


def parity_vector(lat: Lattice, nrhs=None, dtype=torch.complex128) -> torch.Tensor:
    shape = _parity_shape(lat, dtype)
    if nrhs is not None:
        shape = (nrhs,) + shape
    return torch.empty(shape, dtype=dtype, device=lat.device)


def _nrhs_parity(lat, v):
    shp = _parity_shape(lat, v.dtype)
    if tuple(v.shape) == shp:
        return 1
    if v.dim() == len(shp) + 1 and tuple(v.shape[1:]) == shp:
        return v.shape[0]
    raise ValueError(f"{v.dtype} parity vector must be {shp} or [nrhs, *{shp}], got {tuple(v.shape)}")


def convert_parity(lat: Lattice, v: torch.Tensor, dtype) -> torch.Tensor:
    """Parity vector to another precision (and its layout) through the library."""
    n = _nrhs_parity(lat, v)
    out = parity_vector(lat, None if v.dim() == len(_parity_shape(lat, v.dtype)) else n, dtype)
    lat.sync_stream()
    check(lib().ddq_convert_parity(lat.handle, n, _prec(v), _dev(v, "src"), _prec(out), _dev(out, "dst")),
          "ddq_convert_parity")
    return out


def _nrhs_full(lat, f):
    if tuple(f.shape) == lat.full_shape:
        return 1
    if f.dim() == 7 and tuple(f.shape[1:]) == lat.full_shape:
        return f.shape[0]
    raise ValueError(f"full vector must be {lat.full_shape} or [nrhs, ...], got {tuple(f.shape)}")


def pack_parity(lat: Lattice, full: torch.Tensor, parity: int, out: torch.Tensor = None) -> torch.Tensor:
    n = _nrhs_full(lat, full)
    if out is None:
        out = parity_vector(lat, None if full.dim() == 6 else n, full.dtype)
    lat.sync_stream()
    check(lib().ddq_pack_parity(lat.handle, _prec(full), n, int(parity), _dev(full, "full"), _dev(out, "v")),
          "ddq_pack_parity")
    return out


def unpack_parity(lat: Lattice, v: torch.Tensor, parity: int, out: torch.Tensor = None) -> torch.Tensor:
    n = _nrhs_parity(lat, v)
    if out is None:
        shape = lat.full_shape if v.dim() == len(_parity_shape(lat, v.dtype)) else (n,) + lat.full_shape
        out = torch.zeros(shape, dtype=v.dtype, device=lat.device)
    lat.sync_stream()
    check(lib().ddq_unpack_parity(lat.handle, _prec(v), n, int(parity), _dev(v, "v"), _dev(out, "full")),
          "ddq_unpack_parity")
    return out


def apply_schur(lat: Lattice, x_e: torch.Tensor, y_e: torch.Tensor = None, dagger: bool = False) -> torch.Tensor:
    """y_e = D_S x_e (eq. 3), or D_S^H x_e with dagger."""
    n = _nrhs_parity(lat, x_e)
    if y_e is None:
        y_e = torch.empty_like(x_e)
    reserve(lat, n)
    lat.sync_stream()
    check(lib().ddq_apply_schur(lat.handle, _prec(x_e), n, _dev(x_e, "x_e"), _dev(y_e, "y_e"), int(bool(dagger))),
          "ddq_apply_schur")
    return y_e


def apply_schur_noalloc(lat: Lattice, x_e: torch.Tensor, y_e: torch.Tensor, dagger: bool = False) -> torch.Tensor:
    """y_e = D_S x_e (or D_S^H x_e) with the library's fixed work space: the call itself
    allocates nothing, so the caller passes y_e."""
    n = _nrhs_parity(lat, x_e)
    if y_e.dtype != x_e.dtype or y_e.shape != x_e.shape:
        raise ValueError("x_e and y_e must match in dtype and shape")
    lat.sync_stream()
    check(lib().ddq_apply_schur_noalloc(lat.handle, _prec(x_e), n, _dev(x_e, "x_e"), _dev(y_e, "y_e"),
                                        int(bool(dagger))), "ddq_apply_schur_noalloc")
    return y_e


def set_sweep_chunks(lat: Lattice, nc: int) -> None:
    """One-right-hand-side Richardson sweeps launched on nc ranges of t-slices."""
    check(lib().ddq_set_sweep_chunks(lat.handle, int(nc)), "ddq_set_sweep_chunks")


def set_h16_clover(lat: Lattice, fp32: bool) -> None:
    """The 16-bit stencil reads FP32 clover blocks (fp32) or their 16-bit copies."""
    check(lib().ddq_set_h16_clover(lat.handle, int(bool(fp32))), "ddq_set_h16_clover")


DDQ_ENGINE_VALU = 0
DDQ_ENGINE_MFMA = 1


def _mrhs_shape(lat: Lattice, nrhs: int):
    return (int(lat.Vh), 6, int(nrhs), 2)


def _nrhs_mrhs(lat: Lattice, v: torch.Tensor) -> int:
    if v.dtype != torch.complex64 or v.dim() != 4 or tuple(v.shape[:2]) != (lat.Vh, 6) or v.shape[3] != 2:
        raise ValueError(f"an mrhs vector is complex64 [V/2, 6, nrhs, 2], got {v.dtype} {tuple(v.shape)}")
    if not v.is_contiguous():
        raise ValueError("mrhs vectors must be contiguous")
    return int(v.shape[2])


def mrhs_vector(lat: Lattice, nrhs: int) -> torch.Tensor:
    """An uninitialised mrhs-layout vector of nrhs right-hand sides."""
    return torch.empty(_mrhs_shape(lat, nrhs), dtype=torch.complex64, device=lat.device)


def mrhs_pack(lat: Lattice, v: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    """FP32 parity vectors [nrhs, 6, V/2, 2] -> mrhs layout [V/2, 6, nrhs, 2]."""
    n = _nrhs_parity(lat, v)
    if v.dtype != torch.complex64:
        raise ValueError("mrhs vectors are FP32 (complex64)")
    if out is None:
        out = mrhs_vector(lat, n)
    lat.sync_stream()
    check(lib().ddq_mrhs_pack(lat.handle, n, _dev(v, "v"), _dev(out, "out")), "ddq_mrhs_pack")
    return out


def mrhs_unpack(lat: Lattice, v: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    """mrhs layout [V/2, 6, nrhs, 2] -> FP32 parity vectors [nrhs, 6, V/2, 2]."""
    n = _nrhs_mrhs(lat, v)
    if out is None:
        out = torch.empty((n,) + _parity_shape(lat, torch.complex64), dtype=torch.complex64, device=lat.device)
    lat.sync_stream()
    check(lib().ddq_mrhs_unpack(lat.handle, n, _dev(v, "v"), _dev(out, "out")), "ddq_mrhs_unpack")
    return out


def mrhs_apply_schur(lat: Lattice, x: torch.Tensor, y: torch.Tensor = None, engine: int = DDQ_ENGINE_MFMA) -> torch.Tensor:
    """y = D_S x on mrhs-layout vectors."""
    n = _nrhs_mrhs(lat, x)
    if y is None:
        y = torch.empty_like(x)
    reserve(lat, n)
    lat.sync_stream()
    check(lib().ddq_mrhs_apply_schur(lat.handle, n, _dev(x, "x"), _dev(y, "y"), int(engine)), "ddq_mrhs_apply_schur")
    return y


def mrhs_richardson_smooth(lat: Lattice, x: torch.Tensor, b: torch.Tensor, nsweeps: int, omega: float,
                           engine: int = DDQ_ENGINE_MFMA) -> torch.Tensor:
    """Alg. 4 on D_S, in place on the mrhs-layout x."""
    n = _nrhs_mrhs(lat, x)
    if b.shape != x.shape or b.dtype != x.dtype:
        raise ValueError("x and b must match in dtype and shape")
    reserve(lat, n)
    lat.sync_stream()
    check(lib().ddq_mrhs_richardson_smooth(lat.handle, n, _dev(x, "x"), _dev(b, "b"), int(nsweeps), float(omega),
                                           int(engine)), "ddq_mrhs_richardson_smooth")
    return x


def mrhs_set_launch(lat: Lattice, order: int = 1, lds_kb: int = 0, tsteps: int = 0, stage: int = 1) -> None:
    """Workgroup order of the mrhs stencil (0 plain, 1 slab, 2 t walk of tsteps slices),
    the LDS requested per workgroup (an occupancy cap) and LDS staging of links and clover."""
    check(lib().ddq_mrhs_set_launch(lat.handle, int(order), int(lds_kb), int(tsteps), int(stage)),
          "ddq_mrhs_set_launch")


def richardson_smooth(lat: Lattice, x_e: torch.Tensor, b_e: torch.Tensor, nsweeps: int, omega: float) -> torch.Tensor:
    """Alg. 4 on D_S, in place on x_e."""
    n = _nrhs_parity(lat, x_e)
    if b_e.dtype != x_e.dtype or b_e.shape != x_e.shape:
        raise ValueError("x_e and b_e must match in dtype and shape")
    reserve(lat, n)
    lat.sync_stream()
    check(lib().ddq_richardson_smooth(lat.handle, _prec(x_e), n, _dev(x_e, "x_e"), _dev(b_e, "b_e"),
                                      int(nsweeps), float(omega)), "ddq_richardson_smooth")
    return x_e


def set_multi_rhs_tile(lat: Lattice, nrhs: int, nb: int, waves: int = 4, xcd_map: int = 0, passes: int = 1,
                       lds_kb: int = 0) -> None:
    """Tile of the FP32 multi-right-hand-side stencil for launches of nrhs right-hand
    sides (nb = 0: one right-hand side per thread; xcd_map: 0 dispatcher order, c > 0
    chunks of c site blocks per XCD, -1 slab order; passes: launches over consecutive
    groups of right-hand sides; lds_kb: LDS per workgroup capping the resident ones)."""
    t = _lib.MrTile(int(nb), int(waves), int(xcd_map), 0.0, int(passes), int(lds_kb))
    check(lib().ddq_set_multi_rhs_tile(lat.handle, int(nrhs), C.byref(t)), "ddq_set_multi_rhs_tile")


def tune_multi_rhs(lat: Lattice, nrhs: int, reps: int = 5):
    """Time every tile for nrhs right-hand sides and keep the fastest.  Returns
    (chosen, candidates) as dicts."""
    arr = (_lib.MrTile * 512)()
    n = C.c_int()
    best = _lib.MrTile()
    reserve(lat, nrhs)
    lat.sync_stream()
    check(lib().ddq_tune_multi_rhs(lat.handle, int(nrhs), int(reps), arr, 512, C.byref(n), C.byref(best)),
          "ddq_tune_multi_rhs")
    return best.as_dict(), [arr[k].as_dict() for k in range(min(n.value, 512))]


def estimate_lambda_max(lat: Lattice, iters: int, v0: torch.Tensor) -> float:
    if v0.dtype != torch.complex128:
        raise TypeError("v0 must be complex128")
    _nrhs_parity(lat, v0)
    out = C.c_double()
    lat.sync_stream()
    check(lib().ddq_estimate_lambda_max(lat.handle, int(iters), _dev(v0, "v0"), C.byref(out)),
          "ddq_estimate_lambda_max")
    return out.value


def oe_prepare(lat: Lattice, b: torch.Tensor) -> torch.Tensor:
    n = _nrhs_full(lat, b)
    if b.dtype != torch.complex128:
        raise TypeError("b must be complex128")
    bt = parity_vector(lat, None if b.dim() == 6 else n)
    reserve(lat, n)
    lat.sync_stream()
    check(lib().ddq_oe_prepare(lat.handle, n, _dev(b, "b"), _dev(bt, "bt_e")), "ddq_oe_prepare")
    return bt


def oe_reconstruct(lat: Lattice, x_e: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    n = _nrhs_full(lat, b)
    if b.dtype != torch.complex128 or x_e.dtype != torch.complex128:
        raise TypeError("x_e and b must be complex128")
    x = torch.empty_like(b)
    reserve(lat, n)
    lat.sync_stream()
    check(lib().ddq_oe_reconstruct(lat.handle, n, _dev(x_e, "x_e"), _dev(b, "b"), _dev(x, "x")),
          "ddq_oe_reconstruct")
    return x


def oe_gmres_solve(lat: Lattice, b: torch.Tensor, x0: torch.Tensor = None, m: int = 30, max_cycles: int = 100,
                   tol: float = 1e-10, inner_prec: int = DDQ_F64, smoother_sweeps: int = 0, omega: float = 0.0,
                   inner_reduction: float = 0.0, smoother_prec: int = None, orth_passes: int = 2):
    """Odd-even GMRES(m) of Alg. 2 with eq. 2 around it, to |b - D x| <= tol |b|.  b: one
    full vector or [nrhs, ...] (solved one after the other).  Returns (x, info,
    converged): info a dict (one right-hand side) or a list of dicts, converged True
    when every system met tol."""
    n = _full_nrhs(lat, b, "b")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    p = GmresParams(int(m), int(max_cycles), float(tol), int(inner_prec), int(smoother_sweeps), float(omega),
                    float(inner_reduction), int(inner_prec if smoother_prec is None else smoother_prec),
                    int(orth_passes))
    info = (SolveInfo * n)()
    reserve(lat, 1, m, DDQ_RESERVE_SOLVE)
    lat.sync_stream()
    st = check(lib().ddq_oe_gmres_solve(lat.handle, n, _dev(x, "x"), _dev(b, "b"), C.byref(p), info),
               "ddq_oe_gmres_solve", allow=(0, 1))
    infos = [i.as_dict() for i in info]
    return x, (infos[0] if b.dim() == 6 else infos), st == 0


def _full_nrhs(lat, v, name):
    if v.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128")
    if tuple(v.shape) == lat.full_shape:
        return 1
    if v.dim() == len(lat.full_shape) + 1 and tuple(v.shape[1:]) == lat.full_shape:
        return v.shape[0]
    raise ValueError(f"{name} must be {lat.full_shape} or [nrhs, *{lat.full_shape}]")


def apply_dirac(lat: Lattice, x: torch.Tensor, y: torch.Tensor = None) -> torch.Tensor:
    """y = D x on full FP64 vectors (eq. 1)."""
    n = _full_nrhs(lat, x, "x")
    if y is None:
        y = torch.empty_like(x)
    reserve(lat, n, 0, DDQ_RESERVE_FULL)
    lat.sync_stream()
    check(lib().ddq_apply_dirac(lat.handle, n, _dev(x, "x"), _dev(y, "y")), "ddq_apply_dirac")
    return y


def oe_smoother(lat: Lattice, r: torch.Tensor, nsweeps: int, omega: float, prec: int = DDQ_F64,
                z: torch.Tensor = None) -> torch.Tensor:
    """z = M_nu r (Sect. 2.4.5): eq. 2 with D_S^-1 replaced by nsweeps Richardson sweeps
    from zero, the sweeps in prec (DDQ_F64 or DDQ_F32)."""
    n = _full_nrhs(lat, r, "r")
    if z is None:
        z = torch.empty_like(r)
    reserve(lat, n, 0, DDQ_RESERVE_FULL)
    lat.sync_stream()
    check(lib().ddq_oe_smoother(lat.handle, n, _dev(r, "r"), _dev(z, "z"), int(nsweeps), float(omega), int(prec)),
          "ddq_oe_smoother")
    return z


def sap_smooth(lat: Lattice, b: torch.Tensor, x: torch.Tensor, n: int, m: int, prec: int = DDQ_F64) -> torch.Tensor:
    """SAP(n, m) of Alg. 1 on D x = b with 4^4 blocks, in place on x (full FP64); the
    block solves in prec (DDQ_F64 or DDQ_F32)."""
    if _full_nrhs(lat, b, "b") != 1 or _full_nrhs(lat, x, "x") != 1:
        raise ValueError("one right-hand side")
    reserve(lat, 1, 0, DDQ_RESERVE_SAP)
    lat.sync_stream()
    check(lib().ddq_sap_smooth(lat.handle, int(prec), _dev(x, "x"), _dev(b, "b"), int(n), int(m)), "ddq_sap_smooth")
    return x


def fgmres_solve(lat: Lattice, b: torch.Tensor, x0: torch.Tensor = None, m: int = 30, max_cycles: int = 100,
                 tol: float = 1e-10, smoother_sweeps: int = 3, omega: float = 0.0, inner_prec: int = DDQ_F64,
                 inner_reduction: float = 0.0, orth_passes: int = 2):
    """FGMRES(m) of Alg. 2 on the full D x = b with M_nu as right preconditioner.
    Returns (x, info, converged)."""
    if b.dtype != torch.complex128 or tuple(b.shape) != lat.full_shape:
        raise ValueError(f"b must be complex128 of shape {lat.full_shape}")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    p = GmresParams(int(m), int(max_cycles), float(tol), int(inner_prec), int(smoother_sweeps), float(omega),
                    float(inner_reduction), int(inner_prec), int(orth_passes))
    info = SolveInfo()
    reserve(lat, 1, m, DDQ_RESERVE_FULL)
    lat.sync_stream()
    st = check(lib().ddq_fgmres_solve(lat.handle, _dev(x, "x"), _dev(b, "b"), C.byref(p), C.byref(info)),
               "ddq_fgmres_solve", allow=(0, 1))
    return x, info.as_dict(), st == 0


def fgmres_sap_solve(lat: Lattice, b: torch.Tensor, x0: torch.Tensor = None, m: int = 30, max_cycles: int = 100,
                     tol: float = 1e-10, sap_n: int = 1, sap_m: int = 4, inner_prec: int = DDQ_F64,
                     inner_reduction: float = 0.0, orth_passes: int = 2):
    """FGMRES(m) of Alg. 2 on the full D x = b with SAP(sap_n, sap_m) as right
    preconditioner (block solves in inner_prec).  Returns (x, info, converged)."""
    if b.dtype != torch.complex128 or tuple(b.shape) != lat.full_shape:
        raise ValueError(f"b must be complex128 of shape {lat.full_shape}")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    p = GmresParams(int(m), int(max_cycles), float(tol), int(inner_prec), 0, 0.0, float(inner_reduction),
                    int(inner_prec), int(orth_passes))
    info = SolveInfo()
    reserve(lat, 1, m, DDQ_RESERVE_SAP)
    lat.sync_stream()
    st = check(lib().ddq_fgmres_sap_solve(lat.handle, _dev(x, "x"), _dev(b, "b"), C.byref(p), int(sap_n),
                                          int(sap_m), C.byref(info)), "ddq_fgmres_sap_solve", allow=(0, 1))
    return x, info.as_dict(), st == 0


class Batch:
    """Handle of a ddq_batch; keeps its lattices alive while it exists."""

    def __init__(self, handle: C.c_void_p, lats, nrhs):
        self.handle = handle
        self.lats = list(lats)
        self.nrhs = list(nrhs)

    def __del__(self):
        h = getattr(self, "handle", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None  # None at interpreter exit
        if h is not None and L is not None:
            try:
                L.ddq_batch_destroy(h)
            except Exception:  # pragma: no cover
                pass
            self.handle = None


def batch_create(lats, nrhs) -> Batch:
    """A batch of lattices (distinct handles) with nrhs[l] right-hand sides each."""
    lats = list(lats)
    nrhs = [int(n) for n in nrhs]
    if len(lats) != len(nrhs):
        raise ValueError("one nrhs per lattice")
    dev = lats[0].device
    arr = (C.c_void_p * len(lats))(*[l.handle for l in lats])
    nr = (C.c_int * len(lats))(*nrhs)
    h = C.c_void_p()
    s = torch.cuda.current_stream(dev).cuda_stream
    check(lib().ddq_batch_create(arr, nr, len(lats), C.c_void_p(s), C.byref(h)), "ddq_batch_create")
    return Batch(h, lats, nrhs)


def batch_reserve(batch: Batch, max_m: int, cycle_graph: bool = False) -> None:
    """Work space of later solves with m <= max_m (and the tuning of untuned lattices)."""
    check(lib().ddq_batch_reserve(batch.handle, int(max_m), int(bool(cycle_graph))), "ddq_batch_reserve")


def batch_destroy(batch: Batch) -> None:
    if batch.handle is not None:
        check(lib().ddq_batch_destroy(batch.handle), "ddq_batch_destroy")
        batch.handle = None


def batch_solve(batch: Batch, bs, x0s=None, m: int = 50, max_cycles: int = 100, tol: float = 1e-10,
                smoother_sweeps: int = 4, omega=0.0, inner_reduction: float = 0.0, smoother_prec: int = DDQ_F32,
                orth_passes: int = 2, cycle_graph: bool = False):
    """Solve every (lattice, right-hand side) system of the batch.  bs[l]: complex128
    [nrhs[l], Lt, Lz, Ly, Lx, 4, 3]; omega: one weight or one per lattice.
    Returns (xs, infos, converged) with infos in (lattice, right-hand side) order."""
    if len(bs) != len(batch.lats):
        raise ValueError("one right-hand-side tensor per lattice")
    xs = []
    for l, (lat, n, b) in enumerate(zip(batch.lats, batch.nrhs, bs)):
        want = (n,) + lat.full_shape
        if b.dtype != torch.complex128 or tuple(b.shape) != want:
            raise ValueError(f"b[{l}] must be complex128 of shape {want}")
        xs.append(torch.zeros_like(b) if x0s is None else x0s[l].clone())
    om = [float(omega)] * len(bs) if isinstance(omega, (int, float)) else [float(w) for w in omega]
    if len(om) != len(bs):
        raise ValueError("one omega per lattice")
    xp = (C.c_void_p * len(bs))(*[_dev(x, "x").value for x in xs])
    bp = (C.c_void_p * len(bs))(*[_dev(b, "b").value for b in bs])
    op = (C.c_double * len(bs))(*om)
    p = GmresParams(int(m), int(max_cycles), float(tol), DDQ_F32, int(smoother_sweeps), om[0],
                    float(inner_reduction), int(smoother_prec), int(orth_passes), int(bool(cycle_graph)))
    infos = (SolveInfo * sum(batch.nrhs))()
    batch_reserve(batch, m, cycle_graph)
    st = check(lib().ddq_batch_solve(batch.handle, xp, bp, C.byref(p), op, infos), "ddq_batch_solve", allow=(0, 1))
    return xs, [i.as_dict() for i in infos], st == 0


def profile_begin(lat: Lattice) -> None:
    """Start bracketing every stencil launch with HIP events on the lattice's stream."""
    lat.sync_stream()
    check(lib().ddq_profile_begin(lat.handle), "ddq_profile_begin")


def profile_end(lat: Lattice):
    """Stop profiling; per kernel variant: launches, total and mean event time,
    algorithmic bytes per launch."""
    arr = (_lib.KernelStats * 64)()
    n = C.c_int()
    check(lib().ddq_profile_end(lat.handle, arr, 64, C.byref(n)), "ddq_profile_end")
    out = {}
    for k in range(min(n.value, 64)):
        e = arr[k]
        out[e.name.decode()] = {"launches": e.launches, "total_ms": e.total_ms,
                                "mean_ms": e.total_ms / max(e.launches, 1), "bytes_per_launch": e.bytes_per_launch}
    return out


def stream_copy(dst: torch.Tensor, src: torch.Tensor, nontemporal: bool = False) -> None:
    """Device copy through the library's STREAM-style kernel on torch's current stream
    (nontemporal: non-temporal loads and stores)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nb:
        raise ValueError("dst too small")
    s = torch.cuda.current_stream(src.device).cuda_stream
    check(lib().ddq_stream_copy(_dev(dst, "dst"), _dev(src, "src"), nb, int(bool(nontemporal)), C.c_void_p(s)),
          "ddq_stream_copy")


def stencil_stream(lat: Lattice, kernel: int, in_e: torch.Tensor, out: torch.Tensor, x_e: torch.Tensor = None,
                   b_e: torch.Tensor = None) -> None:
    """Streaming ceiling of stencil kernel 0 (A), 1 (B apply) or 2 (B Richardson) on
    FP32 or FP64 parity vectors: the kernel's bytes without gathers or arithmetic
    (out receives meaningless values)."""
    if tuple(in_e.shape) != _parity_shape(lat, in_e.dtype):
        raise ValueError("one right-hand side parity vector expected")
    vecs = [v for v in (in_e, out, x_e, b_e) if v is not None]
    if any(v.dtype != in_e.dtype or v.shape != in_e.shape for v in vecs):
        raise ValueError("all vectors must match in dtype and shape")
    lat.sync_stream()
    check(lib().ddq_stencil_stream(lat.handle, _prec(in_e), int(kernel), _dev(in_e, "in_e"),
                                   None if x_e is None else _dev(x_e, "x_e"),
                                   None if b_e is None else _dev(b_e, "b_e"), _dev(out, "out")),
          "ddq_stencil_stream")


def backward_apply(lat: Lattice, grad_y_e: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    """grad_x_e = D_S^H grad_y_e (the adjoint apply)."""
    n = _nrhs_parity(lat, grad_y_e)
    if out is None:
        out = torch.empty_like(grad_y_e)
    reserve(lat, n)
    lat.sync_stream()
    check(lib().ddq_backward_apply(lat.handle, _prec(grad_y_e), n, _dev(grad_y_e, "grad_y_e"), _dev(out, "grad_x_e")),
          "ddq_backward_apply")
    return out


def backward_link_force(lat: Lattice, chi_e: torch.Tensor, phi_e: torch.Tensor, want_G: bool = True,
                        want_F: bool = False, G: torch.Tensor = None, F: torch.Tensor = None):
    """Derivative of L = Re(chi_e^H D_S(U) phi_e) with respect to the links: G (torch's
    complex-gradient convention, [Lt, Lz, Ly, Lx, 4, 3, 3]) and/or the su(3) force F
    ([Lt, Lz, Ly, Lx, 4, 8]).  Passing G / F accumulates into them."""
    if chi_e.dtype != torch.complex128 or phi_e.dtype != torch.complex128:
        raise TypeError("chi_e and phi_e must be complex128")
    if _nrhs_parity(lat, chi_e) != 1 or _nrhs_parity(lat, phi_e) != 1:
        raise ValueError("one right-hand side")
    acc = G is not None or F is not None
    if acc and ((want_G and G is None) or (want_F and F is None)):
        raise ValueError("pass every requested output when accumulating")
    shp = lat.full_shape[:4] + (4,)
    if want_G and G is None:
        G = torch.empty(shp + (3, 3), dtype=torch.complex128, device=lat.device)
    if want_F and F is None:
        F = torch.empty(shp + (8,), dtype=torch.float64, device=lat.device)
    reserve(lat, 1, 0, DDQ_RESERVE_FORCE)
    lat.sync_stream()
    check(lib().ddq_backward_link_force(lat.handle, _dev(chi_e, "chi_e"), _dev(phi_e, "phi_e"),
                                        _dev(G, "G") if want_G else None, _dev(F, "F") if want_F else None,
                                        int(acc)), "ddq_backward_link_force")
    return G, F


class CoarseOperator:
    """The coarse-grid operator of Sect. 2.3 on the device: nine 2N_v x 2N_v complex
    blocks per coarse site, packed once into the library's FP32 operand order.

    blocks: complex128 or complex64 device tensor [sites, 9, 2 N_v, 2 N_v] (block d = 0
    the site's own, d = 1 + 2 mu + s the neighbour in direction mu, forward s = 0 or
    backward s = 1); cdims: coarse extents (x, y, z, t), site index x fastest; storage:
    DDQ_F32, DDQ_F16 or DDQ_BF16 for the packed blocks (FP32 arithmetic in all cases)."""

    def __init__(self, cdims, blocks: torch.Tensor, storage: int = DDQ_F32):
        self.cdims = tuple(int(c) for c in cdims)
        if len(self.cdims) != 4:
            raise ValueError("cdims needs four extents")
        vc = 1
        for c in self.cdims:
            vc *= c
        if blocks.dim() != 4 or blocks.shape[0] != vc or blocks.shape[1] != 9 or blocks.shape[2] != blocks.shape[3] \
                or blocks.shape[2] % 2:
            raise ValueError(f"blocks must be [{vc}, 9, 2 N_v, 2 N_v], got {tuple(blocks.shape)}")
        if blocks.dtype not in (torch.complex128, torch.complex64):
            raise TypeError("blocks must be complex128 or complex64")
        self.nv = blocks.shape[2] // 2
        self.vc = vc
        self.device = blocks.device
        self._cd = (C.c_int * 4)(*self.cdims)
        self.storage = int(storage)
        nb = C.c_int64()
        check(lib().ddq_coarse_packed_bytes(self._cd, self.nv, self.storage, C.byref(nb)), "ddq_coarse_packed_bytes")
        self.packed = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib().ddq_coarse_pack_blocks(self._cd, self.nv, self.storage, _prec(blocks), _dev(blocks, "blocks"),
                                           _dev(self.packed, "packed"), C.c_void_p(s)), "ddq_coarse_pack_blocks")

    def apply(self, v: torch.Tensor, out: torch.Tensor = None, rhs_tiles_per_wave: int = 0,
              product: int = 0) -> torch.Tensor:
        """y = D_c v; v complex64 [sites, 2 N_v] or [sites, 2 N_v, nrhs] (right-hand side innermost);
        product: 0 default, 1 four real products per complex one, 2 Gauss's three"""
        if v.dtype != torch.complex64:
            raise TypeError("coarse vectors are complex64")
        if v.dim() not in (2, 3) or v.shape[0] != self.vc or v.shape[1] != 2 * self.nv:
            raise ValueError(f"v must be [{self.vc}, {2 * self.nv}(, nrhs)], got {tuple(v.shape)}")
        nrhs = 1 if v.dim() == 2 else v.shape[2]
        y = torch.empty_like(v) if out is None else out
        if y.shape != v.shape or y.dtype != v.dtype:
            raise ValueError("out must match v")
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib().ddq_coarse_apply(self._cd, self.nv, self.storage, nrhs, _dev(self.packed, "packed"), _dev(v, "v"),
                                     _dev(y, "out"), int(rhs_tiles_per_wave), int(product), C.c_void_p(s)),
              "ddq_coarse_apply")
        return y
