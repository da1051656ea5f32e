"""Thin ctypes binding over libsr.so.

Argument marshalling only: every step of the computation runs in the library's HIP
kernels.  Torch supplies device buffers (data_ptr) and the current HIP stream.  If the
library is not built, `lib()` raises instead of falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SR_LIBRARY names another build of the same library (the host-sanitizer build, say)
LIB_PATH = os.environ.get("SR_LIBRARY") or os.path.join(_HERE, "libsr.so")

# enum sr_status
SR_OK, SR_NOT_CONVERGED, SR_BREAKDOWN = 0, 1, 2
SR_ERR_INVALID, SR_ERR_NOMEM, SR_ERR_HIP, SR_ERR_NONFINITE, SR_ERR_NODEVICE, SR_ERR_TIMEOUT = -1, -2, -3, -4, -5, -6
# enum sr_dtype
SR_F64, SR_F32, SR_BF16, SR_F16 = 0, 1, 2, 3

_TORCH_DT = {torch.float64: SR_F64, torch.float32: SR_F32, torch.bfloat16: SR_BF16, torch.float16: SR_F16}
_ELEM = {SR_F64: 8, SR_F32: 4, SR_BF16: 2, SR_F16: 2}

# C prototypes: name -> (restype, argtypes); mirrors include/sr.h
_c_i64, _c_i32, _c_p, _c_d = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double


class SrMatrix(ctypes.Structure):
    _fields_ = [("n_s", _c_i64), ("n_p", _c_i64), ("ld", _c_i64), ("dtype", _c_i32), ("reserved", _c_i32),
                ("O", _c_p), ("O_lo", _c_p), ("col_scale", _c_p), ("col_mean", _c_p), ("lo_cols", _c_p),
                ("n_lo", _c_i64), ("ld_lo", _c_i64)]


class SrCpsMatrix(ctypes.Structure):
    _fields_ = [("n_s", _c_i64), ("n_corr", _c_i64), ("n_states", _c_i32), ("reserved", _c_i32),
                ("idx", _c_p), ("ld_idx", _c_i64), ("val", _c_p), ("dense", SrMatrix), ("col_mean", _c_p)]


class SrStreamAcc(ctypes.Structure):
    _fields_ = [("n_p", _c_i64), ("m", _c_i32), ("reserved", _c_i32), ("A", _c_p), ("s1", _c_p), ("se", _c_p),
                ("scal", _c_p)]


class SrCgOpts(ctypes.Structure):
    _fields_ = [("rtol", _c_d), ("max_iter", _c_i32), ("refresh_every", _c_i32), ("use_x0", _c_i32),
                ("restart_on_refresh", _c_i32), ("res_history", _c_p), ("refresh_drop", _c_d),
                ("precond", _c_i32), ("search_f64", _c_i32), ("reserved", _c_i32)]


class SrCgInfo(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("refreshes", _c_i32), ("status", _c_i32), ("products", _c_i32),
                ("rel_res_recur", _c_d), ("rel_res_true", _c_d)]


BATCH_MAX_RHS = 8


class LmDavidsonOpts(ctypes.Structure):
    _fields_ = [("tol", _c_d), ("max_iter", _c_i32), ("max_sub", _c_i32), ("precond", _c_i32),
                ("reserved", _c_i32)]


class LmDavidsonInfo(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("restarts", _c_i32), ("status", _c_i32), ("reserved", _c_i32),
                ("theta", _c_d), ("res_norm", _c_d)]


class SrBatchSystem(ctypes.Structure):
    _fields_ = [("O", SrMatrix), ("g", _c_p), ("x", _c_p), ("eps", _c_d * BATCH_MAX_RHS)]


class SrShiftSystem(ctypes.Structure):
    _fields_ = [("O", SrMatrix), ("g", _c_p), ("X", _c_p), ("eps", _c_d * BATCH_MAX_RHS)]


PROTOTYPES = {
    "sr_grad": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "sr_sv_product": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, _c_p, _c_d, _c_p]),
    "sr_sv_product_noalloc": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, _c_p, _c_d, _c_p]),
    "sr_cg_solve": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, _c_d, _c_p, ctypes.POINTER(SrCgOpts),
                                   ctypes.POINTER(SrCgInfo), _c_p]),
    "lm_hv_product": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, ctypes.POINTER(SrMatrix), _c_p, _c_p, _c_p]),
    "sr_cg_solve_shifts": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, _c_i32, _c_p, _c_p,
                                          ctypes.POINTER(SrCgOpts), _c_p, _c_p]),
    "sr_set_batch_config": (ctypes.c_int, [_c_i32, _c_i32]),
    "sr_cg_solve_shifts_batched": (ctypes.c_int, [_c_i32, ctypes.POINTER(SrShiftSystem), _c_i32,
                                                  ctypes.POINTER(SrCgOpts), ctypes.POINTER(SrCgInfo), _c_p]),
    "lm_davidson": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, ctypes.POINTER(SrMatrix),
                                   ctypes.POINTER(LmDavidsonOpts), _c_p, ctypes.POINTER(LmDavidsonInfo), _c_p]),
    "sr_quantize": (ctypes.c_int, [_c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_p, _c_p, _c_i64, _c_i32, _c_p, _c_p]),
    "sr_remainder_columns": (ctypes.c_int, [_c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_d, _c_p,
                                            ctypes.POINTER(_c_i64), _c_p]),
    "sr_quantize_remainder": (ctypes.c_int, [_c_i64, _c_i64, _c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p,
                                             _c_i64, _c_p]),
    "sr_cps_grad": (ctypes.c_int, [ctypes.POINTER(SrCpsMatrix), _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "sr_cps_sv_product": (ctypes.c_int, [ctypes.POINTER(SrCpsMatrix), _c_p, _c_p, _c_d, _c_p]),
    "sr_cps_cg_solve": (ctypes.c_int, [ctypes.POINTER(SrCpsMatrix), _c_p, _c_d, _c_p, ctypes.POINTER(SrCgOpts),
                                       ctypes.POINTER(SrCgInfo), _c_p]),
    "sr_stream_begin": (ctypes.c_int, [ctypes.POINTER(SrStreamAcc), _c_p]),
    "sr_stream_accumulate": (ctypes.c_int, [ctypes.POINTER(SrStreamAcc), ctypes.POINTER(SrMatrix),
                                            ctypes.POINTER(SrCpsMatrix), _c_p, _c_p, _c_p]),
    "sr_stream_finish": (ctypes.c_int, [ctypes.POINTER(SrStreamAcc), _c_p, _c_d, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "sr_release": (ctypes.c_int, []),
    "sr_workspace_bytes": (ctypes.c_int64, [ctypes.POINTER(SrMatrix), _c_i32]),
    "sr_workspace_reserve": (ctypes.c_int, [_c_i64, _c_p]),
    "sr_workspace_held": (ctypes.c_int64, [_c_p]),
    "sr_timing": (ctypes.c_int, [_c_i32]),
    "sr_timing_read": (ctypes.c_int, [_c_i32, ctypes.POINTER(_c_d), ctypes.POINTER(_c_i64)]),
    "sr_cg_solve_async": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, _c_d, _c_p, ctypes.POINTER(SrCgOpts), _c_p,
                                         _c_p]),
    "sr_stream_read": (ctypes.c_int, [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p]),
    "sr_adjoint": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_p, _c_p, _c_p, _c_p, _c_p, _c_i32, ctypes.c_int64,
                                  _c_p, _c_p, _c_p]),
    "sr_svk_product": (ctypes.c_int, [ctypes.POINTER(SrMatrix), _c_i32, _c_p, ctypes.POINTER(_c_d), _c_p, _c_i32,
                                      _c_p]),
    "sr_cg_solve_batched": (ctypes.c_int, [_c_i32, ctypes.POINTER(SrBatchSystem), _c_i32, ctypes.POINTER(SrCgOpts),
                                           ctypes.POINTER(SrCgInfo), _c_p]),
    "sr_tile_configs": (ctypes.c_int, [_c_i32, _c_i32, ctypes.POINTER(ctypes.c_int32), _c_i32]),
    "sr_set_tile_config": (ctypes.c_int, [_c_i32, _c_i32, _c_i32, _c_i32, _c_i32, _c_i32, _c_i32, _c_i32]),
    "sr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sr_last_error": (ctypes.c_char_p, []),
    "sr_version": (ctypes.c_int, []),
}

_lib = None


def _release_at_exit():
    """Free the library's device workspaces before the interpreter (and with it the HIP
    runtime) shuts down, after the work queued on the device has finished."""
    if _lib is None:
        return
    try:
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
        _lib.sr_release()
    except Exception:
        pass


atexit.register(_release_at_exit)


def lib():
    """Load libsr.so (built by paper_1108_0900_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsr.so not built at {LIB_PATH}; run `python -m paper_1108_0900_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SrError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        self.status = status
        super().__init__(f"{where}: {L.sr_status_string(status).decode()} ({L.sr_last_error().decode()})")


def _check(status: int, where: str, allow=(SR_OK,)):
    if status not in allow:
        raise SrError(status, where)
    return status


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Matrix:
    """A derivative-ratio matrix as the library sees it (keeps the tensors alive)."""
    O: torch.Tensor              # (n_s, ld) storage; columns [0, n_p) are used
    n_p: int
    scale: torch.Tensor | None = None
    mean: torch.Tensor | None = None
    lo: torch.Tensor | None = None   # second code plane: same layout as O, or compact (n_s, n_lo)
    lo_cols: torch.Tensor | None = None  # int32 parameters of the compact plane's columns

    @property
    def dtype_code(self) -> int:
        return _TORCH_DT[self.O.dtype]

    @property
    def ld(self) -> int:
        if self.O.shape[0] > 1:
            return self.O.stride(0)
        vec = 16 // _ELEM[self.dtype_code]
        return ((self.n_p + vec - 1) // vec) * vec

    def c(self) -> SrMatrix:
        m = SrMatrix()
        m.n_s = self.O.shape[0]
        m.n_p = self.n_p
        m.ld = self.ld
        m.dtype = self.dtype_code
        m.reserved = 0
        m.O = self.O.data_ptr()
        m.O_lo = None if self.lo is None else self.lo.data_ptr()
        m.col_scale = None if self.scale is None else self.scale.data_ptr()
        m.col_mean = None if self.mean is None else self.mean.data_ptr()
        m.lo_cols = None
        m.n_lo = 0
        m.ld_lo = 0
        if self.lo_cols is not None:
            m.lo_cols = self.lo_cols.data_ptr() if self.lo_cols.numel() else None
            m.n_lo = self.lo_cols.numel()
            if m.n_lo:
                m.ld_lo = self.lo.stride(0) if self.lo.shape[0] > 1 else ((m.n_lo + 7) // 8) * 8
            else:
                m.O_lo = None
        return m

    @property
    def n_lo(self) -> int:
        return 0 if self.lo_cols is None else self.lo_cols.numel()


def _padded(t: torch.Tensor, vec: int) -> torch.Tensor:
    """t itself if its layout meets the rules of sr.h (16-byte aligned base, row stride a
    multiple of 16 bytes, unit column stride, rows spanning the allocation), else a copy
    with padded rows."""
    n_s, n = t.shape
    eb = t.element_size()
    ld = t.stride(0) if n_s > 1 else ((n + vec - 1) // vec) * vec
    ok = t.stride(1) == 1 and ld >= n and (ld * eb) % 16 == 0 and t.data_ptr() % 16 == 0
    if ok:
        need = t.storage_offset() + (n_s - 1) * ld + ((n + vec - 1) // vec) * vec
        ok = need <= t.untyped_storage().nbytes() // eb
    if ok:
        return t
    P = torch.zeros(n_s, max(vec, ((n + vec - 1) // vec) * vec), dtype=t.dtype, device=t.device)
    P[:, :n] = t
    return P[:, :n]


def as_matrix(O: torch.Tensor, scale: torch.Tensor | None = None, mean: torch.Tensor | None = None,
              lo: torch.Tensor | None = None, lo_cols: torch.Tensor | None = None) -> Matrix:
    """Wrap a 2-D device tensor (float64/float32, or bfloat16/float16 codes with a float32
    column scale).  A copy with padded rows is made only when the layout rules of sr.h
    (16-byte aligned base, row stride a multiple of 16 bytes, unit column stride, rows
    spanning the allocation) are not met.  `lo` is the second code plane: the full plane
    (shape of O), or with `lo_cols` (int32, increasing) the compact plane of those columns."""
    if O.dim() != 2:
        raise ValueError("O must be 2-D")
    if O.dtype not in _TORCH_DT:
        raise ValueError(f"unsupported dtype {O.dtype}")
    n_s, n_p = O.shape
    code = _TORCH_DT[O.dtype]
    eb = _ELEM[code]
    vec = 16 // eb
    ld = O.stride(0) if n_s > 1 else ((n_p + vec - 1) // vec) * vec
    ok = (O.stride(1) == 1 and ld >= n_p and (ld * eb) % 16 == 0 and O.data_ptr() % 16 == 0)
    if ok:
        need = O.storage_offset() + (n_s - 1) * ld + ((n_p + vec - 1) // vec) * vec
        ok = need <= O.untyped_storage().nbytes() // eb
    if not ok:
        ldp = ((n_p + vec - 1) // vec) * vec
        P = torch.zeros(n_s, ldp, dtype=O.dtype, device=O.device)
        P[:, :n_p] = O
        O = P[:, :n_p]
    if scale is not None:
        scale = scale.contiguous()
    if mean is not None:
        mean = mean.contiguous()
    if lo_cols is not None:
        lo_cols = lo_cols.to(torch.int32).contiguous()
        if lo is None and lo_cols.numel():
            raise ValueError("lo_cols needs the compact plane lo")
        if lo is not None:
            if lo.dim() != 2 or lo.shape != (n_s, lo_cols.numel()) or lo.dtype != O.dtype:
                raise ValueError("the compact plane must be (n_s, len(lo_cols)) of O's dtype")
            if lo_cols.numel():
                lo = _padded(lo, vec)
        return Matrix(O=O, n_p=n_p, scale=scale, mean=mean, lo=lo, lo_cols=lo_cols)
    if lo is not None:
        if lo.shape != O.shape or lo.dtype != O.dtype:
            raise ValueError("lo must have the shape and dtype of O")
        if lo.stride() != O.stride() or lo.data_ptr() % 16:
            ldo = O.stride(0) if n_s > 1 else ((n_p + vec - 1) // vec) * vec
            L = torch.zeros(n_s, ldo, dtype=O.dtype, device=O.device)
            L[:, :n_p] = lo
            lo = L[:, :n_p]
    return Matrix(O=O, n_p=n_p, scale=scale, mean=mean, lo=lo)


def _vec(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    if t.dtype != torch.float64 or t.dim() != 1 or t.shape[0] != n:
        raise ValueError(f"{name} must be a float64 vector of length {n}")
    return t.contiguous()


# ----------------------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ----------------------------------------------------------------------------------------
def sr_grad(M: Matrix, E: torch.Tensor | None, stream=None) -> dict:
    """Column means, diag S, g and <E> in one pass over O (sr_grad)."""
    dev = M.O.device
    n_p = M.n_p
    out = {"mean": torch.empty(n_p, dtype=torch.float64, device=dev),
           "diag": torch.empty(n_p, dtype=torch.float64, device=dev)}
    if E is not None:
        E = _vec(E, M.O.shape[0], "E")
        out["g"] = torch.empty(n_p, dtype=torch.float64, device=dev)
        out["E_mean"] = torch.empty(1, dtype=torch.float64, device=dev)
    m = M.c()
    st = lib().sr_grad(ctypes.byref(m), _ptr(E), _ptr(out.get("g")), _ptr(out.get("E_mean")), _ptr(out["mean"]),
                       _ptr(out["diag"]), _stream(stream))
    _check(st, "sr_grad")
    return out


def sr_sv_product(M: Matrix, v: torch.Tensor, eps: float = 0.0, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """y = (S + eps I) v (sr_sv_product)."""
    v = _vec(v, M.n_p, "v")
    y = torch.empty_like(v) if out is None else out
    m = M.c()
    _check(lib().sr_sv_product(ctypes.byref(m), _ptr(v), _ptr(y), float(eps), _stream(stream)), "sr_sv_product")
    return y


def sr_sv_product_noalloc(M: Matrix, v: torch.Tensor, eps: float, out: torch.Tensor, stream=None) -> torch.Tensor:
    """y = (S + eps I) v with the library's fixed scratch, no allocation
    (sr_sv_product_noalloc); M.mean and `out` are required."""
    v = _vec(v, M.n_p, "v")
    if M.mean is None:
        raise ValueError("sr_sv_product_noalloc needs the column means (M.mean)")
    m = M.c()
    _check(lib().sr_sv_product_noalloc(ctypes.byref(m), _ptr(v), _ptr(out), float(eps), _stream(stream)),
           "sr_sv_product_noalloc")
    return out


def sr_cg_solve(M: Matrix, g: torch.Tensor, eps: float, rtol: float = 1e-10, max_iter: int = 0,
                refresh_every: int = 0, x0: torch.Tensor | None = None, history: bool = False,
                restart_on_refresh: bool = False, refresh_drop: float = 0.0,
                precond: bool = False, search_f64: bool = False, out: torch.Tensor | None = None, raise_on=(SR_ERR_INVALID, SR_ERR_NOMEM, SR_ERR_HIP,
                                                           SR_ERR_NODEVICE, SR_ERR_TIMEOUT), stream=None):
    """CG solve of (S + eps I) x = g (sr_cg_solve).  Returns (x, info dict)."""
    g = _vec(g, M.n_p, "g")
    if x0 is not None:
        x = _vec(x0, M.n_p, "x0").clone() if out is None else out.copy_(x0)
    else:
        x = torch.empty_like(g) if out is None else out
    opts = SrCgOpts()
    opts.rtol = float(rtol)
    opts.max_iter = int(max_iter)
    opts.refresh_every = int(refresh_every)
    opts.use_x0 = 1 if x0 is not None else 0
    opts.restart_on_refresh = 1 if restart_on_refresh else 0
    opts.refresh_drop = float(refresh_drop)
    opts.precond = 1 if precond else 0
    opts.search_f64 = 1 if search_f64 else 0
    hist = None
    if history:
        mi = max_iter if max_iter > 0 else M.n_p + 100
        hist = torch.full((mi + 1,), float("nan"), dtype=torch.float64, device=g.device)
        opts.res_history = hist.data_ptr()
    info = SrCgInfo()
    m = M.c()
    st = lib().sr_cg_solve(ctypes.byref(m), _ptr(g), float(eps), _ptr(x), ctypes.byref(opts), ctypes.byref(info),
                           _stream(stream))
    if st in raise_on:
        raise SrError(st, "sr_cg_solve")
    d = {"status": st, "iters": info.iters, "refreshes": info.refreshes, "products": info.products,
         "rel_res_recur": info.rel_res_recur, "rel_res_true": info.rel_res_true}
    if hist is not None:
        d["history"] = hist
    return x, d


def _cg_opts(rtol, max_iter, refresh_every, use_x0, restart_on_refresh, refresh_drop, precond, search_f64):
    opts = SrCgOpts()
    opts.rtol = float(rtol)
    opts.max_iter = int(max_iter)
    opts.refresh_every = int(refresh_every)
    opts.use_x0 = 1 if use_x0 else 0
    opts.restart_on_refresh = 1 if restart_on_refresh else 0
    opts.refresh_drop = float(refresh_drop)
    opts.precond = 1 if precond else 0
    opts.search_f64 = 1 if search_f64 else 0
    return opts


def sr_cg_solve_async(M: Matrix, g: torch.Tensor, eps: float, x: torch.Tensor, info: torch.Tensor,
                      rtol: float = 1e-10, max_iter: int = 0, refresh_every: int = 0, use_x0: bool = False,
                      restart_on_refresh: bool = False, refresh_drop: float = 0.0, precond: bool = False,
                      search_f64: bool = False, stream=None):
    """CG solve queued on the stream without waiting (sr_cg_solve_async): x (in/out) and
    info, a float64 device tensor of 16 (iters, refreshes, status, products, rel_res_recur,
    rel_res_true, ...), are written when the solve runs."""
    g = _vec(g, M.n_p, "g")
    if info.dtype != torch.float64 or info.numel() < 16 or not info.is_contiguous():
        raise ValueError("info must be a contiguous float64 tensor of at least 16 entries")
    opts = _cg_opts(rtol, max_iter, refresh_every, use_x0, restart_on_refresh, refresh_drop, precond, search_f64)
    m = M.c()
    _check(lib().sr_cg_solve_async(ctypes.byref(m), _ptr(g), float(eps), _ptr(x), ctypes.byref(opts), _ptr(info),
                                   _stream(stream)), "sr_cg_solve_async")
    return x


# ----------------------------------------------------------------------------------------
# Index-coded CPS storage
# ----------------------------------------------------------------------------------------
@dataclass
class CpsMatrix:
    """Index-coded correlator-product-state storage as the library sees it (keeps the
    tensors alive): idx (n_corr, ld_idx) uint8 states, correlator-major; val (n_corr *
    n_states) float64 column values; dense the remaining parameters (a Matrix or None);
    mean the column means of all n_p parameters (or None)."""
    idx: torch.Tensor
    n_s: int
    n_states: int
    val: torch.Tensor
    dense: Matrix | None = None
    mean: torch.Tensor | None = None

    @property
    def n_corr(self) -> int:
        return self.idx.shape[0]

    @property
    def n_sp(self) -> int:
        return self.n_corr * self.n_states

    @property
    def n_d(self) -> int:
        return 0 if self.dense is None else self.dense.n_p

    @property
    def n_p(self) -> int:
        return self.n_sp + self.n_d

    def c(self) -> SrCpsMatrix:
        m = SrCpsMatrix()
        m.n_s = self.n_s
        m.n_corr = self.n_corr
        m.n_states = self.n_states
        m.reserved = 0
        m.idx = self.idx.data_ptr() if self.n_corr else None
        m.ld_idx = self.idx.stride(0) if self.n_corr > 1 else ((self.n_s + 15) // 16) * 16
        m.val = self.val.data_ptr() if self.n_corr else None
        if self.dense is not None:
            m.dense = self.dense.c()
        else:
            m.dense = SrMatrix()
            m.dense.n_s = self.n_s
            m.dense.dtype = SR_F64
        m.col_mean = None if self.mean is None else self.mean.data_ptr()
        return m


def cps_matrix(idx: torch.Tensor, val: torch.Tensor, n_states: int, dense: torch.Tensor | Matrix | None = None,
               dense_scale: torch.Tensor | None = None, mean: torch.Tensor | None = None) -> CpsMatrix:
    """Wrap index-coded CPS storage: idx (n_corr, n_s) uint8 states (correlator-major),
    val (n_corr * n_states) float64 column values, dense (n_s, n_d) the remaining
    parameters (float64, float32, or bfloat16 codes with dense_scale) or a Matrix.  A copy
    of idx with padded rows is made only when its layout breaks the rules of sr.h."""
    if idx.dtype != torch.uint8 or idx.dim() != 2:
        raise ValueError("idx must be a 2-D uint8 tensor (n_corr, n_s)")
    n_corr, n_s = idx.shape
    if dense is not None and not isinstance(dense, Matrix):
        if dense.shape[0] != n_s:
            raise ValueError("dense must have n_s rows")
        dense = as_matrix(dense, scale=dense_scale)
    if n_corr:
        ld = idx.stride(0) if n_corr > 1 else ((n_s + 15) // 16) * 16
        ok = idx.stride(1) == 1 and ld >= n_s and ld % 16 == 0 and idx.data_ptr() % 16 == 0
        if ok:
            ok = idx.storage_offset() + (n_corr - 1) * ld + ((n_s + 15) // 16) * 16 <= idx.untyped_storage().nbytes()
        if not ok:
            P = torch.zeros(n_corr, ((n_s + 15) // 16) * 16, dtype=torch.uint8, device=idx.device)
            P[:, :n_s] = idx
            idx = P[:, :n_s]
    val = val.to(torch.float64).contiguous()
    if val.numel() != n_corr * n_states:
        raise ValueError("val must hold n_corr * n_states values")
    return CpsMatrix(idx=idx, n_s=n_s, n_states=int(n_states), val=val, dense=dense,
                     mean=None if mean is None else mean.contiguous())


def sr_cps_grad(M: CpsMatrix, E: torch.Tensor | None, stream=None) -> dict:
    """Column means, diag S, g and <E> of CPS storage (sr_cps_grad)."""
    dev = M.val.device if M.n_corr else M.dense.O.device
    out = {"mean": torch.empty(M.n_p, dtype=torch.float64, device=dev),
           "diag": torch.empty(M.n_p, dtype=torch.float64, device=dev)}
    if E is not None:
        E = _vec(E, M.n_s, "E")
        out["g"] = torch.empty(M.n_p, dtype=torch.float64, device=dev)
        out["E_mean"] = torch.empty(1, dtype=torch.float64, device=dev)
    m = M.c()
    st = lib().sr_cps_grad(ctypes.byref(m), _ptr(E), _ptr(out.get("g")), _ptr(out.get("E_mean")), _ptr(out["mean"]),
                           _ptr(out["diag"]), _stream(stream))
    _check(st, "sr_cps_grad")
    return out


def sr_cps_sv_product(M: CpsMatrix, v: torch.Tensor, eps: float = 0.0, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """y = (S + eps I) v with CPS storage (sr_cps_sv_product)."""
    v = _vec(v, M.n_p, "v")
    y = torch.empty_like(v) if out is None else out
    m = M.c()
    _check(lib().sr_cps_sv_product(ctypes.byref(m), _ptr(v), _ptr(y), float(eps), _stream(stream)),
           "sr_cps_sv_product")
    return y


def sr_cps_cg_solve(M: CpsMatrix, g: torch.Tensor, eps: float, rtol: float = 1e-10, max_iter: int = 0,
                    refresh_every: int = 0, x0: torch.Tensor | None = None, restart_on_refresh: bool = False,
                    refresh_drop: float = 0.0, search_f64: bool = False, history: bool = False,
                    raise_on=(SR_ERR_INVALID, SR_ERR_NOMEM, SR_ERR_HIP, SR_ERR_NODEVICE, SR_ERR_TIMEOUT), stream=None):
    """CG solve of (S + eps I) x = g with CPS storage (sr_cps_cg_solve).  Returns (x, info)."""
    g = _vec(g, M.n_p, "g")
    x = _vec(x0, M.n_p, "x0").clone() if x0 is not None else torch.empty_like(g)
    opts = _cg_opts(rtol, max_iter, refresh_every, x0 is not None, restart_on_refresh, refresh_drop, False, search_f64)
    hist = None
    if history:
        mi = max_iter if max_iter > 0 else M.n_p + 100
        hist = torch.full((mi + 1,), float("nan"), dtype=torch.float64, device=g.device)
        opts.res_history = hist.data_ptr()
    info = SrCgInfo()
    m = M.c()
    st = lib().sr_cps_cg_solve(ctypes.byref(m), _ptr(g), float(eps), _ptr(x), ctypes.byref(opts), ctypes.byref(info),
                               _stream(stream))
    if st in raise_on:
        raise SrError(st, "sr_cps_cg_solve")
    d = {"status": st, "iters": info.iters, "refreshes": info.refreshes, "products": info.products,
         "rel_res_recur": info.rel_res_recur, "rel_res_true": info.rel_res_true}
    if hist is not None:
        d["history"] = hist
    return x, d


# ----------------------------------------------------------------------------------------
# Products during sampling
# ----------------------------------------------------------------------------------------
@dataclass
class StreamAcc:
    """Accumulators of products during sampling (device tensors kept alive here)."""
    A: torch.Tensor          # (m, n_p)
    s1: torch.Tensor         # (n_p,)
    se: torch.Tensor | None  # (n_p,) or None
    scal: torch.Tensor       # (4,)

    @property
    def n_p(self) -> int:
        return self.A.shape[1]

    @property
    def m(self) -> int:
        return self.A.shape[0]

    def c(self) -> SrStreamAcc:
        a = SrStreamAcc()
        a.n_p, a.m, a.reserved = self.n_p, self.m, 0
        a.A, a.s1, a.scal = self.A.data_ptr(), self.s1.data_ptr(), self.scal.data_ptr()
        a.se = None if self.se is None else self.se.data_ptr()
        return a


def sr_stream_begin(n_p: int, m: int, energies: bool = True, device="cuda", stream=None) -> StreamAcc:
    """New zeroed accumulators for m vectors over n_p parameters (sr_stream_begin)."""
    f64 = dict(dtype=torch.float64, device=device)
    acc = StreamAcc(A=torch.empty(m, n_p, **f64), s1=torch.empty(n_p, **f64),
                    se=torch.empty(n_p, **f64) if energies else None, scal=torch.empty(4, **f64))
    c = acc.c()
    _check(lib().sr_stream_begin(ctypes.byref(c), _stream(stream)), "sr_stream_begin")
    return acc


def sr_stream_accumulate(acc: StreamAcc, batch, E: torch.Tensor | None, Z: torch.Tensor, stream=None):
    """Add one batch of sample rows (a Matrix of dense rows or a CpsMatrix) with its
    energies for the vectors Z (m, n_p) (sr_stream_accumulate)."""
    if Z.dtype != torch.float64 or Z.shape != (acc.m, acc.n_p) or not Z.is_contiguous():
        raise ValueError("Z must be a contiguous float64 (m, n_p) tensor")
    c = acc.c()
    if isinstance(batch, CpsMatrix):
        om, cm, n_s = None, ctypes.byref(batch.c()), batch.n_s
    else:
        om, cm, n_s = ctypes.byref(batch.c()), None, batch.O.shape[0]
    if E is not None:
        E = _vec(E, n_s, "E")
    _check(lib().sr_stream_accumulate(ctypes.byref(c), om, cm, _ptr(E), _ptr(Z), _stream(stream)),
           "sr_stream_accumulate")


def sr_stream_finish(acc: StreamAcc, Z: torch.Tensor, eps: float, stream=None) -> dict:
    """(S + eps I) z_i for every vector, g, the column means and <E> of all samples fed
    (sr_stream_finish)."""
    f64 = dict(dtype=torch.float64, device=acc.A.device)
    out = {"Y": torch.empty(acc.m, acc.n_p, **f64), "mean": torch.empty(acc.n_p, **f64)}
    if acc.se is not None:
        out["g"] = torch.empty(acc.n_p, **f64)
        out["E_mean"] = torch.empty(1, **f64)
    c = acc.c()
    _check(lib().sr_stream_finish(ctypes.byref(c), _ptr(Z.contiguous()), float(eps), _ptr(out["Y"]),
                                  _ptr(out.get("g")), _ptr(out["mean"]), _ptr(out.get("E_mean")), _stream(stream)),
           "sr_stream_finish")
    return out


CALLS = {"grad": 0, "sv_product": 1, "cg_solve": 2, "lm_hv_product": 3, "adjoint": 4}


def workspace_bytes(M: Matrix, call: str) -> int:
    """Bytes of the library workspace the call needs on M (sr_workspace_bytes)."""
    m = M.c()
    b = lib().sr_workspace_bytes(ctypes.byref(m), CALLS[call])
    if b < 0:
        raise SrError(int(b), "sr_workspace_bytes")
    return int(b)


def workspace_reserve(nbytes: int, stream=None):
    _check(lib().sr_workspace_reserve(int(nbytes), _stream(stream)), "sr_workspace_reserve")


TIMING_CLASSES = {"search_step": 0, "residual_phase": 1, "solve_launch": 2}


def timing(enable: bool = True):
    """Start (clear) or stop the library's HIP-event timing of CG launches (sr_timing)."""
    _check(lib().sr_timing(1 if enable else 0), "sr_timing")


def timing_read(cls: str) -> tuple:
    """(total ms, launches) recorded for a class of CG launches (sr_timing_read)."""
    ms, n = _c_d(0.0), _c_i64(0)
    _check(lib().sr_timing_read(TIMING_CLASSES[cls], ctypes.byref(ms), ctypes.byref(n)), "sr_timing_read")
    return ms.value, n.value


def workspace_held(stream=None) -> int:
    return int(lib().sr_workspace_held(_stream(stream)))


def lm_hv_product(M: Matrix, E: torch.Tensor, Dm: Matrix, v: torch.Tensor, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """y = H v of the linear method, length n_p + 1 (lm_hv_product)."""
    E = _vec(E, M.O.shape[0], "E")
    v = _vec(v, M.n_p + 1, "v")
    y = torch.empty_like(v) if out is None else out
    m, d = M.c(), Dm.c()
    _check(lib().lm_hv_product(ctypes.byref(m), _ptr(E), ctypes.byref(d), _ptr(v), _ptr(y), _stream(stream)),
           "lm_hv_product")
    return y


BATCH_CONFIGS = [(r, t) for r in (256, 512, 1024) for t in (1, 2, 4)]


def set_batch_config(split_rows: int = 0, tasks: int = 0):
    """Geometry of the batched products (sr_set_batch_config); no arguments: the defaults."""
    _check(lib().sr_set_batch_config(int(split_rows), int(tasks)), "sr_set_batch_config")


def sr_cg_solve_shifts(M: Matrix, g: torch.Tensor, eps, rtol: float = 1e-10, max_iter: int = 0,
                       refresh_every: int = 0,
                       raise_on=(SR_ERR_INVALID, SR_ERR_NOMEM, SR_ERR_HIP, SR_ERR_NODEVICE, SR_ERR_TIMEOUT),
                       stream=None):
    """Multi-shift CG (sr_cg_solve_shifts): X[i] = (S + eps[i] I)^{-1} g for k <= 8 shifts.
    Returns (X (k, n_p), list of per-shift info dicts, status)."""
    g = _vec(g, M.n_p, "g")
    eps = [float(e) for e in eps]
    k = len(eps)
    X = torch.empty(k, M.n_p, dtype=torch.float64, device=g.device)
    arr = (_c_d * max(k, 1))(*eps)
    opts = SrCgOpts()
    opts.rtol = float(rtol)
    opts.max_iter = int(max_iter)
    opts.refresh_every = int(refresh_every)
    infos = (SrCgInfo * max(k, 1))()
    m = M.c()
    st = lib().sr_cg_solve_shifts(ctypes.byref(m), _ptr(g), k, arr, _ptr(X), ctypes.byref(opts), infos,
                                  _stream(stream))
    if st in raise_on:
        raise SrError(st, "sr_cg_solve_shifts")
    out = [{"status": c.status, "iters": c.iters, "refreshes": c.refreshes, "products": c.products,
            "rel_res_recur": c.rel_res_recur, "rel_res_true": c.rel_res_true} for c in infos[:k]]
    return X, out, st


def sr_cg_solve_shifts_batched(systems, rtol: float = 1e-10, max_iter: int = 0, refresh_every: int = 0,
                               raise_on=(SR_ERR_INVALID, SR_ERR_NOMEM, SR_ERR_HIP, SR_ERR_NODEVICE, SR_ERR_TIMEOUT),
                               stream=None):
    """Multi-shift CG of many systems in one launch (sr_cg_solve_shifts_batched).
    `systems` is a list of (Matrix, g, eps) with g a float64 (n_p,) right-hand side and eps a
    list of k shifts (the same k for all).  Returns (list of X tensors (k, n_p), list of
    per-system lists of per-shift info dicts, status)."""
    k = None
    descs = (SrShiftSystem * len(systems))()
    keep, xs = [], []
    for i, (M, g, eps) in enumerate(systems):
        g = _vec(g, M.n_p, "g")
        if k is None:
            k = len(eps)
        elif len(eps) != k:
            raise ValueError("every system needs the same number of shifts")
        X = torch.empty(k, M.n_p, dtype=torch.float64, device=g.device)
        descs[i].O = M.c()
        descs[i].g = g.data_ptr()
        descs[i].X = X.data_ptr()
        for j in range(BATCH_MAX_RHS):
            descs[i].eps[j] = float(eps[j]) if j < k else 0.0
        keep.append(g)
        xs.append(X)
    opts = SrCgOpts()
    opts.rtol = float(rtol)
    opts.max_iter = int(max_iter)
    opts.refresh_every = int(refresh_every)
    infos = (SrCgInfo * (len(systems) * k))()
    st = lib().sr_cg_solve_shifts_batched(len(systems), descs, k, ctypes.byref(opts), infos, _stream(stream))
    if st in raise_on:
        raise SrError(st, "sr_cg_solve_shifts_batched")
    out = [[{"status": infos[i * k + j].status, "iters": infos[i * k + j].iters,
             "products": infos[i * k + j].products, "rel_res_recur": infos[i * k + j].rel_res_recur,
             "rel_res_true": infos[i * k + j].rel_res_true} for j in range(k)] for i in range(len(systems))]
    return xs, out, st


def lm_davidson(M: Matrix, E: torch.Tensor, Dm: Matrix, tol: float = 1e-8, max_iter: int = 1000, max_sub: int = 40,
                precond: int = 0, raise_on=(SR_ERR_INVALID, SR_ERR_NOMEM, SR_ERR_HIP, SR_ERR_NODEVICE, SR_ERR_TIMEOUT), stream=None):
    """Lowest eigenpair of the linear method, H c = theta S c (lm_davidson); precond 0: the
    residual as new direction, 1: approximate, 2: exact diagonal (Davidson) correction.  Returns
    (theta, c [n_p + 1] float64 with c^T S c = 1, info dict)."""
    E = _vec(E, M.O.shape[0], "E")
    c = torch.empty(M.n_p + 1, dtype=torch.float64, device=M.O.device)
    opts = LmDavidsonOpts()
    opts.tol = float(tol)
    opts.max_iter = int(max_iter)
    opts.max_sub = int(max_sub)
    opts.precond = int(precond)
    info = LmDavidsonInfo()
    m, d = M.c(), Dm.c()
    st = lib().lm_davidson(ctypes.byref(m), _ptr(E), ctypes.byref(d), ctypes.byref(opts), _ptr(c), ctypes.byref(info),
                           _stream(stream))
    if st in raise_on:
        raise SrError(st, "lm_davidson")
    return info.theta, c, {"status": st, "iters": info.iters, "restarts": info.restarts, "res_norm": info.res_norm}


def _rhs_block(V: torch.Tensor, n_p: int, name: str) -> torch.Tensor:
    if V.dtype != torch.float64 or V.dim() != 2 or V.shape[1] != n_p or not 1 <= V.shape[0] <= BATCH_MAX_RHS:
        raise ValueError(f"{name} must be a float64 (k, {n_p}) tensor with 1 <= k <= {BATCH_MAX_RHS}")
    return V.contiguous()


def sr_svk_product(M: Matrix, V: torch.Tensor, eps, exact: bool = False, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """Y = (S + diag(eps)) V for the k rows of V (k <= 8 right-hand sides sharing two passes
    over O, float64-accumulated; `exact` is accepted for either value)."""
    V = _rhs_block(V, M.n_p, "V")
    k = V.shape[0]
    eps = [float(e) for e in eps]
    if len(eps) != k:
        raise ValueError("one eps per right-hand side")
    Y = torch.empty_like(V) if out is None else out
    arr = (_c_d * k)(*eps)
    m = M.c()
    _check(lib().sr_svk_product(ctypes.byref(m), k, _ptr(V), arr, _ptr(Y), 1 if exact else 0, _stream(stream)),
           "sr_svk_product")
    return Y


def sr_cg_solve_batched(systems, rtol: float = 1e-10, max_iter: int = 0, refresh_every: int = 0,
                        refresh_drop: float = 0.0,
                        raise_on=(SR_ERR_INVALID, SR_ERR_NOMEM, SR_ERR_HIP, SR_ERR_NODEVICE, SR_ERR_TIMEOUT),
                        stream=None):
    """Solve many systems in one launch (sr_cg_solve_batched).  `systems` is a list of
    (Matrix, G, eps) with G a float64 (k, n_p) tensor of right-hand sides and eps a list of
    k shifts; k must be the same for all.  Returns (list of X tensors (k, n_p), list of
    per-system lists of per-column info dicts, status)."""
    k = None
    descs = (SrBatchSystem * len(systems))()
    keep, xs = [], []
    for i, (M, G, eps) in enumerate(systems):
        G = _rhs_block(G, M.n_p, "G")
        if k is None:
            k = G.shape[0]
        elif G.shape[0] != k:
            raise ValueError("every system needs the same number of right-hand sides")
        if len(eps) != k:
            raise ValueError("one eps per right-hand side")
        X = torch.empty_like(G)
        descs[i].O = M.c()
        descs[i].g = G.data_ptr()
        descs[i].x = X.data_ptr()
        for j in range(BATCH_MAX_RHS):
            descs[i].eps[j] = float(eps[j]) if j < k else 0.0
        keep.append(G)
        xs.append(X)
    opts = SrCgOpts()
    opts.rtol = float(rtol)
    opts.max_iter = int(max_iter)
    opts.refresh_every = int(refresh_every)
    opts.refresh_drop = float(refresh_drop)
    infos = (SrCgInfo * (len(systems) * k))()
    st = lib().sr_cg_solve_batched(len(systems), descs, k, ctypes.byref(opts), infos, _stream(stream))
    if st in raise_on:
        raise SrError(st, "sr_cg_solve_batched")
    out = []
    for i in range(len(systems)):
        out.append([{"iters": infos[i * k + j].iters, "status": infos[i * k + j].status,
                     "products": infos[i * k + j].products, "rel_res_true": infos[i * k + j].rel_res_true}
                    for j in range(k)])
    return xs, out, st


def sr_adjoint(M: Matrix, E: torch.Tensor, x: torch.Tensor, lam: torch.Tensor, dO_dtype=torch.float32,
               want_dE: bool = True, want_p12: bool = False, want_deps: bool = False, stream=None):
    """Gradients through the SR solve (sr_adjoint): returns (dO, dE, p12), or
    (dO, dE, p12, deps) with want_deps; dO is an (n_s, n_p) tensor of dO_dtype (None if
    dO_dtype is None), dE [n_s] float64 or None, p12 [2, n_s] float64 (p1 = Oc x,
    p2 = Oc lambda) or None, deps a 0-d float64 tensor -lambda . x."""
    n_s = M.O.shape[0]
    E = _vec(E, n_s, "E")
    x = _vec(x, M.n_p, "x")
    lam = _vec(lam, M.n_p, "lam")
    dO = dO_arg = None
    code, ld = 0, 0
    if dO_dtype is not None:
        code = _TORCH_DT[dO_dtype]
        vec = 16 // _ELEM[code]
        ld = ((M.n_p + vec - 1) // vec) * vec
        dO_arg = torch.empty(n_s, ld, dtype=dO_dtype, device=E.device)
        dO = dO_arg[:, :M.n_p]
    dE = torch.empty(n_s, dtype=torch.float64, device=E.device) if want_dE else None
    p12 = torch.empty(2, n_s, dtype=torch.float64, device=E.device) if want_p12 else None
    deps = torch.empty((), dtype=torch.float64, device=E.device) if want_deps else None
    m = M.c()
    _check(lib().sr_adjoint(ctypes.byref(m), _ptr(E), _ptr(x), _ptr(lam), _ptr(dE), _ptr(dO_arg), code, ld,
                            _ptr(p12), _ptr(deps), _stream(stream)), "sr_adjoint")
    if want_deps:
        return dO, dE, p12, deps
    return dO, dE, p12


REMAINDER_TOL = {torch.bfloat16: 2.0 ** -17, torch.float16: 2.0 ** -21}


def sr_remainder_columns(O: torch.Tensor, scale: torch.Tensor, out_dtype=torch.bfloat16, tol: float | None = None,
                         stream=None) -> torch.Tensor:
    """Columns whose single-plane codes miss `tol` (default: the two-plane error bound),
    as an increasing int32 tensor (sr_remainder_columns)."""
    Min = as_matrix(O)
    n_s, n_p = O.shape
    cols = torch.empty(n_p, dtype=torch.int32, device=O.device)
    n = _c_i64(0)
    tol = REMAINDER_TOL[out_dtype] if tol is None else float(tol)
    _check(lib().sr_remainder_columns(n_s, n_p, _ptr(Min.O), Min.ld, Min.dtype_code, _TORCH_DT[out_dtype], _ptr(scale),
                                      tol, _ptr(cols), ctypes.byref(n), _stream(stream)), "sr_remainder_columns")
    return cols[: n.value].clone()


def sr_quantize_remainder(O: torch.Tensor, scale: torch.Tensor, lo_cols: torch.Tensor, out_dtype=torch.bfloat16,
                          stream=None) -> torch.Tensor:
    """The compact remainder plane of the columns lo_cols, (n_s, n_lo) codes viewed from an
    (n_s, ld_lo) tensor (sr_quantize_remainder)."""
    Min = as_matrix(O)
    n_s, n_p = O.shape
    n_lo = lo_cols.numel()
    ld_lo = max(8, ((n_lo + 7) // 8) * 8)
    q_lo = torch.empty(n_s, ld_lo, dtype=out_dtype, device=O.device)
    _check(lib().sr_quantize_remainder(n_s, n_p, _ptr(Min.O), Min.ld, Min.dtype_code, _TORCH_DT[out_dtype],
                                       _ptr(scale), _ptr(lo_cols.to(torch.int32).contiguous()), n_lo, _ptr(q_lo),
                                       ld_lo, _stream(stream)), "sr_quantize_remainder")
    return q_lo[:, :n_lo]


def sr_quantize(O: torch.Tensor, out_dtype=torch.bfloat16, with_lo: bool = False, stream=None):
    """bf16/f16 codes with per-column float32 scales (sr_quantize).  Returns (q, scale), or
    (q, scale, lo) with the second code plane; codes are (n_s, ld) tensors viewed as
    (n_s, n_p).  with_lo="compact" gives (q, scale, lo, lo_cols): the remainder plane of the
    columns that need it only (sr_remainder_columns, sr_quantize_remainder)."""
    if with_lo == "compact":
        q, s = sr_quantize(O, out_dtype, False, stream)
        cols = sr_remainder_columns(O, s, out_dtype, stream=stream)
        return q, s, sr_quantize_remainder(O, s, cols, out_dtype, stream=stream), cols
    if O.dtype not in (torch.float64, torch.float32) or O.dim() != 2:
        raise ValueError("O must be a 2-D float64/float32 tensor")
    Min = as_matrix(O)
    n_s, n_p = O.shape
    ld_out = ((n_p + 7) // 8) * 8
    q = torch.empty(n_s, ld_out, dtype=out_dtype, device=O.device)
    qlo = torch.empty(n_s, ld_out, dtype=out_dtype, device=O.device) if with_lo else None
    s = torch.empty(n_p, dtype=torch.float32, device=O.device)
    ld_in = Min.ld
    st = lib().sr_quantize(n_s, n_p, _ptr(Min.O), ld_in, Min.dtype_code, _ptr(q), _ptr(qlo), ld_out,
                           _TORCH_DT[out_dtype], _ptr(s), _stream(stream))
    _check(st, "sr_quantize")
    if with_lo:
        return q[:, :n_p], s, qlo[:, :n_p]
    return q[:, :n_p], s


def tile_configs(dtype=torch.float64, kind: int = 0) -> list:
    """Tile configurations (nv, rows, lookahead, poll_delay, threads) built for a storage
    type; the first is the default."""
    code = _TORCH_DT[dtype]
    n = lib().sr_tile_configs(code, kind, None, 0)
    arr = (ctypes.c_int32 * (5 * max(n, 1)))()
    lib().sr_tile_configs(code, kind, arr, n)
    return [tuple(arr[5 * i:5 * i + 5]) for i in range(n)]


def set_tile_config(dtype=None, kind: int = 0, nv: int = 0, rows: int = 0, lookahead: int = 0,
                    poll_delay: int = 0, threads: int = 0, col_groups: int = 0):
    """Override the product tile configuration for one storage type and product kind
    (nv = 0: automatic).  set_tile_config() with no arguments restores every automatic
    choice."""
    code = -1 if dtype is None else _TORCH_DT[dtype]
    _check(lib().sr_set_tile_config(code, kind, nv, rows, lookahead, poll_delay, threads, col_groups),
           "sr_set_tile_config")


def release():
    return lib().sr_release()


def stream_read(t: torch.Tensor, blocks_per_cu: int = 2, unroll: int = 4, stream=None) -> torch.Tensor:
    """Read all of t's bytes once with the products' streaming loads (sr_stream_read);
    returns the per-workgroup folded words (to keep the loads)."""
    nbytes = (t.numel() * t.element_size()) // 16 * 16
    cus = torch.cuda.get_device_properties(t.device).multi_processor_count
    sink = torch.empty(cus * blocks_per_cu, dtype=torch.int32, device=t.device)
    _check(lib().sr_stream_read(_ptr(t), nbytes, int(blocks_per_cu), int(unroll), _ptr(sink), _stream(stream)),
           "sr_stream_read")
    return sink
