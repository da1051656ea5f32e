"""Helpers shared by the GPU tests: inputs on the device, oracle references in float64.

Tolerances, derived from the arithmetic of each storage mode, on the element-wise
error relative to the magnitude reference M_i = (|Oc|^T |Oc| |v|)_i / N + eps |v_i|
(the value the product would have if no term cancelled; see magnitude_ref for the
uncentred form used with float32 accumulation):
  * float64 / float32 storage: every term and sum is float64 (u = 2^-53); sums of
    n <= 1e5 terms in any order stay within n u M_i ~ 1e-11 M_i in the worst case and
    ~sqrt(n) u M_i typically, so 1e-12 M_i is used for the sizes tested here.
  * bf16 / f16 storage: dots and O^T w accumulate in float32 (u = 2^-24 = 6e-8) with tree
    reductions across lanes, waves and workgroups, and a sequential sum over the rows a
    thread owns; 2e-5 M_i covers up to ~1e5 rows at ~sqrt(n) u growth.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle as orc
from paper_1108_0900_amd import sr

DEV = "cuda:0"
TOL_PRODUCT = {torch.float64: 1e-12, torch.float32: 1e-12, torch.bfloat16: 2e-5, torch.float16: 2e-5}


def stored_dense(O64: np.ndarray, dtype) -> np.ndarray:
    """The float64 values a storage mode represents, computed by the oracle alone."""
    if dtype == torch.float64:
        return O64
    if dtype == torch.float32:
        return O64.astype(np.float32).astype(np.float64)
    if dtype == torch.bfloat16:
        q, s = orc.quantize_bf16(O64)
        return orc.dequantize_bf16(q, s)
    if dtype == torch.float16:
        q, s = orc.quantize_f16(O64)
        return orc.dequantize_f16(q, s)
    raise ValueError(dtype)


def device_matrix(O64: np.ndarray, dtype, ld: int | None = None, pad_value=float("nan"), with_mean=None):
    """Put O on the GPU in the given storage mode; float64/float32 directly, bf16/f16 via
    the library's quantizer.  `ld` > n_p makes a padded row stride filled with pad_value."""
    n_s, n_p = O64.shape
    src = torch.from_numpy(O64).to(DEV)
    if dtype in (torch.bfloat16, torch.float16):
        q, s = sr.sr_quantize(src, out_dtype=dtype)
        if ld is not None and ld != q.stride(0):
            Q = torch.empty(n_s, ld, dtype=dtype, device=DEV)
            Q.view(torch.int16)[:] = -1       # NaN pattern in the padding
            Q[:, :n_p] = q
            q = Q[:, :n_p]
        return sr.as_matrix(q, scale=s, mean=with_mean)
    t = src.to(dtype)
    if ld is not None:
        P = torch.full((n_s, ld), pad_value, dtype=dtype, device=DEV)
        P[:, :n_p] = t
        t = P[:, :n_p]
    return sr.as_matrix(t, mean=with_mean)


def magnitude_ref(Ostore: np.ndarray, v: np.ndarray, eps: float, dtype=torch.float64) -> np.ndarray:
    """Magnitude reference of (S + eps I) v.  float64 arithmetic: |Oc|^T |Oc| |v| / N.
    float32 accumulation (scaled storage) folds the centering in after the sums, so its
    rounding scales with the uncentred values: (|O|^T |O||v| + |obar| sum_k (|O||v|)_k) / N."""
    n = Ostore.shape[0]
    if dtype in (torch.bfloat16, torch.float16):
        A = np.abs(Ostore)
        t = A @ np.abs(v)
        return (A.T @ t + np.abs(orc.sample_mean(Ostore)) * t.sum()) / n + eps * np.abs(v)
    Oc = np.abs(orc.centred(Ostore))
    return Oc.T @ (Oc @ np.abs(v)) / n + eps * np.abs(v)


def rel_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rand_dense(n_s, n_p, seed, offset=0.0):
    rng = np.random.default_rng(seed)
    s = np.exp(0.5 * rng.standard_normal(n_p))
    O = rng.standard_normal((n_s, n_p)) * s + offset
    u = rng.standard_normal(n_p) / np.sqrt(n_p)
    E = -20.0 + 0.3 * (O @ u) + rng.standard_normal(n_s)
    return O, E


def to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()
