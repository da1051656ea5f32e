"""The entry point that allocates nothing (sr_sv_product_noalloc) against sr_sv_product:
the same kernels over the library's fixed scratch instead of its workspace, so the
results must agree bit for bit.  Two calls in a row, the second on a smaller matrix (the
scratch keeps the first call's contents), for float64 storage and for bf16 codes with a
compact remainder plane."""
import numpy as np
import pytest
import torch

import synth
from paper_1108_0900_amd import sr
from tests.gpu_util import DEV, rand_dense, to_dev

pytestmark = pytest.mark.gpu


def _f64(n_s, n_p, seed):
    O, _ = rand_dense(n_s, n_p, seed=seed, offset=0.3)
    M = sr.as_matrix(to_dev(O))
    M.mean = sr.sr_grad(M, None)["mean"]
    return M


def _compact(n_s, n_corr, n_dense, seed):
    d = synth.cps_inputs(n_s, n_corr, 240, n_dense, seed, device=DEV)
    q, s, lo, cols = sr.sr_quantize(d["O"], out_dtype=torch.bfloat16, with_lo="compact")
    M = sr.as_matrix(q, scale=s, lo=lo, lo_cols=cols)
    M.mean = sr.sr_grad(M, None)["mean"]
    return M


@pytest.mark.parametrize("kind", ["f64", "bf16_compact"])
def test_noalloc_product_equals_workspace_product(kind):
    if kind == "f64":
        cases = [_f64(3000, 70001, 1), _f64(257, 4099, 2)]
    else:
        cases = [_compact(1024, 1500, 9000, 3), _compact(300, 40, 1000, 4)]
    for i, M in enumerate(cases):
        print(f"[noalloc] {kind} call {i}: {M.O.shape[0]} x {M.n_p}", flush=True)
        v = torch.randn(M.n_p, dtype=torch.float64, device=DEV, generator=torch.Generator(DEV).manual_seed(i))
        y_ref = sr.sr_sv_product(M, v, 0.05)
        y = torch.full_like(v, float("nan"))
        sr.sr_sv_product_noalloc(M, v, 0.05, out=y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), float((y - y_ref).abs().max())


def test_noalloc_requires_column_means():
    O, _ = rand_dense(50, 30, seed=5)
    M = sr.as_matrix(to_dev(O))
    with pytest.raises(ValueError):
        sr.sr_sv_product_noalloc(M, to_dev(np.ones(30)), 0.1, out=torch.empty(30, dtype=torch.float64, device=DEV))
    m = M.c()
    import ctypes
    y = torch.empty(30, dtype=torch.float64, device=DEV)
    v = to_dev(np.ones(30))
    st = sr.lib().sr_sv_product_noalloc(ctypes.byref(m), ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                        0.1, None)
    assert st == sr.SR_ERR_INVALID
