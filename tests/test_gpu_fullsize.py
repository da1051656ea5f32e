"""The headline workload at its full size, in the launch configuration the bench times:
CPS-shaped O, 32768 samples x 500000 parameters, stored as bf16 codes with float32 column
scales plus a bf16 remainder plane (compact: only the columns that need it; or full),
against float64 storage of the same matrix.

At this size the CPU oracle cannot run (131 GB of float64), so the checks are properties
that hold at any size and compare two different kernels and storage forms: the two-plane
product against the float64 product (the two planes carry about 16 significant bits, so
the products agree to ~1e-5), and the bf16 CG solution (rtol 1e-6) against the
float64 CG solution (rtol 1e-10) to the 1e-4 accuracy target of the precision form,
each ending on its own true residual.  Element-wise oracle parity of the same kernels
runs at smaller sizes in test_gpu_parity.py."""
from __future__ import annotations

import pytest
import torch

import synth
from paper_1108_0900_amd import sr
from tests.gpu_util import DEV

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form", ["compact", "two_planes"])
def test_headline_bf16_full_size(form):
    cfg = synth.CONFIGS["cps_32768x500000"]
    d = synth.cps_inputs(cfg.n_s, cfg.n_corr, cfg.n_states, cfg.n_dense, cfg.seed, device=DEV)
    O64, E = d["O"], d["E"]
    if form == "compact":
        q, s, lo, cols = sr.sr_quantize(O64, out_dtype=torch.bfloat16, with_lo="compact")
        # the 8480 dense pairing columns need a remainder code, the CPS columns do not
        assert torch.equal(cols.cpu(), torch.arange(cfg.n_corr * cfg.n_states, cfg.n_p, dtype=torch.int32))
        M2 = sr.as_matrix(q, scale=s, lo=lo, lo_cols=cols)
    else:
        q, s, lo = sr.sr_quantize(O64, out_dtype=torch.bfloat16, with_lo=True)
        M2 = sr.as_matrix(q, scale=s, lo=lo)
    M64 = sr.as_matrix(O64)
    st2, st64 = sr.sr_grad(M2, E), sr.sr_grad(M64, E)
    M2.mean, M64.mean = st2["mean"], st64["mean"]
    g2, g64 = st2["g"], st64["g"]
    assert float(torch.linalg.vector_norm(g2 - g64) / torch.linalg.vector_norm(g64)) <= 1e-4
    eps2 = 1e-3 * float(st2["diag"].mean())
    eps64 = 1e-3 * float(st64["diag"].mean())
    assert abs(eps2 - eps64) <= 1e-4 * eps64
    # products
    gen = torch.Generator(device=DEV)
    gen.manual_seed(17)
    v = torch.randn(cfg.n_p, generator=gen, dtype=torch.float64, device=DEV)
    y2 = sr.sr_sv_product(M2, v, eps64)
    y64 = sr.sr_sv_product(M64, v, eps64)
    dy = float(torch.linalg.vector_norm(y2 - y64) / torch.linalg.vector_norm(y64))
    print(f"[full] product rel diff {dy:.2e}", flush=True)
    assert dy <= 1e-4
    # solves
    x2, i2 = sr.sr_cg_solve(M2, g2, eps2, rtol=1e-6, refresh_every=cfg.refresh_every)
    x64, i64 = sr.sr_cg_solve(M64, g64, eps64, rtol=1e-10, refresh_every=cfg.refresh_every)
    assert i2["status"] == 0 and i2["rel_res_true"] <= 1e-6, i2
    assert i64["status"] == 0 and i64["rel_res_true"] <= 1e-10, i64
    err = float(torch.linalg.vector_norm(x2 - x64) / torch.linalg.vector_norm(x64))
    print(f"[full] bf16 {form} solve: {i2}, error vs float64 {err:.2e}", flush=True)
    assert err <= 1e-4
    del O64, q, lo, d
