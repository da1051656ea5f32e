"""Products during sampling (sr_stream_*) against the oracle on all the samples fed.

Batches come from the seeded per-batch generator (synth.cps_stream_batch: index-coded CPS
rows; dense rows are the same batches expanded by the oracle and stored densely, in float64
or as bf16 codes).  The oracle concatenates the batches the device saw (copied to the host),
expands them with cps_expand, and applies its plain definitions to the whole sample set.

Tolerance: the stream sums are uncentred and centred at the end, so the rounding of a
column's product is relative to the uncentred magnitude (|O|^T |O| |z| + |obar| (|O| |z|)) / n,
as for float32 accumulation in gpu_util.magnitude_ref; 1e-12 of that for float64 rows.
"""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from paper_1108_0900_amd import sr
from tests.gpu_util import DEV, magnitude_ref, rel_err, stored_dense, to_dev, to_np

pytestmark = pytest.mark.gpu

SIZES = (700, 700, 512, 333)       # ragged last batch


def _batches(layout, dense_dtype=torch.float64):
    for b, n in enumerate(SIZES):
        yield synth.cps_stream_batch(layout, b, n, device=DEV, dense_dtype=dense_dtype)


def _oracle_rows(layout, batches_host, dense_code=None):
    Os, Es = [], []
    for bh in batches_host:
        dv = bh["dense"]
        if dense_code is not None and dv is not None:
            dv = stored_dense(dv, dense_code)
        Os.append(orc.cps_expand(bh["idx"], layout["val"].cpu().numpy(), layout["n_states"], dv))
        Es.append(bh["E"])
    return np.concatenate(Os), np.concatenate(Es)


@pytest.mark.parametrize("form", ["cps", "dense_f64", "dense_bf16"])
def test_stream_products_match_oracle(form):
    layout = synth.cps_stream_layout(7, 12, 40, 31, device=DEV)
    n_p = 7 * 12 + 40
    m = 3
    Z = torch.from_numpy(np.random.default_rng(5).standard_normal((m, n_p))).to(DEV)
    acc = sr.sr_stream_begin(n_p, m, device=DEV)
    seen = []
    for b in _batches(layout):
        if form == "cps":
            batch = sr.cps_matrix(b["idx"], layout["val"], 12, b["dense"])
            host = {"idx": b["idx"].cpu().numpy(), "dense": b["dense"].cpu().numpy(), "E": b["E"].cpu().numpy()}
        else:
            O = orc.cps_expand(b["idx"].cpu().numpy(), layout["val"].cpu().numpy(), 12, b["dense"].cpu().numpy())
            host = {"idx": b["idx"].cpu().numpy(), "dense": b["dense"].cpu().numpy(), "E": b["E"].cpu().numpy()}
            if form == "dense_f64":
                batch = sr.as_matrix(to_dev(O))
            else:
                q, s = sr.sr_quantize(to_dev(O), out_dtype=torch.bfloat16)
                batch = sr.as_matrix(q, scale=s)
                host["O"] = orc.dequantize_bf16(*orc.quantize_bf16(O))
        sr.sr_stream_accumulate(acc, batch, b["E"], Z)
        seen.append(host)
        del batch, b
    eps = 0.21
    out = sr.sr_stream_finish(acc, Z, eps)
    if form == "dense_bf16":
        O_all = np.concatenate([h["O"] for h in seen])
        E_all = np.concatenate([h["E"] for h in seen])
    else:
        O_all, E_all = _oracle_rows(layout, seen)
    assert O_all.shape == (sum(SIZES), n_p)
    tol = 1e-12 if form != "dense_bf16" else 2e-5
    Zh = to_np(Z)
    for i in range(m):
        ref = orc.sv_product_swapped(O_all, Zh[i], eps)
        mag = magnitude_ref(O_all, Zh[i], eps, torch.bfloat16)
        err = (np.abs(to_np(out["Y"][i]) - ref) / mag).max()
        print(f"[stream {form}] vector {i}: worst error / magnitude {err:.2e}", flush=True)
        assert err <= tol, err
    np.testing.assert_allclose(to_np(out["mean"]), orc.sample_mean(O_all), rtol=1e-12, atol=1e-14)
    g_ref = orc.energy_gradient(O_all, E_all)
    gscale = (np.abs(O_all).T @ np.abs(E_all)) * 2 / O_all.shape[0]
    assert (np.abs(to_np(out["g"]) - g_ref) / gscale).max() <= 1e-12
    assert abs(float(out["E_mean"]) - E_all.mean()) <= 1e-13 * abs(E_all.mean())


def test_stream_equals_stored_product_and_repeats_bit_for_bit():
    """Streaming the batches again (regenerated from the seed) gives the same bits; the
    result equals the product over the stored, concatenated index-coded matrix."""
    layout = synth.cps_stream_layout(20, 30, 64, 47, device=DEV)
    n_p = 20 * 30 + 64
    Z = torch.from_numpy(np.random.default_rng(6).standard_normal((1, n_p))).to(DEV)
    outs = []
    for _ in range(2):
        acc = sr.sr_stream_begin(n_p, 1, device=DEV)
        for b in _batches(layout):
            sr.sr_stream_accumulate(acc, sr.cps_matrix(b["idx"], layout["val"], 30, b["dense"]), b["E"], Z)
        outs.append(sr.sr_stream_finish(acc, Z, 0.05))
    torch.cuda.synchronize()
    assert torch.equal(outs[0]["Y"], outs[1]["Y"]) and torch.equal(outs[0]["g"], outs[1]["g"])
    bs = list(_batches(layout))
    n = sum(SIZES)
    idx = torch.full((20, ((n + 15) // 16) * 16), 255, dtype=torch.uint8, device=DEV)
    idx[:, :n] = torch.cat([b["idx"] for b in bs], dim=1)
    M = sr.cps_matrix(idx[:, :n], layout["val"], 30, torch.cat([b["dense"] for b in bs]))
    E = torch.cat([b["E"] for b in bs])
    st = sr.sr_cps_grad(M, E)
    M.mean = st["mean"]
    y = sr.sr_cps_sv_product(M, Z[0].contiguous(), 0.05)
    assert rel_err(to_np(outs[0]["Y"][0]), to_np(y)) <= 1e-12
    assert rel_err(to_np(outs[0]["g"]), to_np(st["g"])) <= 1e-12
