"""GPU parity of the precision forms against the FP64 CPU oracle.

* Compact remainder plane: bf16/f16 codes for every column plus a second code only for
  the columns whose single-plane error exceeds the two-plane bound.  Column selection and
  codes are compared bit for bit; products, the prepare pass and CG against the oracle's
  dense solve of the stored (dequantized) values, including the 500,000-column shape of
  the headline workload (64 column groups of the fused product) through the oracle's dual
  solve.
* Full second plane: product and CG at the headline's column count.
* Non-finite input and the float64 residual refresh of the one-plane solve.

Tolerances: products accumulate in float32 over the streamed codes (2e-5 of the magnitude
reference, as for one plane), residual products in float64; a CG solution is compared
with the dense solution of the stored system at what the true residual it reports allows
(||x - x*|| / ||x*|| <= kappa ||r|| / ||g||, kappa from the oracle's eigenvalues where the
matrix is small enough).
"""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from paper_1108_0900_amd import sr
from tests.gpu_util import DEV, TOL_PRODUCT, magnitude_ref, rand_dense, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

CODES = {torch.bfloat16: "bf16", torch.float16: "f16"}


def _dname(dt):
    return str(dt).split(".")[-1]


def _bits(t: torch.Tensor) -> np.ndarray:
    return t.contiguous().view(torch.int16).cpu().numpy().view(np.uint16)


def _cps_permuted(n_s, n_corr, n_states, n_dense, seed):
    """CPS-shaped O with its columns shuffled, so that the columns needing a remainder
    code are scattered over the matrix."""
    d = synth.cps_inputs(n_s, n_corr, n_states, n_dense, seed)
    O, E = d["O"].numpy(), d["E"].numpy()
    perm = np.random.default_rng(seed).permutation(O.shape[1])
    return np.ascontiguousarray(O[:, perm]), E


def _compact_matrix(O, dtype, with_mean=None):
    q, s, lo, cols = sr.sr_quantize(torch.from_numpy(O).to(DEV), out_dtype=dtype, with_lo="compact")
    return sr.as_matrix(q, scale=s, lo=lo, lo_cols=cols, mean=with_mean), cols, lo


CASES = {
    "dense300x2049": lambda: rand_dense(300, 2049, seed=5, offset=0.5),
    "cps1500x1061": lambda: _cps_permuted(1500, 8, 120, 101, seed=6),
    "cps37x9999": lambda: _cps_permuted(37, 40, 240, 399, seed=7),
    "dense5x7": lambda: rand_dense(5, 7, seed=8),
}


@pytest.mark.parametrize("dtype", list(CODES), ids=_dname)
@pytest.mark.parametrize("case", list(CASES))
def test_remainder_columns_and_codes_bit_exact(case, dtype):
    O, _ = CASES[case]()
    print(f"[compact-codes] {case} {dtype}", flush=True)
    M, cols, lo = _compact_matrix(O, dtype)
    q_hi, s, cols_ref, lo_ref = orc.quantize_cols(O, CODES[dtype])
    assert np.array_equal(to_np(cols).astype(np.int64), cols_ref)
    assert np.array_equal(to_np(M.scale), s)
    assert np.array_equal(_bits(M.O), q_hi)
    assert np.array_equal(_bits(lo), lo_ref)
    if case.startswith("cps"):
        # the CPS columns hold one value each and are exact with one plane
        assert 0 < cols_ref.size < O.shape[1]


@pytest.mark.parametrize("dtype", list(CODES), ids=_dname)
@pytest.mark.parametrize("case", list(CASES))
def test_compact_product_and_grad_match_oracle(case, dtype):
    O, E = CASES[case]()
    n_s, n_p = O.shape
    print(f"[compact-product] {case} {dtype}", flush=True)
    Os = orc.dequantize_cols(*orc.quantize_cols(O, CODES[dtype]), CODES[dtype])
    M, _, _ = _compact_matrix(O, dtype)
    st = sr.sr_grad(M, to_dev(E))
    np.testing.assert_allclose(to_np(st["mean"]), orc.sample_mean(Os), rtol=1e-12, atol=1e-12 * np.abs(Os).max())
    dref = orc.diag_overlap(Os)
    assert np.all(np.abs(to_np(st["diag"]) - dref) <= 1e-11 * (dref + np.abs(orc.centred(Os)).max(0) ** 2 * 1e-3))
    gref = orc.energy_gradient(Os, E)
    gmag = 2 * np.abs(orc.centred(Os)).T @ np.abs(E - E.mean()) / n_s
    assert np.all(np.abs(to_np(st["g"]) - gref) <= 1e-12 * gmag + 1e-300)
    v = np.random.default_rng(3).standard_normal(n_p)
    for mean in (None, st["mean"]):           # column means computed by the call, or given
        M.mean = mean
        y = to_np(sr.sr_sv_product(M, to_dev(v), 0.02))
        ref = orc.sv_product_swapped(Os, v, 0.02)
        mag = magnitude_ref(Os, v, 0.02, dtype)
        assert np.all(np.abs(y - ref) <= TOL_PRODUCT[dtype] * mag + 1e-300), float(np.max(np.abs(y - ref) / mag))


@pytest.mark.parametrize("search_f64", [False, True], ids=["f32_search", "f64_search"])
@pytest.mark.parametrize("dtype", list(CODES), ids=_dname)
def test_cg_compact_matches_stored_system(dtype, search_f64):
    """CG over the compact plane (float32 or float64 search products, float64 refreshes)
    reaches the dense solution of the stored system, and is within the two-plane accuracy
    of the float64 solution."""
    O, E = _cps_permuted(2048, 16, 240, 530, seed=21)
    Os = orc.dequantize_cols(*orc.quantize_cols(O, CODES[dtype]), CODES[dtype])
    M, _, _ = _compact_matrix(O, dtype)
    st = sr.sr_grad(M, to_dev(E))
    M.mean = st["mean"]
    eps = 1e-3 * float(st["diag"].mean())
    x, info = sr.sr_cg_solve(M, st["g"], eps, rtol=1e-10, refresh_every=20, search_f64=search_f64)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-10, info
    g_ref = orc.energy_gradient(Os, E)
    eps_ref = 1e-3 * orc.diag_overlap(Os).mean()
    x_ref = orc.solve_dense(Os, g_ref, eps_ref)
    lam = np.linalg.eigvalsh(orc.overlap_matrix(Os))
    kappa = (lam[-1] + eps_ref) / (max(lam[0], 0.0) + eps_ref)
    err = rel_err(to_np(x), x_ref)
    assert err <= kappa * 2e-10, (err, kappa, info)
    x64 = orc.solve_dense(O, orc.energy_gradient(O, E), 1e-3 * orc.diag_overlap(O).mean())
    assert rel_err(to_np(x), x64) <= 1e-4, rel_err(to_np(x), x64)


def _headline_shaped(n_s, seed):
    """CPS-shaped rows of the 500,000-parameter workload: 2048 correlators x 240 states and
    8480 dense pairing columns."""
    d = synth.cps_inputs(n_s, 2048, 240, 8480, seed)
    return d["O"].numpy(), d["E"].numpy()


@pytest.mark.slow
def test_compact_product_headline_width():
    n_s = 37
    O, E = _headline_shaped(n_s, seed=31)
    print("[compact-500k] product", flush=True)
    Os = orc.dequantize_cols(*orc.quantize_cols(O, "bf16"), "bf16")
    M, cols, _ = _compact_matrix(O, torch.bfloat16)
    assert np.array_equal(to_np(cols), np.arange(491520, 500000))
    v = np.random.default_rng(4).standard_normal(O.shape[1])
    y = to_np(sr.sr_sv_product(M, to_dev(v), 0.01))
    ref = orc.sv_product_swapped(Os, v, 0.01)
    mag = magnitude_ref(Os, v, 0.01, torch.bfloat16)
    assert np.all(np.abs(y - ref) <= TOL_PRODUCT[torch.bfloat16] * mag + 1e-300), float(np.max(np.abs(y - ref) / mag))


@pytest.mark.slow
@pytest.mark.parametrize("form", ["compact", "two_planes"])
def test_cg_headline_width_matches_dual_solve(form):
    """CG at the headline's 500,000 columns (the fused product's 64 column groups) against
    the oracle's exact dual solve of the stored system, every product float64-accumulated.
    With N_s << N_p, S + eps I is eps (about 1e-6 of S's nonzero eigenvalues) on the null
    space of S; the solution and the Krylov space lie in the range of S, where the system
    is well conditioned, so rtol 1e-11 gives an error near 1e-11.  Then the float32 search
    products of the compact plane at the workload's rtol 1e-6: the oracle's product gives
    the true residual of that solution."""
    n_s = 301
    O, E = _headline_shaped(n_s, seed=32)
    print(f"[cg-500k] {form}", flush=True)
    if form == "compact":
        Os = orc.dequantize_cols(*orc.quantize_cols(O, "bf16"), "bf16")
        M, _, _ = _compact_matrix(O, torch.bfloat16)
    else:
        Os = orc.dequantize_split(*orc.quantize_split(O, "bf16"), "bf16")
        q, s, lo = sr.sr_quantize(torch.from_numpy(O).to(DEV), out_dtype=torch.bfloat16, with_lo=True)
        M = sr.as_matrix(q, scale=s, lo=lo)
    st = sr.sr_grad(M, to_dev(E))
    M.mean = st["mean"]
    g_ref = orc.energy_gradient(Os, E)
    gmag = 2 * np.abs(orc.centred(Os)).T @ np.abs(E - E.mean()) / n_s
    assert np.all(np.abs(to_np(st["g"]) - g_ref) <= 1e-12 * gmag + 1e-300)
    eps_ref = 1e-3 * orc.diag_overlap(Os).mean()
    eps = 1e-3 * float(st["diag"].mean())
    assert abs(eps - eps_ref) <= 1e-12 * eps_ref
    x, info = sr.sr_cg_solve(M, st["g"], eps, rtol=1e-11, refresh_every=20, search_f64=True)
    assert info["status"] == 0, info
    x_ref = orc.solve_dual(Os, g_ref, eps_ref)
    # kappa of S + eps I from the nonzero eigenvalues of S (those of the N_s x N_s Gram
    # matrix): a residual component on the null space of S is eps times the error there
    Oc = orc.centred(Os)
    lam_max = np.linalg.eigvalsh(Oc @ Oc.T / n_s)[-1]
    kappa = (lam_max + eps_ref) / eps_ref
    err = rel_err(to_np(x), x_ref)
    print(f"[cg-500k] {form} float64 search: {info}, error {err:.2e}, kappa {kappa:.2e}", flush=True)
    assert err <= 2 * kappa * info["rel_res_true"], (err, kappa, info)
    if form == "compact":
        x, info = sr.sr_cg_solve(M, st["g"], eps, rtol=1e-6, refresh_every=20)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-6, info
        r = g_ref - orc.sv_product_swapped(Os, to_np(x), eps_ref)
        assert np.linalg.norm(r) <= 2e-6 * np.linalg.norm(g_ref)
        print(f"[cg-500k] float32 search at rtol 1e-6: {info}, error {rel_err(to_np(x), x_ref):.2e}", flush=True)


@pytest.mark.slow
def test_two_plane_product_headline_width():
    n_s = 37
    O, _ = _headline_shaped(n_s, seed=33)
    print("[two-plane-500k] product", flush=True)
    Os = orc.dequantize_split(*orc.quantize_split(O, "bf16"), "bf16")
    q, s, lo = sr.sr_quantize(torch.from_numpy(O).to(DEV), out_dtype=torch.bfloat16, with_lo=True)
    M = sr.as_matrix(q, scale=s, lo=lo)
    v = np.random.default_rng(5).standard_normal(O.shape[1])
    y = to_np(sr.sr_sv_product(M, to_dev(v), 0.01))
    ref = orc.sv_product_swapped(Os, v, 0.01)
    # float64 accumulation of the two-plane values
    assert np.all(np.abs(y - ref) <= 1e-12 * magnitude_ref(Os, v, 0.01) + 1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=_dname)
def test_cg_nan_in_O_reports_nonfinite(dtype):
    """A NaN inside O reaches the products; CG stops with SR_ERR_NONFINITE."""
    O, E = rand_dense(200, 150, seed=43)
    g = orc.energy_gradient(O, E)             # finite: from the clean matrix
    O[17, 33] = np.nan
    src = torch.from_numpy(O).to(DEV)
    if dtype == torch.bfloat16:
        q, s = sr.sr_quantize(src, out_dtype=dtype)
        M = sr.as_matrix(q, scale=s, mean=torch.zeros(150, dtype=torch.float64, device=DEV))
    else:
        M = sr.as_matrix(src.to(dtype), mean=torch.zeros(150, dtype=torch.float64, device=DEV))
    x, info = sr.sr_cg_solve(M, to_dev(g), 1e-3, rtol=1e-10)
    assert info["status"] == sr.SR_ERR_NONFINITE, info


@pytest.mark.parametrize("dtype", list(CODES), ids=_dname)
def test_cg_one_plane_float64_refresh_reaches_rtol(dtype):
    """One code plane: float32 search products, float64 refreshes.  The solution meets the
    requested true residual of the stored system (checked by the oracle's product), and its
    error against the dense solution is within kappa times that residual."""
    n_s, n_p = 2000, 1500
    O, E = rand_dense(n_s, n_p, seed=31)
    code = CODES[dtype]
    Os = orc.dequantize_bf16(*orc.quantize_bf16(O)) if code == "bf16" else orc.dequantize_f16(*orc.quantize_f16(O))
    q, s = sr.sr_quantize(torch.from_numpy(O).to(DEV), out_dtype=dtype)
    M = sr.as_matrix(q, scale=s)
    st = sr.sr_grad(M, to_dev(E))
    M.mean = st["mean"]
    eps = 1e-3 * float(st["diag"].mean())
    rtol = 1e-10
    x, info = sr.sr_cg_solve(M, st["g"], eps, rtol=rtol, refresh_every=20)
    assert info["status"] == 0, info
    g_ref = orc.energy_gradient(Os, E)
    eps_ref = 1e-3 * orc.diag_overlap(Os).mean()
    r = g_ref - orc.sv_product_swapped(Os, to_np(x), eps_ref)
    assert np.linalg.norm(r) <= 2 * rtol * np.linalg.norm(g_ref), np.linalg.norm(r) / np.linalg.norm(g_ref)
    lam = np.linalg.eigvalsh(orc.overlap_matrix(Os))
    kappa = (lam[-1] + eps_ref) / (lam[0] + eps_ref)
    x_ref = orc.solve_dense(Os, g_ref, eps_ref)
    assert rel_err(to_np(x), x_ref) <= 2 * kappa * rtol, (rel_err(to_np(x), x_ref), kappa)


def test_autotune_on_cg_with_compact_plane(tmp_path):
    """Tiles of scaled storage timed on a short CG solve over the compact plane: a built
    configuration is selected and cached, and the solve with it matches the oracle."""
    from paper_1108_0900_amd import tune
    O, E = _cps_permuted(600, 12, 240, 300, seed=51)
    M, _, _ = _compact_matrix(O, torch.bfloat16)
    cache = str(tmp_path / "tune.json")
    try:
        res = tune.autotune(M, kind=0, reps=2, cache_path=cache, cg_iters=3)
        assert res["best"][:5] in sr.tile_configs(torch.bfloat16, 0) and not res["cached"]
        again = tune.autotune(M, kind=0, cache_path=cache, cg_iters=3)
        assert again["cached"] and again["best"] == res["best"]
        Os = orc.dequantize_cols(*orc.quantize_cols(O, "bf16"), "bf16")
        st = sr.sr_grad(M, to_dev(E))
        M.mean = st["mean"]
        eps = 1e-2 * float(st["diag"].mean())
        x, info = sr.sr_cg_solve(M, st["g"], eps, rtol=1e-8, refresh_every=20)
        assert info["status"] == 0, info
        g_ref = orc.energy_gradient(Os, E)
        r = g_ref - orc.sv_product_swapped(Os, to_np(x), 1e-2 * orc.diag_overlap(Os).mean())
        assert np.linalg.norm(r) <= 2e-8 * np.linalg.norm(g_ref)
    finally:
        sr.set_tile_config()
