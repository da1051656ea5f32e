"""GPU checks of the boundary helpers: workspace sizing (a reserve of what
sr_workspace_bytes reports makes the call allocate nothing more), the asynchronous CG
solve (device-side outcome, same solution as the oracle's), and dL/deps computed by
sr_adjoint."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_1108_0900_amd import sr
from tests.gpu_util import DEV, rand_dense, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

MIB = 1 << 20


def _dense(n_s, n_p, seed, dtype=torch.float64):
    O, E = rand_dense(n_s, n_p, seed=seed, offset=0.2)
    return O, E, sr.as_matrix(torch.from_numpy(O).to(DEV).to(dtype))


@pytest.mark.parametrize("call", ["grad", "sv_product", "cg_solve", "lm_hv_product", "adjoint"])
@pytest.mark.parametrize("shape", [(300, 513), (64, 70001)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_workspace_bytes_cover_the_call(call, shape):
    O, E, M = _dense(*shape, seed=7)
    Et = to_dev(E)
    for with_mean in (False, True):
        M.mean = sr.sr_grad(M, None)["mean"] if with_mean else None
        need = sr.workspace_bytes(M, call)
        assert need > 0
        torch.cuda.synchronize()
        sr.release()
        sr.workspace_reserve(need)
        held = sr.workspace_held()
        assert held >= need
        v = torch.randn(M.n_p, dtype=torch.float64, device=DEV)
        if call == "grad":
            sr.sr_grad(M, Et)
        elif call == "sv_product":
            sr.sr_sv_product(M, v, 0.1)
        elif call == "cg_solve":
            sr.sr_cg_solve(M, v, 0.1, rtol=1e-8, max_iter=5,
                           raise_on=(sr.SR_ERR_INVALID, sr.SR_ERR_NOMEM, sr.SR_ERR_HIP, sr.SR_ERR_TIMEOUT))
        elif call == "lm_hv_product":
            D = sr.as_matrix(torch.randn(M.O.shape[0], M.n_p, dtype=torch.float64, device=DEV) * 0.1)
            sr.lm_hv_product(M, Et, D, torch.randn(M.n_p + 1, dtype=torch.float64, device=DEV))
        else:
            sr.sr_adjoint(M, Et, v, v, dO_dtype=torch.float32)
        torch.cuda.synchronize()
        assert sr.workspace_held() == held, (call, with_mean, need, held, sr.workspace_held())


def test_workspace_bytes_compact_plane_cg():
    d = __import__("synth").cps_inputs(700, 30, 240, 500, 9, device=DEV)
    q, s, lo, cols = sr.sr_quantize(d["O"], out_dtype=torch.bfloat16, with_lo="compact")
    M = sr.as_matrix(q, scale=s, lo=lo, lo_cols=cols)
    for call in ("grad", "cg_solve"):
        need = sr.workspace_bytes(M, call)
        torch.cuda.synchronize()
        sr.release()
        sr.workspace_reserve(need)
        held = sr.workspace_held()
        if call == "grad":
            sr.sr_grad(M, d["E"])
        else:
            sr.sr_cg_solve(M, torch.randn(M.n_p, dtype=torch.float64, device=DEV), 0.1, rtol=1e-6, refresh_every=5)
        torch.cuda.synchronize()
        assert sr.workspace_held() == held


def test_cg_solve_async_matches_sync_and_oracle():
    O, E, M = _dense(2000, 1500, seed=11)
    st = sr.sr_grad(M, to_dev(E))
    M.mean = st["mean"]
    eps = 1e-3 * float(st["diag"].mean())
    x_sync, info = sr.sr_cg_solve(M, st["g"], eps, rtol=1e-12, refresh_every=20)
    x = torch.empty_like(x_sync)
    dinfo = torch.full((16,), float("nan"), dtype=torch.float64, device=DEV)
    sr.sr_cg_solve_async(M, st["g"], eps, x, dinfo, rtol=1e-12, refresh_every=20)
    torch.cuda.synchronize()
    h = dinfo.cpu().numpy()
    assert int(h[2]) == sr.SR_OK and int(h[0]) == info["iters"] and int(h[3]) == info["products"]
    assert torch.equal(x, x_sync)          # the same single-launch kernel for float64 storage
    x_ref = orc.solve_dense(O, orc.energy_gradient(O, E), 1e-3 * orc.diag_overlap(O).mean())
    assert rel_err(to_np(x), x_ref) <= 1e-9
    # max_iter reached: the status lands in device memory
    sr.sr_cg_solve_async(M, st["g"], eps, x, dinfo, rtol=1e-14, max_iter=3)
    torch.cuda.synchronize()
    h = dinfo.cpu().numpy()
    assert int(h[2]) == sr.SR_NOT_CONVERGED and int(h[0]) == 3


def test_cg_solve_async_scaled_storage():
    """bf16 codes, one plane: the async solve runs in one launch (both product codes) and
    reaches the requested true residual of the stored system."""
    O, E = rand_dense(1500, 1000, seed=12)
    q, s = sr.sr_quantize(torch.from_numpy(O).to(DEV), out_dtype=torch.bfloat16)
    M = sr.as_matrix(q, scale=s)
    st = sr.sr_grad(M, to_dev(E))
    M.mean = st["mean"]
    eps = 1e-2 * float(st["diag"].mean())
    x = torch.empty(M.n_p, dtype=torch.float64, device=DEV)
    dinfo = torch.zeros(16, dtype=torch.float64, device=DEV)
    sr.sr_cg_solve_async(M, st["g"], eps, x, dinfo, rtol=1e-8, refresh_every=20)
    torch.cuda.synchronize()
    h = dinfo.cpu().numpy()
    assert int(h[2]) == sr.SR_OK and h[5] <= 1e-8
    Os = orc.dequantize_bf16(*orc.quantize_bf16(O))
    g_ref = orc.energy_gradient(Os, E)
    r = g_ref - orc.sv_product_swapped(Os, to_np(x), 1e-2 * orc.diag_overlap(Os).mean())
    assert np.linalg.norm(r) <= 2e-8 * np.linalg.norm(g_ref)


def test_adjoint_deps_alone_and_with_gradients():
    O, E, M = _dense(300, 200, seed=13)
    rng = np.random.default_rng(14)
    x, lam = rng.standard_normal(200), rng.standard_normal(200)
    want = -float(lam @ x)
    _, _, _, deps = sr.sr_adjoint(M, to_dev(E), to_dev(x), to_dev(lam), dO_dtype=None, want_dE=False, want_deps=True)
    assert abs(float(deps) - want) <= 1e-13 * np.abs(lam) @ np.abs(x)
    dO, dE, _, deps2 = sr.sr_adjoint(M, to_dev(E), to_dev(x), to_dev(lam), dO_dtype=torch.float64, want_deps=True)
    assert float(deps2) == float(deps) and dO is not None and dE is not None
