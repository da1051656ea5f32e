"""The named workloads at their full sizes against the FP64 CPU oracle.

* dense 8192 x 4000 float64: CG to rtol 1e-13 against the oracle's dense solve (form S,
  Cholesky), error <= 1e-10 (the parity reading of the float64 target);
* CPS-shaped 65536 x 24512, float64 and float32 storage, CG to rtol 1e-8: the true residual
  of each GPU solution computed by the oracle's matrix-free product on the host, with the
  oracle's own g and eps;
* dense 16384 x 16384 (the differentiation workload), float64 storage: the implicit-adjoint
  backward of L = w . x against the oracle's closed-form gradient over all entries, and
  against central finite differences (h = 1e-3) on 32 entries of O and 16 of E, with
  float64 CG to rtol 1e-12 (kappa is about 2.5e4 here, so float64 CG cannot attain the
  workload's 1e-13: the true residual stalls near kappa * 1e-16).

Inputs are the seeded generators of synth at the workload's seed, made on the device and
copied to the host for the oracle; nothing the oracle uses comes from the GPU path.
"""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from paper_1108_0900_amd import sr
from paper_1108_0900_amd.autograd import sr_solve
from tests.gpu_util import DEV, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_dense_8192x4000_float64_parity():
    cfg = synth.CONFIGS["dense_8192x4000"]
    d = synth.dense_inputs(cfg.n_s, cfg.n_p, cfg.seed, device=DEV)
    O, E = d["O"], d["E"]
    M = sr.as_matrix(O)
    st = sr.sr_grad(M, E)
    M.mean = st["mean"]
    eps = cfg.eps_rel * float(st["diag"].mean())
    x, info = sr.sr_cg_solve(M, st["g"], eps, rtol=1e-13, refresh_every=20)
    print(f"[dense-8192x4000] {info}", flush=True)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-13, info
    Oh, Eh = O.cpu().numpy(), E.cpu().numpy()
    g_ref = orc.energy_gradient(Oh, Eh)
    eps_ref = cfg.eps_rel * orc.diag_overlap(Oh).mean()
    assert abs(eps - eps_ref) <= 1e-12 * eps_ref
    x_ref = orc.solve_dense(Oh, g_ref, eps_ref)
    err = rel_err(to_np(x), x_ref)
    print(f"[dense-8192x4000] error vs dense solve {err:.2e}", flush=True)
    assert err <= 1e-10, err


@pytest.mark.slow
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["float64", "float32"])
def test_cps_65536x24512_true_residual_by_oracle(dtype):
    cfg = synth.CONFIGS["cps_65536x24512"]
    d = synth.cps_inputs(cfg.n_s, cfg.n_corr, cfg.n_states, cfg.n_dense, cfg.seed, device=DEV)
    O64, E = d["O"], d["E"]
    Ot = O64 if dtype == torch.float64 else O64.to(dtype)
    M = sr.as_matrix(Ot)
    st = sr.sr_grad(M, E)
    M.mean = st["mean"]
    eps = cfg.eps_rel * float(st["diag"].mean())
    x, info = sr.sr_cg_solve(M, st["g"], eps, rtol=cfg.rtol, refresh_every=20)
    print(f"[cps-65536x24512 {dtype}] {info}", flush=True)
    assert info["status"] == 0, info
    Oh = Ot.double().cpu().numpy()            # the stored values, in float64
    del M, Ot, O64, d
    torch.cuda.empty_cache()
    Eh = E.cpu().numpy()
    g_ref = orc.energy_gradient(Oh, Eh)
    eps_ref = cfg.eps_rel * orc.diag_overlap(Oh).mean()
    assert abs(eps - eps_ref) <= 1e-12 * eps_ref
    assert rel_err(to_np(st["g"]), g_ref) <= 1e-12
    r = g_ref - orc.sv_product_swapped(Oh, to_np(x), eps_ref)
    rel = float(np.linalg.norm(r) / np.linalg.norm(g_ref))
    print(f"[cps-65536x24512 {dtype}] oracle true residual {rel:.2e}", flush=True)
    assert rel <= 2 * cfg.rtol, rel


@pytest.mark.slow
def test_differentiation_16384_oracle_gradient_and_finite_differences():
    """dL/dO and dL/dE of L = w . x, x = (S + eps I)^{-1} g, on the 16384 x 16384 workload
    (float64 storage of its values, eps = 1e-3):

    * against the oracle's closed-form adjoint gradient (dense Cholesky solves on the host),
      element-wise over the whole of dL/dO and dL/dE;
    * against central differences h = 1e-3 of float64 solves to rtol 1e-12 (32 entries of
      O, 16 of E).  kappa is about 2.5e4, so each solve carries an error near kappa * rtol
      that a difference quotient divides by 2h; the test measures that floor (the spread of
      L over solves of the unperturbed system from different starting points) and allows
      1e-3 relative plus twice the floor over h.
    """
    cfg = synth.CONFIGS["dense_16384"]
    d = synth.dense_inputs(cfg.n_s, cfg.n_p, cfg.seed, device=DEV, dtype=torch.float32)
    O = d["O"].double()
    E = d["E"]
    del d
    n_s, n_p = O.shape
    gen = torch.Generator(device=DEV)
    gen.manual_seed(55)
    w = torch.randn(n_p, generator=gen, dtype=torch.float64, device=DEV)
    rtol = 1e-12
    Ot = O.clone().requires_grad_(True)
    Et = E.clone().requires_grad_(True)
    x = sr_solve(Ot, Et, cfg.eps_abs, rtol, 20, True)
    (x * w).sum().backward()
    gO, gE = Ot.grad, Et.grad
    x0 = x.detach()
    del Ot, Et

    # the oracle's gradient
    ref = orc.solve_adjoint_gradients(O.cpu().numpy(), E.cpu().numpy(), cfg.eps_abs, w.cpu().numpy())
    err_x = rel_err(to_np(x0), ref["x"])
    err_O = rel_err(to_np(gO), ref["dO"])
    err_E = rel_err(to_np(gE), ref["dE"])
    print(f"[grad-16384] vs oracle: x {err_x:.2e}  dL/dO {err_O:.2e}  dL/dE {err_E:.2e}", flush=True)
    assert err_x <= 1e-6 and err_O <= 1e-6 and err_E <= 1e-6, (err_x, err_O, err_E)
    del ref

    def loss(Om, Em, start=None):
        Mm = sr.as_matrix(Om)
        st = sr.sr_grad(Mm, Em)
        Mm.mean = st["mean"]
        xm, info = sr.sr_cg_solve(Mm, st["g"], cfg.eps_abs, rtol=rtol, refresh_every=20,
                                  x0=x0 if start is None else start, precond=True)
        assert info["status"] == 0, info
        return float(xm @ w)

    h = 1e-3
    base = [loss(O, E), loss(O, E, start=torch.zeros_like(x0)), loss(O, E, start=x0 * (1 + 1e-6))]
    floor = (max(base) - min(base)) / h
    print(f"[fd-16384] L spread over starting points {max(base) - min(base):.2e}, "
          f"difference-quotient floor {floor:.2e}", flush=True)
    pick = torch.Generator().manual_seed(9)
    rows = torch.randint(0, n_s, (32,), generator=pick).tolist()
    cols = torch.randint(0, n_p, (32,), generator=pick).tolist()
    worst = 0.0
    for k, j in zip(rows, cols):
        old = float(O[k, j])
        O[k, j] = old + h
        lp = loss(O, E)
        O[k, j] = old - h
        lm = loss(O, E)
        O[k, j] = old
        fd = (lp - lm) / (2 * h)
        an = float(gO[k, j])
        worst = max(worst, abs(fd - an) / (1e-3 * abs(an) + 2 * floor))
    print(f"[fd-16384] dL/dO worst |fd - analytic| / (1e-3 |analytic| + 2 floor) = {worst:.2f}", flush=True)
    assert worst <= 1.0, worst
    worstE = 0.0
    for k in torch.randint(0, n_s, (16,), generator=pick).tolist():
        Ep, Em = E.clone(), E.clone()
        Ep[k] += h
        Em[k] -= h
        fd = (loss(O, Ep) - loss(O, Em)) / (2 * h)
        an = float(gE[k])
        worstE = max(worstE, abs(fd - an) / (1e-3 * abs(an) + 2 * floor))
    print(f"[fd-16384] dL/dE worst |fd - analytic| / (1e-3 |analytic| + 2 floor) = {worstE:.2f}", flush=True)
    assert worstE <= 1.0, worstE
