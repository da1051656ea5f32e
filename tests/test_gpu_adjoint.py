"""GPU parity of the implicit-adjoint backward (sr_adjoint and the SRSolve autograd
function) against the float64 oracle's closed form (itself pinned to finite differences
and torch autograd on the CPU in test_oracle.py) and against central finite differences
of GPU solves.

Tolerances: p1, p2 accumulate in float64 for every storage type, with the centring
folded in after the sums (p1_k = O_k.x - obar.x), so sr_adjoint with the oracle's x and
lambda agrees to ~n_p u of the magnitude
    M_kj = ( (2|e_k| + m_k(x)) |lambda_j| + m_k(lambda) |x_j| ) / N,
    m_k(v) = |O_k|.|v| + |obar|.|v|
(1e-12 M for float64 output, plus float32 rounding 2^-24 |dO| for float32 output).
Through SRSolve the CG solutions carry their own residual tolerance, so the comparison
is norm-wise at 1e-8 (rtol 1e-13 solves of well-conditioned systems).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as orc
import synth
from paper_1108_0900_amd import sr
from paper_1108_0900_amd.autograd import sr_solve
from tests.gpu_util import DEV, device_matrix, rand_dense, rel_err, stored_dense

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def to_np(t):
    return t.detach().double().cpu().numpy()


def _dot_mag(Os, v):
    """m_k(v) = |O_k|.|v| + |obar|.|v| (uncentred: the kernel centres after summing)."""
    return np.abs(Os) @ np.abs(v) + np.abs(orc.sample_mean(Os)) @ np.abs(v)


def _magnitude(Os, E, x, lam):
    n = Os.shape[0]
    ec = np.abs(E - E.mean())
    a = 2 * ec + _dot_mag(Os, x)
    b = _dot_mag(Os, lam)
    return (np.outer(a, np.abs(lam)) + np.outer(b, np.abs(x))) / n


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16, torch.float16],
                         ids=lambda d: str(d).split(".")[-1])
@pytest.mark.parametrize("shape", [(1, 5), (7, 3), (300, 257), (129, 4099), (2000, 33)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("out", [torch.float64, torch.float32], ids=["out64", "out32"])
def test_adjoint_matches_closed_form(shape, dtype, out):
    n_s, n_p = shape
    print(f"[adj] {n_s}x{n_p} {dtype} -> {out}", flush=True)
    O, E = rand_dense(n_s, n_p, seed=11 * n_s + n_p, offset=0.2)
    Os = stored_dense(O, dtype)
    w = np.random.default_rng(n_p).standard_normal(n_p)
    eps = 0.05 * (orc.diag_overlap(Os).mean() + 1.0)
    ref = orc.solve_adjoint_gradients(Os, E, eps, w)
    M = device_matrix(O, dtype, ld=None if n_s == 1 else None)
    dO, dE, p12 = sr.sr_adjoint(M, to_dev(E), to_dev(ref["x"]), to_dev(ref["lam"]), dO_dtype=out, want_p12=True)
    torch.cuda.synchronize()
    mag = _magnitude(Os, E, ref["x"], ref["lam"])
    tol = 1e-12 * mag + (2.0 ** -24 * np.abs(ref["dO"]) if out == torch.float32 else 0.0) + 1e-300
    assert dO.dtype == out and tuple(dO.shape) == (n_s, n_p)
    assert np.all(np.abs(to_np(dO) - ref["dO"]) <= tol), float(np.max(np.abs(to_np(dO) - ref["dO"]) / mag))
    Oc = orc.centred(Os)
    assert np.all(np.abs(to_np(dE) - ref["dE"]) <= 1e-12 * 2 * _dot_mag(Os, ref["lam"]) / n_s + 1e-300)
    assert np.all(np.abs(to_np(p12[0]) - Oc @ ref["x"]) <= 1e-12 * _dot_mag(Os, ref["x"]) + 1e-300)


def test_adjoint_padded_rows_with_nan_padding():
    n_s, n_p = 97, 1001
    O, E = rand_dense(n_s, n_p, seed=3)
    w = np.random.default_rng(0).standard_normal(n_p)
    ref = orc.solve_adjoint_gradients(O, E, 0.3, w)
    M = device_matrix(O, torch.float64, ld=1024 + 32)
    dO, dE, _ = sr.sr_adjoint(M, to_dev(E), to_dev(ref["x"]), to_dev(ref["lam"]), dO_dtype=torch.float64)
    assert np.all(np.isfinite(to_np(dO))) and np.all(np.isfinite(to_np(dE)))
    mag = _magnitude(O, E, ref["x"], ref["lam"])
    assert np.all(np.abs(to_np(dO) - ref["dO"]) <= 1e-12 * mag)


@pytest.mark.parametrize("precond", [False, True], ids=["plain", "jacobi"])
def test_srsolve_autograd_matches_oracle_f64(precond):
    n_s, n_p = 400, 300
    O, E = rand_dense(n_s, n_p, seed=21)
    w = np.random.default_rng(5).standard_normal(n_p)
    eps0 = 1e-2 * orc.diag_overlap(O).mean()
    Ot = to_dev(O).requires_grad_(True)
    Et = to_dev(E).requires_grad_(True)
    epst = torch.tensor(eps0, dtype=torch.float64, requires_grad=True)
    x = sr_solve(Ot, Et, epst, 1e-13, 20, precond)
    loss = (x * to_dev(w)).sum()
    loss.backward()
    ref = orc.solve_adjoint_gradients(O, E, eps0, w)
    assert rel_err(to_np(x), ref["x"]) <= 1e-10
    assert rel_err(to_np(Ot.grad), ref["dO"]) <= 1e-8, rel_err(to_np(Ot.grad), ref["dO"])
    assert rel_err(to_np(Et.grad), ref["dE"]) <= 1e-8
    assert abs(float(epst.grad) - ref["deps"]) <= 1e-8 * abs(ref["deps"])


def test_srsolve_finite_differences():
    """Central differences (h = 1e-3, float64 GPU solves) of L = w . x."""
    n_s, n_p = 200, 60
    O, E = rand_dense(n_s, n_p, seed=23)
    w = np.random.default_rng(6).standard_normal(n_p)
    eps0 = 0.05
    wt = to_dev(w)

    def L(Om, Em, ep):
        with torch.no_grad():
            return float((sr_solve(to_dev(Om), to_dev(Em), ep, 1e-13, 10) * wt).sum())

    Ot = to_dev(O).requires_grad_(True)
    Et = to_dev(E).requires_grad_(True)
    epst = torch.tensor(eps0, dtype=torch.float64, requires_grad=True)
    (sr_solve(Ot, Et, epst, 1e-13, 10) * wt).sum().backward()
    gO, gE, geps = to_np(Ot.grad), to_np(Et.grad), float(epst.grad)
    h = 1e-3
    rng = np.random.default_rng(7)
    for _ in range(6):
        k, j = int(rng.integers(n_s)), int(rng.integers(n_p))
        Op, Om = O.copy(), O.copy()
        Op[k, j] += h
        Om[k, j] -= h
        fd = (L(Op, E, eps0) - L(Om, E, eps0)) / (2 * h)
        assert abs(fd - gO[k, j]) <= 1e-4 * (abs(fd) + 1e-3 * np.abs(gO).max()), (k, j, fd, gO[k, j])
    for _ in range(4):
        k = int(rng.integers(n_s))
        Ep, Em = E.copy(), E.copy()
        Ep[k] += h
        Em[k] -= h
        fd = (L(O, Ep, eps0) - L(O, Em, eps0)) / (2 * h)
        assert abs(fd - gE[k]) <= 1e-4 * (abs(fd) + 1e-3 * np.abs(gE).max()), (k, fd, gE[k])
    fd = (L(O, E, eps0 + h) - L(O, E, eps0 - h)) / (2 * h)
    assert abs(fd - geps) <= 1e-4 * abs(fd)


def test_srsolve_float32_storage():
    n_s, n_p = 1500, 700
    O, E = rand_dense(n_s, n_p, seed=25)
    O32 = stored_dense(O, torch.float32)
    w = np.random.default_rng(8).standard_normal(n_p)
    Ot = torch.from_numpy(O).to(DEV).to(torch.float32).requires_grad_(True)
    Et = to_dev(E).requires_grad_(True)
    x = sr_solve(Ot, Et, 1e-3, 1e-12, 20)
    (x * to_dev(w)).sum().backward()
    ref = orc.solve_adjoint_gradients(O32, E, 1e-3, w)
    assert Ot.grad.dtype == torch.float32
    assert rel_err(to_np(x), ref["x"]) <= 1e-8
    assert rel_err(to_np(Ot.grad), ref["dO"]) <= 1e-6, rel_err(to_np(Ot.grad), ref["dO"])
    assert rel_err(to_np(Et.grad), ref["dE"]) <= 1e-6


def test_adjoint_full_size_differentiation_case():
    """16384 x 16384 float32 O, eps = 1e-3, L = w . x: forward and backward at full size.
    Checked where the oracle can compute one by one: lambda's residual through the
    matrix-free product, and sampled rows of dL/dO and dL/dE recomputed in float64 from
    the same O, x and lambda; dL/deps = -lambda . x."""
    cfg = synth.CONFIGS["dense_16384"]
    d = synth.dense_inputs(cfg.n_s, cfg.n_p, cfg.seed, device=DEV, dtype=torch.float32)
    O, E = d["O"], d["E"]
    n_s, n_p = O.shape
    gen = torch.Generator(device=DEV)
    gen.manual_seed(55)
    w = torch.randn(n_p, generator=gen, dtype=torch.float64, device=DEV)
    Ot = O.clone().requires_grad_(True)
    Et = E.clone().requires_grad_(True)
    epst = torch.tensor(cfg.eps_abs, dtype=torch.float64, requires_grad=True)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    x = sr_solve(Ot, Et, epst, 1e-9, 20)
    e1.record()
    (x * w).sum().backward()
    e2.record()
    e2.synchronize()
    print(f"[adj-full] forward {e0.elapsed_time(e1):.1f} ms, backward {e1.elapsed_time(e2):.1f} ms", flush=True)
    # lambda from the gradient of eps: deps = -lambda . x, and lambda solves (S + eps I) lambda = w
    M = sr.as_matrix(O)
    M.mean = sr.sr_grad(M, None)["mean"]
    lam, info = sr.sr_cg_solve(M, w, cfg.eps_abs, rtol=1e-9, refresh_every=20)
    assert info["status"] == 0
    lx = float(lam @ x.detach())
    assert abs(float(epst.grad) + lx) <= 1e-6 * abs(lx)
    res = sr.sr_sv_product(M, lam, cfg.eps_abs) - w
    assert float(res.norm() / w.norm()) <= 1e-8
    # sampled rows, recomputed in float64 on the CPU from the stored float32 values
    rows = torch.randperm(n_s, generator=torch.Generator().manual_seed(3))[:48].tolist()
    Ocpu = O.double().cpu().numpy()
    mean = Ocpu.mean(axis=0)
    Ecpu, xc, lc = E.cpu().numpy(), to_np(x), to_np(lam)
    ec = Ecpu - Ecpu.mean()
    gO = Ot.grad
    for k in rows:
        oc = Ocpu[k] - mean
        p1, p2 = oc @ xc, oc @ lc
        ref = ((2 * ec[k] - p1) * lc - p2 * xc) / n_s
        mx = np.abs(Ocpu[k]) @ np.abs(xc) + np.abs(mean) @ np.abs(xc)
        ml = np.abs(Ocpu[k]) @ np.abs(lc) + np.abs(mean) @ np.abs(lc)
        mag = ((2 * abs(ec[k]) + mx) * np.abs(lc) + ml * np.abs(xc)) / n_s
        got = gO[k].double().cpu().numpy()
        assert np.all(np.abs(got - ref) <= 1e-10 * mag + 2.0 ** -23 * np.abs(ref) + 1e-300), k
        assert abs(float(Et.grad[k]) - 2 * p2 / n_s) <= 1e-10 * 2 * ml / n_s + 1e-300
