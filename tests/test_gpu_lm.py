"""GPU parity of the generalized Davidson solver of the linear method (lm_davidson,
Sec. II.B) against the oracle's dense generalized eigensolve of the same sampled H and S.

The Ritz value converges with the residual: for the tolerance 1e-10 used here the lowest
eigenvalue matches the dense one to 1e-9 (relative); the Ritz vector is compared through
its residual with the oracle's dense H and S (which does not depend on the eigenvector's
normalization or sign) and its S-norm."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as orc
from paper_1108_0900_amd import sr
from tests.gpu_util import DEV, device_matrix, rand_dense, stored_dense

pytestmark = pytest.mark.gpu


def _case(n_s, n_p, seed):
    O, E = rand_dense(n_s, n_p, seed=seed)
    D = 0.1 * np.random.default_rng(seed + 1).standard_normal((n_s, n_p))
    return O, E, D


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(400, 7), (3000, 120), (5000, 600)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("max_sub", [40, 8])
@pytest.mark.parametrize("precond", [0, 1, 2], ids=["residual", "approx-diag", "exact-diag"])
def test_davidson_matches_dense_eigensolve(shape, dtype, max_sub, precond):
    n_s, n_p = shape
    print(f"[davidson] {n_s}x{n_p} {dtype} max_sub={max_sub} precond={precond}", flush=True)
    O, E, D = _case(n_s, n_p, seed=n_p + 3)
    Os, Ds = stored_dense(O, dtype), stored_dense(D, dtype)
    M, Md = device_matrix(O, dtype), device_matrix(D, dtype)
    theta, c, info = sr.lm_davidson(M, torch.from_numpy(E).to(DEV), Md, tol=1e-10, max_iter=3000, max_sub=max_sub,
                                    precond=precond)
    assert info["status"] == 0, info
    H, S = orc.lm_matrices(Os, E, Ds)
    ev, _ = orc.lm_lowest_eigenpair(H, S)
    assert abs(theta - ev) <= 1e-9 * abs(ev), (theta, ev, info)
    cn = c.cpu().numpy()
    assert abs(cn @ S @ cn - 1.0) <= 1e-9
    res = np.linalg.norm(H @ cn - theta * (S @ cn))
    assert res <= 1e-9 * abs(theta) * 10, (res, info)
    if max_sub == 8 and n_p >= 120 and not precond:
        assert info["restarts"] > 0


def test_davidson_not_converged_reports_status():
    O, E, D = _case(2000, 300, seed=9)
    M, Md = device_matrix(O, torch.float64), device_matrix(D, torch.float64)
    theta, c, info = sr.lm_davidson(M, torch.from_numpy(E).to(DEV), Md, tol=1e-14, max_iter=3, max_sub=8,
                                    raise_on=())
    assert info["status"] == sr.SR_NOT_CONVERGED and info["iters"] == 3
    assert np.isfinite(theta) and torch.isfinite(c).all()


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16], ids=["bf16", "f16"])
def test_davidson_scaled_storage(dtype):
    """bf16/f16 codes with column scales: the products accumulate in float32, so the Ritz
    value matches the dense eigensolve of the dequantized matrices to 1e-5 (relative)."""
    O, E, D = _case(3000, 200, seed=41)
    Os, Ds = stored_dense(O, dtype), stored_dense(D, dtype)
    M, Md = device_matrix(O, dtype), device_matrix(D, dtype)
    theta, c, info = sr.lm_davidson(M, torch.from_numpy(E).to(DEV), Md, tol=1e-6, max_iter=2000, max_sub=40,
                                    precond=2)
    assert info["status"] == 0, info
    H, S = orc.lm_matrices(Os, E, Ds)
    ev, _ = orc.lm_lowest_eigenpair(H, S)
    assert abs(theta - ev) <= 1e-5 * abs(ev), (theta, ev, info)


def test_davidson_deterministic():
    O, E, D = _case(3000, 250, seed=13)
    M, Md = device_matrix(O, torch.float64), device_matrix(D, torch.float64)
    Et = torch.from_numpy(E).to(DEV)
    t1, c1, i1 = sr.lm_davidson(M, Et, Md, tol=1e-9, max_sub=16, precond=2)
    t2, c2, i2 = sr.lm_davidson(M, Et, Md, tol=1e-9, max_sub=16, precond=2)
    assert t1 == t2 and torch.equal(c1, c2) and i1 == i2
