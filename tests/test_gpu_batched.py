"""GPU parity of the batched form: the K-right-hand-side product and the batched CG
(several systems, several shifted right-hand sides each, one persistent launch) against
the float64 oracle, column by column.

Tolerances: every batched product accumulates in float64 (exact = 0 and 1 alike), so the
product matches to 1e-12 of the centred magnitude reference |Oc|^T |Oc| |v| / N + eps |v|,
as the one-column float64 product does.  Batched solves end on a float64-accumulated
true residual <= rtol; their error against the dense oracle solution is bounded by
kappa * rtol, so well-conditioned cases are compared at 1e-7.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as orc
import synth
from paper_1108_0900_amd import sr
from tests.gpu_util import DEV, device_matrix, rand_dense, rel_err, stored_dense

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def to_np(t):
    return t.detach().double().cpu().numpy()


def _mag(Os, v, eps):
    n = Os.shape[0]
    Oc = np.abs(orc.centred(Os))
    return Oc.T @ (Oc @ np.abs(v)) / n + eps * np.abs(v)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(1, 9), (37, 1000), (300, 4099), (129, 70001)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("k", [1, 3, 8])
@pytest.mark.parametrize("exact", [False, True], ids=["exact0", "exact1"])
def test_multi_rhs_product_matches_oracle(shape, dtype, k, exact):
    n_s, n_p = shape
    print(f"[svk] {n_s}x{n_p} {dtype} k={k} exact={exact}", flush=True)
    O, _ = rand_dense(n_s, n_p, seed=n_s + 3 * n_p, offset=0.3)
    Os = stored_dense(O, dtype)
    rng = np.random.default_rng(k)
    V = rng.standard_normal((k, n_p))
    eps = list(10.0 ** rng.uniform(-4, -1, k))
    M = device_matrix(O, dtype)
    Y = to_np(sr.sr_svk_product(M, to_dev(V), eps, exact=exact))
    tol = 1e-12
    for i in range(k):
        ref = orc.sv_product_swapped(Os, V[i], eps[i])
        mag = _mag(Os, V[i], eps[i])
        assert np.all(np.abs(Y[i] - ref) <= tol * mag + 1e-300), (i, float(np.max(np.abs(Y[i] - ref) / mag)))


def test_multi_rhs_product_wide_matches_single_products():
    """A wide shape (12000 rows, 140000 columns: 69 column blocks, 12 splits of 1000 rows,
    too large for the CPU oracle): every column of the 8-column product equals the
    one-column float64 product (a different kernel, itself checked against the oracle) to
    1e-12 of the magnitude reference."""
    n_s, n_p = 12000, 140000
    gen = torch.Generator(device=DEV)
    gen.manual_seed(91)
    O = (torch.randn(n_s, n_p, generator=gen, device=DEV, dtype=torch.float32) + 0.3)
    M = sr.as_matrix(O)
    M.mean = sr.sr_grad(M, None)["mean"]
    V = torch.randn(8, n_p, generator=gen, device=DEV, dtype=torch.float64)
    eps = [10.0 ** (-i) for i in range(8)]
    Y = sr.sr_svk_product(M, V, eps)
    A = (O - M.mean.float()).abs().double()
    for i in range(8):
        y1 = sr.sr_sv_product(M, V[i], eps[i])
        mag = (A.T @ (A @ V[i].abs())) / n_s + eps[i] * V[i].abs()
        assert float(((Y[i] - y1).abs() / mag).max()) <= 1e-12, i
    del O, A


@pytest.mark.parametrize("cfg", sr.BATCH_CONFIGS, ids=lambda c: f"split{c[0]}-tasks{c[1]}")
def test_multi_rhs_product_every_batch_config(cfg):
    """Every batched geometry the autotuner chooses from gives the oracle's product."""
    n_s, n_p = 3000, 9001
    O, _ = rand_dense(n_s, n_p, seed=5, offset=0.3)
    M = device_matrix(O, torch.float32)
    Os = stored_dense(O, torch.float32)
    V = np.random.default_rng(6).standard_normal((8, n_p))
    eps = [0.1 * (i + 1) for i in range(8)]
    try:
        sr.set_batch_config(*cfg)
        Y = to_np(sr.sr_svk_product(M, to_dev(V), eps))
    finally:
        sr.set_batch_config()
    for i in range(8):
        ref = orc.sv_product_swapped(Os, V[i], eps[i])
        mag = _mag(Os, V[i], eps[i])
        assert np.all(np.abs(Y[i] - ref) <= 1e-12 * mag), (cfg, i)


def test_batched_autotuner_selects_a_config(tmp_path):
    from paper_1108_0900_amd import tune
    O, _ = rand_dense(4000, 20000, seed=8)
    M = device_matrix(O, torch.float32)
    cache = str(tmp_path / "tiles.json")
    try:
        res = tune.autotune(M, kind=2, reps=2, cache_path=cache)
        assert tuple(res["best"]) in sr.BATCH_CONFIGS and not res["cached"]
        assert len(res["ms"]) == len(sr.BATCH_CONFIGS)
        res2 = tune.autotune(M, kind=2, cache_path=cache)
        assert res2["cached"] and tuple(res2["best"]) == tuple(res["best"])
    finally:
        sr.set_batch_config()


def _batch_case(dtype, shapes, k, seed):
    systems, refs = [], []
    for s, (n_s, n_p) in enumerate(shapes):
        O, E = rand_dense(n_s, n_p, seed=seed + s)
        Os = stored_dense(O, dtype)
        M = device_matrix(O, dtype)
        g = orc.energy_gradient(Os, E)
        rng = np.random.default_rng(seed + 100 + s)
        G = np.stack([g] + [rng.standard_normal(n_p) for _ in range(k - 1)])
        dS = orc.diag_overlap(Os).mean()
        eps = list(dS * np.logspace(-1, 0, k))          # well-conditioned shifts
        systems.append((M, to_dev(G), eps))
        refs.append([orc.solve_dense(Os, G[i], eps[i]) for i in range(k)])
    return systems, refs


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("k", [1, 5, 8])
def test_batched_cg_matches_dense_solves(dtype, k):
    shapes = [(300, 257), (1000, 1200), (64, 3000), (2000, 90), (513, 4099)]
    systems, refs = _batch_case(dtype, shapes, k, seed=40)
    X, info, st = sr.sr_cg_solve_batched(systems, rtol=1e-11, refresh_every=20)
    assert st == sr.SR_OK, info
    for s in range(len(shapes)):
        for i in range(k):
            assert info[s][i]["status"] == 0 and info[s][i]["rel_res_true"] <= 1e-11, info[s][i]
            assert rel_err(to_np(X[s][i]), refs[s][i]) <= 1e-7, (s, i, rel_err(to_np(X[s][i]), refs[s][i]))


def test_batched_cg_zero_rhs_and_single_sample():
    O1, _ = rand_dense(1, 40, seed=1)
    O2, E2 = rand_dense(200, 50, seed=2)
    M1, M2 = device_matrix(O1, torch.float64), device_matrix(O2, torch.float64)
    G1 = torch.zeros(2, 40, dtype=torch.float64, device=DEV)            # zero right-hand sides
    G1[1, 3] = 1.0                                                       # S = 0 here: x = g / eps
    G2 = to_dev(np.stack([orc.energy_gradient(O2, E2), np.zeros(50)]))
    X, info, st = sr.sr_cg_solve_batched([(M1, G1, [0.5, 0.25]), (M2, G2, [0.1, 0.1])], rtol=1e-12)
    assert st == sr.SR_OK
    assert torch.count_nonzero(X[0][0]) == 0 and float(X[0][1][3]) == pytest.approx(4.0, rel=1e-14)
    assert torch.count_nonzero(X[1][1]) == 0
    ref = orc.solve_dense(O2, orc.energy_gradient(O2, E2), 0.1)
    assert rel_err(to_np(X[1][0]), ref) <= 1e-9


def test_batched_cg_not_converged_reports_status():
    O, E = rand_dense(500, 800, seed=5)
    M = device_matrix(O, torch.float64)
    G = to_dev(np.stack([orc.energy_gradient(O, E)] * 2))
    X, info, st = sr.sr_cg_solve_batched([(M, G, [1e-6, 1e-6])], rtol=1e-14, max_iter=3, raise_on=())
    assert st == sr.SR_NOT_CONVERGED
    assert all(c["status"] == 1 for c in info[0])
    assert all(np.isfinite(to_np(X[0][i])).all() for i in range(2))


def test_batched_cg_deterministic():
    systems, _ = _batch_case(torch.float32, [(700, 3000), (300, 500)], 8, seed=60)
    X1, _, _ = sr.sr_cg_solve_batched(systems, rtol=1e-9)
    X2, _, _ = sr.sr_cg_solve_batched(systems, rtol=1e-9)
    for a, b in zip(X1, X2):
        assert torch.equal(a, b)


def test_batched_full_size_workload():
    """64 systems (N_p in [1000, 60000], N_s in [4096, 32768], float32 O), 8 shifts
    1e-4..1e-1 of mean(diag S) each, g the SR gradient, one launch.  Every column must
    end converged; its residual is re-checked with the one-column float64 product (a
    different kernel), and on the smallest systems with the CPU oracle."""
    cfg = synth.CONFIGS["batched_64sys"]
    shapes = synth.batched_shapes(seed=cfg.seed)
    shifts = synth.relative_shifts(8)
    systems, grads = [], []
    for s, (n_s, n_p) in enumerate(shapes):
        d = synth.dense_inputs(n_s, n_p, cfg.seed * 1000 + s, device=DEV, dtype=torch.float32)
        M = sr.as_matrix(d["O"])
        st = sr.sr_grad(M, d["E"])
        M.mean = st["mean"]
        dS = float(st["diag"].mean())
        G = st["g"].unsqueeze(0).repeat(8, 1).contiguous()
        systems.append((M, G, [dS * r for r in shifts]))
        grads.append(st["g"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    X, info, st = sr.sr_cg_solve_batched(systems, rtol=cfg.rtol, refresh_every=20)
    e1.record()
    e1.synchronize()
    print(f"[batched-full] {e0.elapsed_time(e1):.1f} ms, products "
          f"{sum(i[0]['products'] for i in info)}", flush=True)
    assert st == sr.SR_OK
    for s, (M, G, eps) in enumerate(systems):
        for i in range(8):
            assert info[s][i]["status"] == 0 and info[s][i]["rel_res_true"] <= cfg.rtol
            r = sr.sr_sv_product(M, X[s][i], eps[i]) - grads[s]
            assert float(r.norm() / grads[s].norm()) <= 2 * cfg.rtol, (s, i)
    # the two smallest systems against the CPU oracle's matrix-free product
    order = sorted(range(len(shapes)), key=lambda s: shapes[s][0] * shapes[s][1])[:2]
    for s in order:
        M, G, eps = systems[s]
        Ocpu = M.O.double().cpu().numpy()
        g = grads[s].cpu().numpy()
        for i in (0, 7):
            r = orc.sv_product_swapped(Ocpu, to_np(X[s][i]), eps[i]) - g
            assert np.linalg.norm(r) <= 2 * cfg.rtol * np.linalg.norm(g), (s, i)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_shifts_batched_match_dense_solves(dtype):
    """Multi-shift CG of several systems of different shapes in one launch (shifts given in
    scrambled order) against the oracle's dense solve of each stored system and shift."""
    shapes = [(300, 130), (1200, 4099), (77, 513), (2500, 2000)]
    rel = list(10.0 ** np.linspace(-4, -1, 6))
    systems, refs = [], []
    for s, (n_s, n_p) in enumerate(shapes):
        O, E = rand_dense(n_s, n_p, seed=90 + s)
        Os = stored_dense(O, dtype)
        M = device_matrix(O, dtype)
        st = sr.sr_grad(M, to_dev(E))
        if s % 2 == 0:
            M.mean = st["mean"]                 # the others have their means computed by the call
        dS = float(st["diag"].mean())
        eps = [dS * rel[i] for i in (2, 0, 5, 1, 4, 3)]
        systems.append((M, st["g"], eps))
        g_ref = orc.energy_gradient(Os, E)
        dS_ref = orc.diag_overlap(Os).mean()
        refs.append([orc.solve_dense(Os, g_ref, e / dS * dS_ref) for e in eps])
    X, info, status = sr.sr_cg_solve_shifts_batched(systems, rtol=1e-11)
    assert status == 0, info
    for s in range(len(shapes)):
        for i in range(6):
            assert info[s][i]["status"] == 0 and info[s][i]["rel_res_true"] <= 1e-11, (s, i, info[s][i])
            err = rel_err(to_np(X[s][i]), refs[s][i])
            assert err <= 1e-8, (s, i, err)


def test_shifts_batched_equal_one_system_calls():
    """The same systems one call each (sr_cg_solve_shifts) and all in one launch: the same
    arithmetic in the same order, so the same solutions."""
    systems = []
    for s, (n_s, n_p) in enumerate([(500, 700), (900, 300)]):
        O, E = rand_dense(n_s, n_p, seed=120 + s)
        M = device_matrix(O, torch.float32)
        st = sr.sr_grad(M, to_dev(E))
        M.mean = st["mean"]
        dS = float(st["diag"].mean())
        systems.append((M, st["g"], [dS * 1e-3, dS * 1e-2, dS * 1e-1]))
    Xb, _, sb = sr.sr_cg_solve_shifts_batched(systems, rtol=1e-10)
    assert sb == 0
    for s, (M, g, eps) in enumerate(systems):
        X1, _, s1 = sr.sr_cg_solve_shifts(M, g, eps, rtol=1e-10)
        assert s1 == 0
        assert rel_err(to_np(Xb[s]), to_np(X1)) <= 1e-14


def test_shifts_batched_full_size_workload():
    """The 64-system workload (N_p in [1000, 60000], N_s in [4096, 32768], float32 O, 8
    shifts 1e-4..1e-1 of mean(diag S), g the SR gradient) by multi-shift CG in one launch:
    every shift converged, its residual re-checked with the one-column product, the two
    smallest systems with the CPU oracle."""
    cfg = synth.CONFIGS["batched_64sys"]
    shapes = synth.batched_shapes(seed=cfg.seed)
    shifts = synth.relative_shifts(8)
    systems = []
    for s, (n_s, n_p) in enumerate(shapes):
        d = synth.dense_inputs(n_s, n_p, cfg.seed * 1000 + s, device=DEV, dtype=torch.float32)
        M = sr.as_matrix(d["O"])
        st = sr.sr_grad(M, d["E"])
        M.mean = st["mean"]
        dS = float(st["diag"].mean())
        systems.append((M, st["g"], [dS * r for r in shifts]))
    sr.timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    X, info, status = sr.sr_cg_solve_shifts_batched(systems, rtol=cfg.rtol, refresh_every=20)
    e1.record()
    e1.synchronize()
    ms, launches = sr.timing_read("solve_launch")
    sr.timing(False)
    # a shift that missed rtol in the launch continued with its own solve: more products
    cont = sum(1 for s in info for c in s if c["products"] > min(x["products"] for x in s))
    print(f"[shifts-batched-full] {e0.elapsed_time(e1):.1f} ms, launch {ms:.1f} ms, launches {launches}, "
          f"continued shifts {cont}", flush=True)
    assert status == sr.SR_OK
    assert launches == 1
    for s, (M, g, eps) in enumerate(systems):
        for i in range(8):
            assert info[s][i]["status"] == 0 and info[s][i]["rel_res_true"] <= cfg.rtol, (s, i, info[s][i])
            r = sr.sr_sv_product(M, X[s][i], eps[i]) - g
            assert float(r.norm() / g.norm()) <= 2 * cfg.rtol, (s, i)
    order = sorted(range(len(shapes)), key=lambda s: shapes[s][0] * shapes[s][1])[:2]
    for s in order:
        M, g, eps = systems[s]
        Ocpu = M.O.double().cpu().numpy()
        gh = g.cpu().numpy()
        for i in (0, 7):
            r = orc.sv_product_swapped(Ocpu, to_np(X[s][i]), eps[i]) - gh
            assert np.linalg.norm(r) <= 2 * cfg.rtol * np.linalg.norm(gh), (s, i)
