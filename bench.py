"""Benchmark of the matrix-free SR hot path on one MI355X.

A step is one pass of the hot path over one synthetic batch: the prepare/gradient pass
(column means, diag S, g and <E> in one read of O) followed by the persistent CG solve of
(S + eps I) x = g, whose products read O once each.  The default workload is the
CPS-shaped 32768 x 500000 matrix stored as bf16 codes with float32 column scales; the
float64 solve of the same matrix is timed beside it for the bf16-vs-f64 comparison.

Prints ONE JSON line on stdout (progress goes to stderr).
  value       algorithmic GB/s of the step: (one O read for the prepare pass + one O read
              per product) / step time, inputs resident in HBM
  roofline    the CG kernel (the step's dominant kernel): algorithmic bytes per launch /
              its duration measured with HIP events on its stream, against 8 TB/s
  cpu_baseline  the CPU oracle's matrix-free product on a bounded row sample, same unit;
              with the smaller workloads also the oracle's dense solve of the 8192 x 4000
              matrix on the host cores
  batched     64 independent float32 systems x 8 shifts in one launch; one system against
              8 single-column solves; the 8-column product alone
  adjoint     forward and backward of the differentiable solve on 16384 x 16384 float32,
              plain and Jacobi-preconditioned; sr_adjoint alone
  other_configs  dense 8192 x 4000 float64 and CPS 65536 x 24512 float64 / float32 solves;
              the linear method's Davidson eigensolve on the dense samples
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "SR CG solve time & S·v GB/s (frac of HBM peak), N_p=5e5 N_s=32k, BF16 vs FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def elem_bytes(dt):
    import torch
    return {torch.float64: 8, torch.float32: 4, torch.bfloat16: 2, torch.float16: 2}[dt]


def product_bytes(n_s, n_p, dt, scaled):
    """Algorithmic bytes of one product: one read of O in its storage type plus the O(N_p)
    vectors (scale, column mean, v, y) and the N_s row weights."""
    return n_s * n_p * elem_bytes(dt) + n_p * ((4 if scaled else 0) + 3 * 8) + n_s * 8


def grad_bytes(n_s, n_p, dt, scaled):
    """Algorithmic bytes of the prepare pass: one read of O and E, the O(N_p) outputs."""
    return n_s * n_p * elem_bytes(dt) + n_s * 8 + n_p * ((4 if scaled else 0) + 3 * 8)


KERNEL_SOURCES = ("sr_device.hpp", "sr_product.hpp", "sr_kernels.hpp", "sr_launch.hpp", "sr_kernels_bf16.hip")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_cg_step_bf16_compact_cps500k_traffic.md")
def step_kernel_name(tile):
    """Name of the bf16 split-CG search kernel of tile (nv, rows, lookahead, poll, threads)."""
    nv, r, look, pd, nt = tile
    return f"void sr::k_cg_step<2, {nv}, {r}, {look}, {pd}, {nt}>(sr::CgArgs)"


def kernel_source_hash():
    """sha256 of the device sources of the bf16 kernels (to tell whether a counter record
    still describes the built kernel)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1108_0900_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(kernel_name):
    """HBM bytes per launch of the CG kernel from the committed FETCH_SIZE / WRITE_SIZE
    record, or None if there is none for this kernel or its sources changed since."""
    try:
        text = open(TRAFFIC_RECORD).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel") != kernel_name or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def make_workload(name, device):
    import synth
    from synth.configs import CONFIGS
    cfg = CONFIGS[name]
    t0 = time.time()
    if cfg.kind == "cps":
        d = synth.cps_inputs(cfg.n_s, cfg.n_corr, cfg.n_states, cfg.n_dense, cfg.seed, device=device)
    else:
        d = synth.dense_inputs(cfg.n_s, cfg.n_p, cfg.seed, device=device)
    log(f"[bench] generated {name}: O {tuple(d['O'].shape)} in {time.time() - t0:.1f}s")
    return cfg, d


def timed_events(fn):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    e1.synchronize()
    return out, e0.elapsed_time(e1)


def host_facts():
    """The host the CPU baseline ran on: usable cores, CPU model, BLAS threads."""
    import platform
    facts = {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count(),
             "cpu_count": os.cpu_count(), "machine": platform.machine()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                facts["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        facts["blas"] = [{"api": i.get("internal_api"), "threads": i.get("num_threads")} for i in threadpool_info()]
    except Exception:
        pass
    return facts


def cpu_cg_timing(O_dev, E_dev, eps_rel, eps_abs, iters, gpu_products, name):
    """The oracle's matrix-free CG (two products with the stored O per iteration, float64,
    numpy/OpenBLAS) on the whole matrix of a workload, run for `iters` iterations; the
    full solve is estimated as the time per product times the GPU solve's product count."""
    import numpy as np
    import oracle as orc
    O = O_dev.double().cpu().numpy()
    E = E_dev.cpu().numpy()
    g = orc.energy_gradient(O, E)
    eps = eps_abs if eps_abs is not None else eps_rel * float(orc.diag_overlap(O).mean())
    t0 = time.perf_counter()
    _, it, _ = orc.cg_solve(lambda u: orc.sv_product_swapped(O, u, eps), g, rtol=1e-300, max_iter=iters)
    t = time.perf_counter() - t0
    per = t / max(it, 1)
    del O
    return {"workload": name, "iterations_timed": it, "s_per_iteration": round(per, 4),
            "gpu_products": gpu_products, "estimated_solve_s": round(per * gpu_products, 2),
            "method": "oracle cg_solve with sv_product_swapped (float64, numpy/OpenBLAS)"}


def cpu_baseline(O_dev, n_rows, eps, budget_s=15.0):
    """The oracle's matrix-free product (sv_product_swapped) on the first n_rows rows."""
    import numpy as np
    import oracle as orc
    sample = O_dev[:n_rows].double().cpu().numpy()
    n_p = sample.shape[1]
    v = np.random.default_rng(0).standard_normal(n_p)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    orc.sv_product_swapped(sample, v, eps)            # warm
    reps, t_tot = 0, 0.0
    while t_tot < budget_s and reps < 50:
        t0 = time.perf_counter()
        orc.sv_product_swapped(sample, v, eps)
        t_tot += time.perf_counter() - t0
        reps += 1
    t = t_tot / reps
    gbps = product_bytes(n_rows, n_p, __import__("torch").float64, False) / t / 1e9
    return {"value": round(gbps, 3), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle sv_product_swapped (float64, numpy/OpenBLAS) on the first {n_rows} rows x {n_p} "
                      f"columns of the same matrix, {reps} repetitions, {t * 1e3:.1f} ms each",
            "host": host_facts()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cps_32768x500000",
                    choices=["dense_8192x4000", "cps_65536x24512", "cps_32768x500000", "dense_16384"])
    ap.add_argument("--rtol", type=float, default=None, help="CG tolerance of the timed bf16 solve")
    ap.add_argument("--no-f64", action="store_true", help="skip the float64 comparison solve")
    ap.add_argument("--one-plane", action="store_true",
                    help="time the single-plane bf16 solve (no quantisation-remainder plane)")
    ap.add_argument("--two-planes", action="store_true",
                    help="time the solve over a full remainder plane (default: compact remainder plane)")
    ap.add_argument("--search-f64", action="store_true",
                    help="bf16 search-direction products accumulate in float64 too")
    ap.add_argument("--refresh-drop", type=float, default=None)
    ap.add_argument("--cpu-rows", type=int, default=256)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--quick", action="store_true",
                    help="timed steps only (for profiler passes): no tuning, float64 solves, standalone "
                         "products or CPU baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation-form measurement")
    ap.add_argument("--no-cps", action="store_true", help="skip the index-coded CPS storage measurement")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the dense 8192 x 4000 and CPS 65536 x 24512 solves")
    ap.add_argument("--batched-two-pass", action="store_true",
                    help="also time the two-pass 8-column batched solve (distinct right-hand sides)")
    ap.add_argument("--batched-systems", type=int, default=64,
                    help="systems of the batched workload timed in one launch (its first n)")
    ap.add_argument("--copy-gb", type=float, default=0.0,
                    help="after the steps, copy a buffer of this many GB three times (a plain kernel of "
                         "known traffic, to calibrate hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding over several GPUs is "
              f"designed but not built in this repository.", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    out = measure_single(args)
    torch.cuda.empty_cache()
    out["batched"] = None if (args.quick or args.no_batched) else measure_batched(args)
    torch.cuda.empty_cache()
    out["adjoint"] = None if (args.quick or args.no_adjoint) else measure_adjoint(args)
    torch.cuda.empty_cache()
    out["other_configs"] = None
    if not (args.quick or args.no_small):
        out["other_configs"], dense_case = measure_other_configs(args)
        if out["cpu_baseline"] is not None:
            out["cpu_baseline"]["dense_solve"] = cpu_baseline_dense(*dense_case)
    if out["cpu_baseline"] is not None:
        cg = [c for c in ((out.get("other_configs") or {}).pop("_cpu_cg", []) +
                          [(out.get("adjoint") or {}).pop("_cpu_cg", None)]) if c]
        out["cpu_baseline"]["cg_solves"] = cg
    print(json.dumps(out), flush=True)


def cpu_baseline_dense(O, E, x_gpu, x_gpu_tight):
    """The oracle's dense solve (explicit S, Cholesky, float64 on the host cores) of the
    dense 8192 x 4000 workload, and the GPU solutions' errors against it (CG to the
    workload's 1e-10 and to 1e-13)."""
    import numpy as np
    import oracle as orc
    t0 = time.perf_counter()
    x_ref = orc.solve_dense(O, orc.energy_gradient(O, E), 1e-3 * orc.diag_overlap(O).mean())
    t = time.perf_counter() - t0
    return {"workload": "dense float64 O 8192 x 4000, eps = 1e-3 mean(diag S)", "kind": "oracle",
            "method": "form S, Cholesky (numpy/OpenBLAS)", "seconds": round(t, 3),
            "gpu_cg_err_vs_oracle": float(np.linalg.norm(x_gpu - x_ref) / np.linalg.norm(x_ref)),
            "gpu_cg_rtol_1e-13_err_vs_oracle": float(np.linalg.norm(x_gpu_tight - x_ref) / np.linalg.norm(x_ref))}


def measure_other_configs(args):
    """Solves of the two smaller workloads: dense 8192 x 4000 float64 (CG to 1e-10, plain
    and Jacobi-preconditioned; the linear method's Davidson eigensolve and H product on
    the same samples) and CPS 65536 x 24512 in float64 and float32 (CG to 1e-8, error of
    float32 against float64).  Returns the record and the dense
    case's host arrays (O, E, x) for the CPU baseline."""
    import torch
    import synth
    from paper_1108_0900_amd import sr, tune
    dev = "cuda:0"
    res = {}
    cfg, d = make_workload("dense_8192x4000", dev)
    O, E = d["O"], d["E"]
    n_s, n_p = O.shape
    M = sr.as_matrix(O)
    tune.autotune(M, kind=0, reps=3)

    def solve(M, tol, precond=False):
        st = sr.sr_grad(M, E)
        M.mean = st["mean"]
        eps = 1e-3 * float(st["diag"].mean())
        sr.sr_cg_solve(M, st["g"], eps, rtol=tol, refresh_every=20, precond=precond)      # warm
        (x, info), ms = timed_events(lambda: sr.sr_cg_solve(M, st["g"], eps, rtol=tol, refresh_every=20,
                                                            precond=precond))
        if info["status"] != 0:
            raise RuntimeError(f"CG did not converge: {info}")
        return x, info, ms, eps
    x, info, ms, eps = solve(M, cfg.rtol)
    xt, infot, mst, _ = solve(M, 1e-13)
    xj, infoj, msj, _ = solve(M, cfg.rtol, True)
    pb = product_bytes(n_s, n_p, torch.float64, False)
    c1 = {"workload": "dense float64 O 8192 x 4000 N(0,1) x lognormal(0, 0.5), eps = 1e-3 mean(diag S), CG to 1e-10",
          "cg_ms": round(ms, 2), "iters": info["iters"], "products": info["products"],
          "GBps": round(info["products"] * pb / ms / 1e6, 1),
          "rtol_1e-13": {"cg_ms": round(mst, 2), "iters": infot["iters"], "products": infot["products"]},
          "jacobi": {"cg_ms": round(msj, 2), "iters": infoj["iters"], "products": infoj["products"],
                     "x_rel_diff_vs_plain": float(torch.linalg.vector_norm(xj - x) / torch.linalg.vector_norm(x))}}
    res["dense_8192x4000_f64"] = c1
    dense_case = (O.cpu().numpy(), E.cpu().numpy(), x.cpu().numpy(), xt.cpu().numpy())
    res["_cpu_cg"] = [cpu_cg_timing(O, E, 1e-3, None, 20, info["products"], "dense float64 O 8192 x 4000, CG to 1e-10")]
    # the linear method on the same samples: D = 0.1 N(0,1) s_j, lowest eigenpair of
    # H c = theta S c by generalized Davidson (one H and one S product per iteration), and
    # the H product alone
    Dt = synth.lm_derivatives(n_s, d["col_scale"], device=dev)
    Md = sr.as_matrix(Dt)
    M.mean = sr.sr_grad(M, None)["mean"]
    sr.lm_davidson(M, E, Md, tol=1e-8, max_sub=40)                          # warm
    (th, cvec, dinfo), ms_d = timed_events(lambda: sr.lm_davidson(M, E, Md, tol=1e-8, max_sub=40))
    (thp, cvp, dinfp), ms_p = timed_events(lambda: sr.lm_davidson(M, E, Md, tol=1e-8, max_sub=40, precond=1))
    (thx, cvx, dinfx), ms_x = timed_events(lambda: sr.lm_davidson(M, E, Md, tol=1e-8, max_sub=40, precond=2))
    v = torch.randn(n_p + 1, dtype=torch.float64, device=dev)
    sr.lm_hv_product(M, E, Md, v)
    ts = sorted(timed_events(lambda: sr.lm_hv_product(M, E, Md, v))[1] for _ in range(7))
    res["lm_davidson_8192x4000_f64"] = {
        "workload": "dense float64 O and D = 0.1 N(0,1) s_j, 8192 x 4000; lowest eigenpair to "
                    "||H c - theta S c|| <= 1e-8 |theta|, subspace 40",
        "ms": round(ms_d, 2), "iters": dinfo["iters"], "restarts": dinfo["restarts"], "theta": th,
        "res_norm": dinfo["res_norm"], "status": dinfo["status"],
        "approx_diagonal_correction": {"ms": round(ms_p, 2), "iters": dinfp["iters"],
                                       "restarts": dinfp["restarts"], "theta": thp, "status": dinfp["status"]},
        "exact_diagonal_correction": {"ms": round(ms_x, 2), "iters": dinfx["iters"],
                                      "restarts": dinfx["restarts"], "theta": thx, "status": dinfx["status"]},
        "lm_hv_product_ms": round(ts[3], 4),
        "lm_hv_product_GBps": round(2 * n_s * n_p * 8 / ts[3] / 1e6, 1)}
    del Dt, Md
    del d, O, M, x, xj
    torch.cuda.empty_cache()

    cfg, d = make_workload("cps_65536x24512", dev)
    O64, E = d["O"], d["E"]
    n_s, n_p = O64.shape
    out2 = {"workload": "CPS-shaped O 65536 x 24512 (64 correlators x 256 states + 8128 dense pairing columns), "
                        "eps = 1e-3 mean(diag S), CG to 1e-8"}
    xs = {}
    for name, Ot, dt in (("f64", O64, torch.float64), ("f32", O64.float(), torch.float32)):
        M = sr.as_matrix(Ot)
        tune.autotune(M, kind=0, reps=3)
        x, info, ms, _ = solve(M, cfg.rtol)
        xs[name] = x
        out2[name] = {"cg_ms": round(ms, 2), "iters": info["iters"], "products": info["products"],
                      "GBps": round(info["products"] * product_bytes(n_s, n_p, dt, False) / ms / 1e6, 1)}
        if name == "f64":
            res["_cpu_cg"].append(cpu_cg_timing(O64, E, 1e-3, None, 2, info["products"],
                                                "CPS-shaped float64 O 65536 x 24512, CG to 1e-8"))
        del M, Ot
    out2["f32_err_vs_f64"] = float(torch.linalg.vector_norm(xs["f32"] - xs["f64"]) /
                                   torch.linalg.vector_norm(xs["f64"]))
    res["cps_65536x24512"] = out2
    log(f"[bench] other configs: {res}")
    return res, dense_case


def measure_adjoint(args):
    """The differentiation form on dense float32 O 16384 x 16384, eps = 1e-3, L = w . x:
    forward (prepare pass + CG) and backward (adjoint CG + sr_adjoint) through
    torch.autograd, and sr_adjoint alone (one read of O, one write of dL/dO)."""
    import torch
    import synth
    from paper_1108_0900_amd import sr
    from paper_1108_0900_amd.autograd import sr_solve
    dev = "cuda:0"
    cfg = synth.CONFIGS["dense_16384"]
    d = synth.dense_inputs(cfg.n_s, cfg.n_p, cfg.seed, device=dev, dtype=torch.float32)
    O, E = d["O"], d["E"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(55)
    w = torch.randn(cfg.n_p, generator=gen, dtype=torch.float64, device=dev)
    rtol = 1e-9

    def fwd_bwd(precond=False):
        Ot = O.clone().requires_grad_(True)
        Et = E.clone().requires_grad_(True)
        torch.cuda.synchronize()
        x, ms_f = timed_events(lambda: sr_solve(Ot, Et, cfg.eps_abs, rtol, 20, precond))
        _, ms_b = timed_events(lambda: (x * w).sum().backward())
        return ms_f, ms_b, x.detach()
    fwd_bwd()                                                   # warm
    ms_f, ms_b, x_plain = fwd_bwd()
    ms_fj, ms_bj, x_jac = fwd_bwd(True)
    M = sr.as_matrix(O)
    st = sr.sr_grad(M, E)
    M.mean = st["mean"]
    x, info_x = sr.sr_cg_solve(M, st["g"], cfg.eps_abs, rtol=rtol, refresh_every=20)
    lam, info_l = sr.sr_cg_solve(M, w, cfg.eps_abs, rtol=rtol, refresh_every=20)
    _, info_xj = sr.sr_cg_solve(M, st["g"], cfg.eps_abs, rtol=rtol, refresh_every=20, precond=True)
    _, info_lj = sr.sr_cg_solve(M, w, cfg.eps_abs, rtol=rtol, refresh_every=20, precond=True)
    sr.sr_adjoint(M, E, x, lam, dO_dtype=torch.float32)
    ts = sorted(timed_events(lambda: sr.sr_adjoint(M, E, x, lam, dO_dtype=torch.float32))[1] for _ in range(5))
    gb = 2 * O.numel() * 4 / 1e9
    out = {"workload": "dense float32 O %d x %d N(0,1) x lognormal(0, 0.5), eps = %g, L = w . x, CG to %g, "
                       "refresh every 20" % (cfg.n_s, cfg.n_p, cfg.eps_abs, rtol),
           "forward_ms": round(ms_f, 2), "backward_ms": round(ms_b, 2),
           "forward_products": info_x["products"], "adjoint_cg_products": info_l["products"],
           "jacobi": {"forward_ms": round(ms_fj, 2), "backward_ms": round(ms_bj, 2),
                      "forward_products": info_xj["products"], "adjoint_cg_products": info_lj["products"],
                      "x_rel_diff_vs_plain": float(torch.linalg.vector_norm(x_jac - x_plain) /
                                                   torch.linalg.vector_norm(x_plain))},
           "sr_adjoint_ms": round(ts[2], 3), "sr_adjoint_GBps": round(gb / ts[2] * 1e3, 1),
           "_cpu_cg": None if args.quick else cpu_cg_timing(O, E, None, cfg.eps_abs, 5, info_x["products"],
                                                            "dense float32 O 16384 x 16384 (float64 on the host), "
                                                            "eps = 1e-3, CG to 1e-9")}
    log(f"[bench] adjoint: {out}")
    return out


def measure_batched(args):
    """The batched form: many independent systems (float32 O), 8 shifts each of one
    right-hand side, solved by multi-shift CG system after system in one persistent launch
    (one single-vector product per iteration per system, O read once per product).  Beside
    it: the same systems one multi-shift call each, the 8-column product, and (option) the
    two-pass 8-column batched solve meant for distinct right-hand sides."""
    import torch
    import synth
    from paper_1108_0900_amd import sr
    dev = "cuda:0"
    cfg = synth.CONFIGS["batched_64sys"]
    shapes = synth.batched_shapes(seed=cfg.seed)[: args.batched_systems]
    shifts = synth.relative_shifts(8)
    systems = []
    for s_i, (ns, npar) in enumerate(shapes):
        d = synth.dense_inputs(ns, npar, cfg.seed * 1000 + s_i, device=dev, dtype=torch.float32)
        M = sr.as_matrix(d["O"])
        st = sr.sr_grad(M, d["E"])
        M.mean = st["mean"]
        dS = float(st["diag"].mean())
        systems.append((M, st["g"], [dS * r for r in shifts]))
        del d
        if s_i % 8 == 7:
            log(f"[bench] batched workload: {s_i + 1} systems built")
    gb_o = [M.O.numel() * 4 / 1e9 for M, _, _ in systems]
    workload = ("%d independent systems, N_p in [1000, 60000], N_s in [4096, 32768], dense float32 O N(0,1) x "
                "lognormal(0, 0.5) column scales, 8 shifts 1e-4..1e-1 of mean(diag S) of one right-hand side (the "
                "SR gradient) each, CG to rel. true residual %g" % (len(systems), cfg.rtol))
    sr.sr_cg_solve_shifts_batched(systems[:2], rtol=cfg.rtol)      # warm
    log("[bench] batched: multi-shift CG of every system in one launch")
    sr.timing(True)
    (res, ms) = timed_events(lambda: sr.sr_cg_solve_shifts_batched(systems, rtol=cfg.rtol))
    launch_ms, launches = sr.timing_read("solve_launch")
    sr.timing(False)
    X, info, status = res
    # products of the launch: the shared sequence and the residual check of each shift
    prods = [min(c["products"] for c in sys_i) for sys_i in info]
    continued = sum(1 for sys_i in info for c in sys_i if c["products"] > min(x["products"] for x in sys_i))
    worst = max(c["rel_res_true"] for sys_i in info for c in sys_i)
    o_gb = sum(p * g for p, g in zip(prods, gb_o))
    out = {"workload": workload, "O_GB": round(sum(gb_o), 1), "method": "multi-shift CG, one persistent launch",
           "ms": round(ms, 1), "launch_ms": round(launch_ms, 1), "launches": launches, "status": status,
           "column_solves": 8 * len(systems), "products": sum(prods), "continued_shifts": continued,
           "worst_rel_res_true": worst, "O_read_GB": round(o_gb, 1),
           "O_GBps": round(o_gb / launch_ms * 1e3, 1), "frac": round(o_gb / launch_ms * 1e3 / HBM_PEAK_GBPS, 4)}
    del X
    # the same systems, one multi-shift call each
    worst_m = 0.0
    statuses = []
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for Ms, gs, es in systems:
        Xm, inf_m, st_m = sr.sr_cg_solve_shifts(Ms, gs, es, rtol=cfg.rtol)
        statuses.append(st_m)
        worst_m = max(worst_m, max(c["rel_res_true"] for c in inf_m))
        del Xm
    e1.record()
    e1.synchronize()
    out["multi_shift_one_call_per_system"] = {"ms": round(e0.elapsed_time(e1), 1), "calls": len(systems),
                                              "all_ok": all(st_m == 0 for st_m in statuses),
                                              "worst_rel_res_true": worst_m}
    # the 8-column product alone on the largest system (distinct right-hand sides)
    big = max(range(len(systems)), key=lambda k: gb_o[k])
    Mb = systems[big][0]
    V = torch.randn(8, Mb.n_p, dtype=torch.float64, device=dev)
    sr.sr_svk_product(Mb, V, [0.1] * 8)
    ts = sorted(timed_events(lambda: sr.sr_svk_product(Mb, V, [0.1] * 8))[1] for _ in range(5))
    ms_k = ts[2]
    ts1 = sorted(timed_events(lambda: sr.sr_sv_product(Mb, V[0], 0.1))[1] for _ in range(5))
    out["svk_product"] = {"n_s": Mb.O.shape[0], "n_p": Mb.n_p, "ms_8_columns": round(ms_k, 3),
                          "ms_1_column": round(ts1[2], 3),
                          "O_stream_GBps": round(2 * gb_o[big] / ms_k * 1e3, 1),
                          "columns_per_O_read_equivalent": round(8 * ts1[2] / ms_k, 2)}
    if args.batched_two_pass:
        # eight distinct right-hand sides per system: two-pass 8-column products in one launch
        sys8 = [(M, g.unsqueeze(0).repeat(8, 1).contiguous(), es) for M, g, es in systems]
        (res8, ms8) = timed_events(lambda: sr.sr_cg_solve_batched(sys8, rtol=cfg.rtol, refresh_every=20))
        out["two_pass_8_columns"] = {"ms": round(ms8, 1), "status": res8[2]}
    log(f"[bench] batched: {out}")
    return out


def measure_stream_ceiling(T, reps=3):
    """Streaming-read ceiling: sr_stream_read over the tensor T (the products' own loads),
    every built unroll and 1, 2, 4 workgroups per CU; the fastest setting's median GB/s."""
    import torch
    from paper_1108_0900_amd import sr
    nbytes = (T.numel() * T.element_size()) // 16 * 16
    out = {}
    for bpc in (1, 2, 4):
        for unroll in (2, 4, 8):
            sr.stream_read(T, bpc, unroll)
            ts = sorted(timed_events(lambda: sr.stream_read(T, bpc, unroll))[1] for _ in range(reps))
            out[f"{bpc}x{unroll}"] = round(nbytes / ts[len(ts) // 2] / 1e6, 1)
    best = max(out, key=out.get)
    return {"GBps": out[best], "frac": round(out[best] / HBM_PEAK_GBPS, 4), "bytes": nbytes,
            "setting_blocks_per_cu_x_unroll": best, "all": out,
            "kernel": "k_stream_read (sr_stream_read): non-temporal 16-byte loads, grid-stride"}


def cps_product_bytes(n_s, n_corr, n_states, n_d, dense_dt):
    """Algorithmic bytes of one product with index-coded CPS storage: one read of the state
    bytes and of the dense block, the O(N_p) vectors (v, y, column means of the dense
    block, the value table) and the N_s row values."""
    n_p = n_corr * n_states + n_d
    return n_s * n_corr + n_s * n_d * elem_bytes(dense_dt) + n_p * 3 * 8 + n_s * 8


def measure_cps(cfg, x64, rtol, refresh, dev):
    """The same workload in index-coded CPS storage (one state byte per correlator per
    sample, the pairing block dense): product time and GB/s against the algorithmic bytes
    of that form, CG solve time, and the error against the float64 dense-storage solution,
    for the pairing block in bf16 (float32 accumulation), float32 and float64."""
    import torch
    import synth
    from paper_1108_0900_amd import sr
    ix = synth.cps_index_inputs(cfg.n_s, cfg.n_corr, cfg.n_states, cfg.n_dense, cfg.seed, device=dev)
    out = {"state_bytes": int(cfg.n_s * cfg.n_corr), "forms": {}}
    v = torch.randn(cfg.n_p, dtype=torch.float64, device=dev)
    for name, dt in (("bf16", torch.bfloat16), ("f32", torch.float32), ("f64", torch.float64)):
        if dt == torch.bfloat16:
            q, s = sr.sr_quantize(ix["dense"], out_dtype=torch.bfloat16)
            Md = sr.as_matrix(q, scale=s)
        else:
            Md = sr.as_matrix(ix["dense"].to(dt))
        M = sr.cps_matrix(ix["idx"], ix["val"], cfg.n_states, Md)
        st = sr.sr_cps_grad(M, ix["E"])
        M.mean = st["mean"]
        eps = cfg.eps_rel * float(st["diag"].mean())
        alg = cps_product_bytes(cfg.n_s, cfg.n_corr, cfg.n_states, cfg.n_dense, dt)
        y = torch.empty_like(v)
        sr.sr_cps_sv_product(M, v, eps, out=y)
        ts = sorted(timed_events(lambda: sr.sr_cps_sv_product(M, v, eps, out=y))[1] for _ in range(7))
        pm = ts[len(ts) // 2]
        sr.sr_cps_cg_solve(M, st["g"], eps, rtol=rtol, refresh_every=refresh)       # warm
        (x, info), ms = timed_events(lambda: sr.sr_cps_cg_solve(M, st["g"], eps, rtol=rtol, refresh_every=refresh))
        rec = {"product_ms": round(pm, 4), "product_GBps": round(alg / pm / 1e6, 1),
               "product_frac": round(alg / pm / 1e6 / HBM_PEAK_GBPS, 4), "algorithmic_bytes_per_product": int(alg),
               "cg_ms": round(ms, 3), "iters": info["iters"], "products": info["products"],
               "per_product_ms": round(ms / max(info["products"], 1), 4),
               "rel_res_true": info["rel_res_true"], "rtol": rtol, "status": info["status"]}
        if x64 is not None:
            rec["err_vs_f64"] = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
        out["forms"][name] = rec
        log(f"[bench] cps index form, {name} pairing block: {rec}")
        del M, Md, x
    return out


def measure_stream(cfg, dev, n_batches=8):
    """Products during sampling over the index-coded CPS workload: its N_s samples arrive as
    n_batches batches of rows (the seeded per-batch generator stands in for a sampler), each
    added to uncentred accumulators for m vectors, centred once at the end (sr_stream_*).
    Time of one sample set, and GB/s against what the method must move: one read of every
    batch (state bytes, pairing block, energies) plus the accumulators' read and write and
    the m vectors per batch."""
    import torch
    import synth
    from paper_1108_0900_amd import sr
    rows = cfg.n_s // n_batches
    layout = synth.cps_stream_layout(cfg.n_corr, cfg.n_states, cfg.n_dense, cfg.seed, device=dev)
    n_p = cfg.n_corr * cfg.n_states + cfg.n_dense
    out = {"workload": "CPS %d correlators x %d states + %d pairing columns, %d samples fed as %d batches of "
                       "%d rows (one state byte per correlator, pairing block dense), centred once at the end"
                       % (cfg.n_corr, cfg.n_states, cfg.n_dense, cfg.n_s, n_batches, rows), "forms": {}}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        batches = []
        for b in range(n_batches):
            bt = synth.cps_stream_batch(layout, b, rows, device=dev, dense_dtype=torch.float64)
            if dt == torch.bfloat16:
                q, s = sr.sr_quantize(bt["dense"], out_dtype=torch.bfloat16)
                Md = sr.as_matrix(q, scale=s)
            else:
                Md = sr.as_matrix(bt["dense"].to(dt))
            batches.append((sr.cps_matrix(bt["idx"], layout["val"], cfg.n_states, Md), bt["E"]))
            del bt
        sample_bytes = cfg.n_s * (cfg.n_corr + cfg.n_dense * elem_bytes(dt) + 8)
        out["forms"][name] = {}
        for m in (1, 8):
            Z = torch.randn(m, n_p, dtype=torch.float64, device=dev)

            def run():
                acc = sr.sr_stream_begin(n_p, m, device=dev)
                for M, E in batches:
                    sr.sr_stream_accumulate(acc, M, E, Z)
                return sr.sr_stream_finish(acc, Z, 0.0)
            run()
            ts = sorted(timed_events(run)[1] for _ in range(5))
            ms = ts[len(ts) // 2]
            # per batch: the accumulators A (m x n_p), s1, se read and written, Z read
            acc_bytes = n_batches * n_p * 8 * (2 * m + 4 + m)
            alg = sample_bytes + acc_bytes
            out["forms"][name]["m%d" % m] = {"ms": round(ms, 3), "us_per_sample": round(1e3 * ms / cfg.n_s, 4),
                                             "sample_bytes": int(sample_bytes), "accumulator_bytes": int(acc_bytes),
                                             "GBps": round(alg / ms / 1e6, 1),
                                             "frac": round(alg / ms / 1e6 / HBM_PEAK_GBPS, 4)}
        log(f"[bench] products during sampling, {name} pairing block: {out['forms'][name]}")
        del batches
    return out


def measure_single(args):
    import torch
    from paper_1108_0900_amd import sr
    dev = "cuda:0"

    cfg, d = make_workload(args.config, dev)
    O64, E = d["O"], d["E"]
    n_s, n_p = O64.shape
    refresh = cfg.refresh_every or 20
    del d

    # ---- storage forms ----
    scaled = args.config == "cps_32768x500000"
    form = "plain"
    n_lo = 0
    if scaled:
        form = "one_plane" if args.one_plane else ("two_planes" if args.two_planes else "compact")
        q, s = sr.sr_quantize(O64, out_dtype=torch.bfloat16)
        M1 = sr.as_matrix(q, scale=s)                 # first code plane only
        if form == "compact":
            cols = sr.sr_remainder_columns(O64, s, torch.bfloat16)
            lo = sr.sr_quantize_remainder(O64, s, cols, torch.bfloat16)
            Mt = sr.as_matrix(q, scale=s, lo=lo, lo_cols=cols)
            n_lo = int(cols.numel())
        elif form == "two_planes":
            _, _, lo = sr.sr_quantize(O64, out_dtype=torch.bfloat16, with_lo=True)
            Mt = sr.as_matrix(q, scale=s, lo=lo)
        else:
            Mt = M1
        torch.cuda.synchronize()
        dt_t, dtype_name = torch.bfloat16, "bf16"
        default_rtol = 1e-6
        rtol = args.rtol if args.rtol is not None else default_rtol
    else:
        Mt = sr.as_matrix(O64)
        dt_t, dtype_name = O64.dtype, {torch.float64: "f64", torch.float32: "f32"}[O64.dtype]
        rtol = args.rtol if args.rtol is not None else cfg.rtol
    M64 = sr.as_matrix(O64)
    eb = elem_bytes(dt_t)

    # bytes of one product: the algorithmic count reads one plane of O (plus the O(N_p)
    # vectors); the streamed count adds what the storage form reads besides (the
    # remainder plane's columns)
    alg_pb = product_bytes(n_s, n_p, dt_t, scaled)
    extra_search = {"compact": n_s * n_lo * eb, "two_planes": n_s * n_p * eb}.get(form, 0)
    extra_res = {"compact": n_s * n_lo * eb, "two_planes": n_s * n_p * eb}.get(form, 0)

    # ---- tile autotuning (not timed): every built configuration on these matrices ----
    from paper_1108_0900_amd import tune
    tiles = {}
    for name, M in (("f64", M64), (dtype_name, Mt)):
        if name in tiles or args.quick:
            continue
        # scaled storage: timed on a short CG solve (its search steps and residual products
        # are separate kernels); float64: on the product
        res = tune.autotune(M, kind=0, reps=3, cg_iters=4 if M is Mt and scaled and form != "two_planes" else 0)
        tiles[name] = {"best": list(res["best"]), "ms": {str(list(k)): round(v, 3) for k, v in res["ms"].items()}}
        log(f"[bench] tuned {name}: {res['best']}  {tiles[name]['ms']}")
    drop = args.refresh_drop if args.refresh_drop is not None else 0.0

    def step(M, tol, search_f64=False):
        st = sr.sr_grad(M, E)
        M.mean = st["mean"]
        eps = 1e-3 * float(st["diag"].mean()) if cfg.eps_abs is None else cfg.eps_abs
        kw = dict(refresh_every=refresh, refresh_drop=drop, search_f64=search_f64)
        (x, info), ms_cg = timed_events(lambda: sr.sr_cg_solve(M, st["g"], eps, rtol=tol, **kw))
        if info["status"] != 0:
            raise RuntimeError(f"CG did not converge: {info}")
        return x, info, ms_cg, eps

    def solve_summary(info, ms, tol, dt):
        pb = product_bytes(n_s, n_p, dt, dt in (torch.bfloat16, torch.float16))
        return {"solve_ms": round(ms, 3), "iters": info["iters"], "products": info["products"],
                "rel_res_true": info["rel_res_true"], "rtol": tol, "GBps": round(info["products"] * pb / ms / 1e6, 1)}

    # ---- float64 solves of the same matrix (reference solution and time-to-accuracy) ----
    f64 = None
    x64 = None
    if scaled and not args.no_f64 and not args.quick:
        log("[bench] float64 solves")
        step(M64, 1e-10)      # warm
        x64, info64, ms64, _ = step(M64, 1e-10)
        xr, infor, msr, _ = step(M64, rtol)
        f64 = {"reference": solve_summary(info64, ms64, 1e-10, torch.float64),
               "same_rtol": solve_summary(infor, msr, rtol, torch.float64)}
        f64["same_rtol"]["err_vs_reference"] = float(torch.linalg.vector_norm(xr - x64) /
                                                     torch.linalg.vector_norm(x64))
        del xr
        log(f"[bench] f64: {f64}")

    # ---- single-plane bf16 solve, for its error against float64 (not timed as a step) ----
    err_one_plane = None
    if scaled and form != "one_plane" and x64 is not None:
        x1, info1, _, _ = step(M1, rtol)
        err_one_plane = float(torch.linalg.vector_norm(x1 - x64) / torch.linalg.vector_norm(x64))
        log(f"[bench] one-plane bf16 solve: {info1}, err vs f64 {err_one_plane:.3e}")
        del x1

    # ---- timed steps ----
    log(f"[bench] warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        step(Mt, rtol, args.search_f64)
    torch.cuda.synchronize()
    cg_ms, infos = [], []
    sr.timing(True)           # HIP events around the CG launches, on their stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, info, ms_cg, eps = step(Mt, rtol, args.search_f64)
        cg_ms.append(ms_cg)
        infos.append(info)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    launch_cls = "search_step" if (form in ("compact", "one_plane", "plain") and not args.search_f64) \
        else "solve_launch"
    t_ms, t_n = sr.timing_read(launch_cls)
    if launch_cls == "search_step" and t_n == 0 and sr.timing_read("solve_launch")[1] > 0:
        # small float64 / float32 products run the one-launch solve
        launch_cls = "solve_launch"
        t_ms, t_n = sr.timing_read(launch_cls)
    sr.timing(False)
    ms_per_step = wall_ms / args.steps
    products = sum(i["products"] for i in infos) / len(infos)
    # a converged solve makes one search-direction product per iteration; the others are
    # residual products (refreshes, exit checks)
    searches = sum(i["iters"] for i in infos) / len(infos)
    residuals = products - searches
    cg_alg_bytes = products * alg_pb
    cg_streamed_bytes = cg_alg_bytes + searches * extra_search + residuals * extra_res
    step_bytes = grad_bytes(n_s, n_p, dt_t, scaled) + cg_alg_bytes
    value = step_bytes / (ms_per_step * 1e6)
    cg_avg = sum(cg_ms) / len(cg_ms)
    # the dominant kernel: one search step per launch (a product and the CG updates) for
    # the split solves of scaled storage, the whole solve's launch otherwise
    if launch_cls == "search_step" and t_n == 0:
        # products below the per-launch state-check size run in queued rounds, untimed per
        # launch: the solve's average per product stands in
        launch_ms = cg_avg / max(products, 1)
        launch_alg = alg_pb
        launch_streamed = alg_pb + extra_search
        kernel_name = "k_cg_step (split CG; solve time per product)"
    elif launch_cls == "search_step":
        launch_ms = t_ms / max(t_n, 1)
        launch_alg = alg_pb
        launch_streamed = alg_pb + extra_search
        kernel_name = "k_cg_step (one search iteration of the split CG: fused product + CG updates)"
    else:
        launch_ms = t_ms / max(t_n, 1)
        launch_alg = cg_alg_bytes
        launch_streamed = cg_streamed_bytes
        kernel_name = "k_cg (persistent CG; products read O once each)"
    achieved = launch_alg / (launch_ms * 1e6)
    streamed = launch_streamed / (launch_ms * 1e6)
    log(f"[bench] {dtype_name} {form}: {ms_per_step:.2f} ms/step, CG {cg_avg:.2f} ms, products {products}, "
        f"{value:.0f} GB/s step, {achieved:.0f} GB/s CG (algorithmic), {streamed:.0f} GB/s streamed")

    # ---- standalone product timing ----
    def sv_time(M, reps=5):
        v = torch.randn(n_p, dtype=torch.float64, device=dev)
        y = torch.empty_like(v)
        sr.sr_sv_product(M, v, 0.1, out=y)
        ts = []
        for _ in range(reps):
            _, ms = timed_events(lambda: sr.sr_sv_product(M, v, 0.1, out=y))
            ts.append(ms)
        ts.sort()
        return ts[len(ts) // 2]
    sv = {}
    ceiling = None
    if args.copy_gb > 0:
        nbytes = int(args.copy_gb * 1e9) // 16 * 16
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        # the products' own load type: non-temporal 16-byte streaming reads of every byte
        for _ in range(3):
            sr.stream_read(src, 1, 4)
        torch.cuda.synchronize()
        log(f"[bench] counter calibration: 3 copies of {nbytes} bytes (read {nbytes}, write {nbytes} each), "
            f"3 streaming reads of the same {nbytes} bytes")
        del src, dst
    if args.quick:
        sv = None
    else:
        def rec(ms, alg, streamed_b=None):
            r = {"ms": round(ms, 3), "GBps": round(alg / ms / 1e6, 1), "frac": round(alg / ms / 1e6 / HBM_PEAK_GBPS, 4)}
            if streamed_b is not None:
                r["streamed_GBps"] = round(streamed_b / ms / 1e6, 1)
            return r
        if scaled:
            sv["bf16_one_plane"] = rec(sv_time(M1), alg_pb)
            if form in ("compact", "two_planes"):
                sv[f"bf16_{form}"] = rec(sv_time(Mt), alg_pb, alg_pb + extra_res)
            b64 = product_bytes(n_s, n_p, torch.float64, False)
            sv["f64"] = rec(sv_time(M64), b64)
        else:
            sv[dtype_name] = rec(sv_time(Mt), alg_pb)
        ceiling = measure_stream_ceiling(M1.O if scaled else Mt.O)
        log(f"[bench] streaming ceiling: {ceiling}")

    err = None
    if x64 is not None:
        err = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))

    # ---- CPU baseline (oracle, bounded sample) ----
    cpu = None
    if not args.quick:
        log("[bench] cpu baseline")
        cpu = cpu_baseline(O64, min(args.cpu_rows, n_s), eps, args.cpu_budget)

    cps = None
    if scaled and not args.quick and not args.no_cps:
        cps = measure_cps(cfg, x64, rtol, refresh, dev)
        cps["during_sampling"] = measure_stream(cfg, dev)

    # HBM traffic of the CG launch from the committed counter record (same kernel build and
    # same algorithmic bytes per launch), else null
    traffic = None
    used_tile = tuple(tiles[dtype_name]["best"]) if dtype_name in tiles else tuple(sr.tile_configs(dt_t, 0)[0])
    rec_t = traffic_record(step_kernel_name(used_tile[:5])) if (scaled and form == "compact") else None
    if rec_t is not None and abs(rec_t["algorithmic_bytes"] - alg_pb) <= 1e-6 * alg_pb:
        traffic = round(rec_t["traffic_bytes"] / 1e9, 1)

    forms = {"compact": "bf16 codes + float32 column scales + a bf16 remainder plane for the %d columns whose "
                        "one-plane error exceeds 2^-17 (the dense pairing columns); search products accumulate in "
                        "%s, residual refreshes in float64" % (n_lo, "float64" if args.search_f64 else "float32"),
             "two_planes": "bf16 codes + float32 column scales + a full bf16 remainder plane (4 bytes per element); "
                           "every product accumulates in float64",
             "one_plane": "bf16 codes + float32 column scales; search products accumulate in float32, refreshes in "
                          "float64"}
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"compact": "bf16 (f64 accumulation)" if args.search_f64 else "bf16 (f32 accumulation)",
                  "one_plane": "bf16 (f32 accumulation)",
                  "two_planes": "bf16 x2 planes (f64 accumulation)"}.get(form, dtype_name),
        "data": "synthetic",
        "config": {
            "workload": {"cps_32768x500000": "CPS-shaped O, 32768 samples x 500000 parameters (2048 correlators x 240 "
                                             "states + 8480 dense pairing columns), %s; prepare pass + CG to rel. "
                                             "residual %g, float64 residual refresh every %d" % (forms[form], rtol,
                                                                                                  refresh),
                         "dense_8192x4000": "dense O 8192 x 4000 float64; prepare pass + CG to %g" % rtol,
                         "cps_65536x24512": "CPS-shaped O 65536 x 24512 float64; prepare pass + CG to %g" % rtol,
                         "dense_16384": "dense O 16384 x 16384 float32; prepare pass + CG to %g" % rtol}[args.config],
            "n_s": n_s, "n_p": n_p, "seed": cfg.seed, "parallelism": "single GPU", "storage_form": form,
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": kernel_name,
                     "algorithmic_bytes_per_product": int(alg_pb),
                     "algorithmic_bytes_per_launch": int(round(launch_alg)),
                     "streamed_bytes_per_launch": int(round(launch_streamed)),
                     "streamed_GBps": round(streamed, 1), "launch_ms": round(launch_ms, 4),
                     "launches_timed": t_n,
                     "solve": {"cg_ms": round(cg_avg, 3), "algorithmic_GB": round(cg_alg_bytes / 1e9, 2),
                               "GBps": round(cg_alg_bytes / (cg_avg * 1e6), 1),
                               "frac": round(cg_alg_bytes / (cg_avg * 1e6) / HBM_PEAK_GBPS, 4)},
                     "stream_ceiling": ceiling,
                     "frac_of_stream_ceiling": round(achieved / ceiling["GBps"], 4) if ceiling else None},
        "cpu_baseline": cpu,
        "solve": {"cg_ms": round(cg_avg, 3), "iters": infos[-1]["iters"], "products": products,
                  "residual_products": residuals, "storage_form": form, "remainder_columns": n_lo,
                  "rel_res_true": infos[-1]["rel_res_true"], "rtol": rtol, "eps": eps},
        "sv_product": sv,
        "tiles": tiles,
        "f64_solve": f64,
        "err_vs_f64": err,
        "err_vs_f64_one_plane": err_one_plane,
        "cps_index": cps,
    }
    if f64 is not None:
        out["speedup_vs_f64_same_rtol"] = round(f64["same_rtol"]["solve_ms"] / cg_avg, 3)
    return out


if __name__ == "__main__":
    main()
