"""Tile-configuration autotuner for the fused products.

libsr is built with several tile configurations per storage type (16-byte vectors per
thread, rows per tile, lookahead, poll depth, threads; `sr.tile_configs`).  Which one is
fastest depends on the matrix shape: the number of column groups that exchange partial
dots per row, the rows per row group, and the bytes per element.  `autotune` times every
configuration on the caller's own matrix with HIP events and selects the fastest for
that storage type and product kind, process-wide (`sr.set_tile_config`).  Results can
be cached in a JSON file keyed by device, storage type, shape and product kind, so a
later process reuses them without timing.  The CG solve uses the configuration of the SR product (kind 0);
with `cg_iters` > 0 the configurations are timed on a CG solve of that many iterations
(what the solve runs: for scaled storage its search steps and residual products are
separate kernels, which need not rank like the standalone product).
Kind 2 tunes the batched products' geometry (`sr.BATCH_CONFIGS`: rows per update split,
tasks per workgroup) by timing the 8-column product on the caller's matrix.
"""
from __future__ import annotations

import json
import os

import torch

from . import sr

CACHE_ENV = "SR_TUNE_CACHE"


def _key(M: sr.Matrix, kind: int, cg_iters: int = 0) -> str:
    dev = torch.cuda.get_device_name(M.O.device)
    extra = f"|cg{cg_iters}|lo{M.n_lo}" if cg_iters else ""
    return f"{dev}|{str(M.O.dtype).split('.')[-1]}|{M.O.shape[0]}|{M.n_p}|kind{kind}{extra}"


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(path, table):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _median_ms(fn, reps: int, warm: int = 1) -> float:
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


_VEC = {torch.float64: 2, torch.float32: 4, torch.bfloat16: 8, torch.float16: 8}


def _col_group_choices(M: sr.Matrix, cfg) -> list:
    """0 (automatic) and, when the automatic choice may be an uneven number of column
    groups, the power of two that holds the streamed columns."""
    if M.O.dtype == torch.float64:
        return [0]
    nv, _, _, _, nt = cfg
    vec = _VEC[M.O.dtype]
    n_v = M.n_p if M.lo_cols is None else -(-M.n_p // vec) * vec + M.lo_cols.numel()
    cmin = -(-n_v // (nv * vec * nt))
    p2 = 1
    while p2 < cmin:
        p2 *= 2
    return [0, p2] if cmin < p2 <= 256 and cmin <= 32 else [0]


def autotune(M: sr.Matrix, kind: int = 0, reps: int = 3, cache_path: str | None = None,
             E: torch.Tensor | None = None, D: sr.Matrix | None = None, apply: bool = True,
             cg_iters: int = 0) -> dict:
    """Time every built configuration of the product of `kind` (0: (S + eps I) v,
    1: linear-method H v, which needs E and D, 2: the 8-column batched product, whose
    configurations are (split_rows, tasks)) on M; select the fastest if `apply`.
    kind 0 with cg_iters > 0 times a CG solve of cg_iters iterations instead (M may carry a
    compact remainder plane then).

    Returns {"best": (nv, rows, lookahead, poll_depth, threads, col_groups), "ms": {config: ms},
    "cached": bool}.  A configuration whose call fails (for example, one that cannot hold
    n_p columns) is skipped.  M's column means are computed first if missing.
    """
    if kind not in (0, 1, 2):
        raise ValueError("kind must be 0 (SR product), 1 (linear-method product) or 2 (batched products)")
    if kind == 1 and (E is None or D is None):
        raise ValueError("the linear-method product needs E and D")
    if M.lo is not None and not (kind == 0 and cg_iters > 0 and M.lo_cols is not None):
        raise ValueError("tune the first code plane alone (full two-plane products use a fixed tile)")
    cache_path = cache_path or os.environ.get(CACHE_ENV)
    table = _load(cache_path)
    key = _key(M, kind, cg_iters if kind == 0 else 0)
    if key in table:
        best = tuple(table[key]["best"])
        if apply:
            if kind == 2:
                sr.set_batch_config(*best)
            else:
                sr.set_tile_config(M.O.dtype, kind, *best)
        return {"best": best, "ms": {tuple(json.loads(k)): v for k, v in table[key]["ms"].items()}, "cached": True}

    if M.mean is None:
        M.mean = sr.sr_grad(M, None)["mean"]
    gen = torch.Generator(device=M.O.device)
    gen.manual_seed(0)
    if kind == 2:
        V = torch.randn(8, M.n_p, generator=gen, dtype=torch.float64, device=M.O.device)
        Y = torch.empty_like(V)
        times = {}
        try:
            for cfg in sr.BATCH_CONFIGS:
                sr.set_batch_config(*cfg)
                times[cfg] = _median_ms(lambda: sr.sr_svk_product(M, V, [0.1] * 8, out=Y), reps)
        finally:
            sr.set_batch_config()
        best = min(times, key=times.get)
        if apply:
            sr.set_batch_config(*best)
        table[key] = {"best": list(best), "ms": {json.dumps(list(k)): v for k, v in times.items()}}
        _save(cache_path, table)
        return {"best": best, "ms": times, "cached": False}
    n = M.n_p + (1 if kind == 1 else 0)
    v = torch.randn(n, generator=gen, dtype=torch.float64, device=M.O.device)
    y = torch.empty_like(v)
    if kind == 0 and cg_iters > 0:
        g = torch.randn(M.n_p, generator=gen, dtype=torch.float64, device=M.O.device)
        x = torch.empty_like(g)

        def call():
            sr.sr_cg_solve(M, g, 0.1, rtol=1e-300, max_iter=cg_iters, refresh_every=0, out=x,
                           raise_on=(sr.SR_ERR_INVALID, sr.SR_ERR_NOMEM, sr.SR_ERR_HIP, sr.SR_ERR_NODEVICE,
                                     sr.SR_ERR_TIMEOUT))
    elif kind == 0:
        def call():
            sr.sr_sv_product(M, v, 0.1, out=y)
    else:
        def call():
            sr.lm_hv_product(M, E, D, v, out=y)

    times = {}
    try:
        for cfg in sr.tile_configs(M.O.dtype, kind):
            # the automatic column groups (uneven ones where they give more row groups, for
            # 4- and 2-byte storage) and, where that differs, the power of two above them
            for cg in _col_group_choices(M, cfg):
                sr.set_tile_config(M.O.dtype, kind, *cfg, col_groups=cg)
                try:
                    times[cfg + (cg,)] = _median_ms(call, reps)
                except sr.SrError:
                    continue
    finally:
        sr.set_tile_config(M.O.dtype, kind)
    if not times:
        raise RuntimeError("no tile configuration could run this product")
    best = min(times, key=times.get)
    if apply:
        sr.set_tile_config(M.O.dtype, kind, *best)
    table[key] = {"best": list(best), "ms": {json.dumps(list(k)): v for k, v in times.items()}}
    _save(cache_path, table)
    return {"best": best, "ms": times, "cached": False}
