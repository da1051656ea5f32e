"""Seeded synthetic workloads.

The paper's samples come from variational Monte Carlo runs that are not available, so
random matrices with the shapes, value distributions and sparsity of its examples stand
in for them (Sec. III; parameter counts 4x10^3 to 5x10^5).  Every generator takes a seed
and a torch device; the same call on the same device always returns the same tensors.

Distribution conventions: N(0, a) has variance a; lognormal(0, b) has log-standard-
deviation b.  Local energies follow one recipe everywhere:
    E_k = -20 + 0.3 (O_k . u) + N(0, 1),   u ~ N(0, 1/N_p).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch


@dataclass(frozen=True)
class Config:
    name: str
    kind: str                 # "dense" | "cps" | "batched"
    n_s: int
    n_p: int
    seed: int
    dtypes: tuple
    rtol: float
    eps_rel: float | None = None     # eps = eps_rel * mean(diag S)
    eps_abs: float | None = None     # eps given directly
    n_corr: int = 0
    n_states: int = 0
    n_dense: int = 0
    refresh_every: int = 0
    extra: dict = field(default_factory=dict)


CONFIGS = {
    # dense O 8192 x 4000 float64 (4,048-parameter scale of the hydrogen lattice, Sec. III.C)
    "dense_8192x4000": Config("dense_8192x4000", "dense", 8192, 4000, 1, ("f64",), 1e-10, eps_rel=1e-3),
    # CPS-shaped: 64 plaquettes x 256 states + 8128 pairing columns (8x8 lattice, Sec. III.B)
    "cps_65536x24512": Config("cps_65536x24512", "cps", 65536, 64 * 256 + 8128, 2, ("f64", "f32"), 1e-8, eps_rel=1e-3,
                 n_corr=64, n_states=256, n_dense=8128),
    # CPS-shaped, 500,000 parameters (524,784-parameter scale of Sec. III.A), bf16 vs f64
    "cps_32768x500000": Config("cps_32768x500000", "cps", 32768, 2048 * 240 + 8480, 3, ("bf16", "f64"), 1e-10, eps_rel=1e-3,
                 n_corr=2048, n_states=240, n_dense=8480, refresh_every=20),
    # 64 independent systems, 8 relative shifts each
    "batched_64sys": Config("batched_64sys", "batched", 0, 0, 4, ("f32",), 1e-8, extra={"n_sys": 64, "n_shift": 8,
                 "n_p_range": (1000, 60000), "n_s_range": (4096, 32768)}),
    # differentiation case, f32 O, absolute eps
    "dense_16384": Config("dense_16384", "dense", 16384, 16384, 5, ("f32",), 1e-10, eps_abs=1e-3),
}


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    return g


def _energies(O: torch.Tensor, gen: torch.Generator, row_chunk: int = 4096) -> torch.Tensor:
    """E_k = -20 + 0.3 (O_k . u) + N(0,1), u ~ N(0, 1/N_p); O_k . u in float64."""
    n_s, n_p = O.shape
    dev = O.device
    u = torch.randn(n_p, generator=gen, device=dev, dtype=torch.float64) * math.sqrt(1.0 / n_p)
    noise = torch.randn(n_s, generator=gen, device=dev, dtype=torch.float64)
    ou = torch.empty(n_s, dtype=torch.float64, device=dev)
    for r0 in range(0, n_s, row_chunk):
        r1 = min(n_s, r0 + row_chunk)
        ou[r0:r1] = O[r0:r1].to(torch.float64) @ u
    return -20.0 + 0.3 * ou + noise


def dense_inputs(n_s: int, n_p: int, seed: int, device="cpu", dtype=torch.float64,
                 scale_sigma: float = 0.5, row_chunk: int = 4096):
    """Dense O_kj = N(0,1) s_j with s_j ~ lognormal(0, scale_sigma), plus E.

    Returns dict(O, E, col_scale) with O of shape (n_s, n_p) in `dtype`."""
    gen = _gen(seed, device)
    s = torch.exp(scale_sigma * torch.randn(n_p, generator=gen, device=device, dtype=torch.float64))
    O = torch.empty(n_s, n_p, dtype=dtype, device=device)
    for r0 in range(0, n_s, row_chunk):
        r1 = min(n_s, r0 + row_chunk)
        blk = torch.randn(r1 - r0, n_p, generator=gen, device=device, dtype=torch.float64) * s
        O[r0:r1] = blk.to(dtype)
        del blk
    E = _energies(O, gen)
    return {"O": O, "E": E, "col_scale": s}


def cps_inputs(n_s: int, n_corr: int, n_states: int, n_dense: int, seed: int, device="cpu",
               dtype=torch.float64, dense_var: float = 0.2, row_chunk: int = 4096):
    """CPS-shaped O: for each correlator p, every row has exactly one nonzero among that
    correlator's n_states columns, at a uniformly drawn state s_kp, with value 1/c_{p,s}
    (c ~ U[0.5, 1.5] drawn once per column); then n_dense pairing columns N(0, dense_var).

    Columns are ordered [correlator 0 states | correlator 1 states | ... | dense].
    Returns dict(O, E, c, state) where c has shape (n_corr, n_states) and state (n_s, n_corr).
    The vector with entries c_{p,s} on correlator p's columns and zeros elsewhere is, for
    every p, a null vector of the centred overlap (each row holds exactly one 1/c there).
    """
    gen = _gen(seed, device)
    n_sparse = n_corr * n_states
    n_p = n_sparse + n_dense
    c = 0.5 + torch.rand(n_corr, n_states, generator=gen, device=device, dtype=torch.float64)
    inv_c = (1.0 / c).to(dtype)
    state = torch.empty(n_s, n_corr, dtype=torch.int64, device=device)
    O = torch.zeros(n_s, n_p, dtype=dtype, device=device)
    pcols = (torch.arange(n_corr, device=device, dtype=torch.int64) * n_states)[None, :]
    for r0 in range(0, n_s, row_chunk):
        r1 = min(n_s, r0 + row_chunk)
        st = torch.randint(0, n_states, (r1 - r0, n_corr), generator=gen, device=device)
        state[r0:r1] = st
        cols = pcols + st
        vals = inv_c.reshape(-1)[cols.reshape(-1)].reshape(r1 - r0, n_corr)
        O[r0:r1].scatter_(1, cols, vals)
        if n_dense:
            d = torch.randn(r1 - r0, n_dense, generator=gen, device=device, dtype=torch.float64)
            O[r0:r1, n_sparse:] = (d * math.sqrt(dense_var)).to(dtype)
            del d
    E = _energies(O, gen)
    return {"O": O, "E": E, "c": c, "state": state}


def small_cps_inputs(seed: int = 12, device="cpu", dtype=torch.float64, n_s: int = 3000,
                     n_corr: int = 6, n_states: int = 16, n_dense: int = 70):
    """A CPS-shaped case small enough for the dense oracle."""
    return cps_inputs(n_s, n_corr, n_states, n_dense, seed, device=device, dtype=dtype)


def lm_derivatives(n_s: int, col_scale: torch.Tensor, seed: int = 6, device="cpu", dtype=torch.float64):
    """Local-energy derivatives D_kj = 0.1 N(0,1) s_j for the linear-method product."""
    gen = _gen(seed, device)
    n_p = col_scale.shape[0]
    d = torch.randn(n_s, n_p, generator=gen, device=device, dtype=torch.float64) * 0.1
    return (d * col_scale.to(device=device, dtype=torch.float64)).to(dtype)


def batched_shapes(seed: int = 4, n_sys: int = 64, n_p_range=(1000, 60000), n_s_range=(4096, 32768)):
    """(N_s, N_p) of each independent system, drawn uniformly (inclusive ranges)."""
    gen = _gen(seed, "cpu")
    n_p = torch.randint(n_p_range[0], n_p_range[1] + 1, (n_sys,), generator=gen)
    n_s = torch.randint(n_s_range[0], n_s_range[1] + 1, (n_sys,), generator=gen)
    return [(int(a), int(b)) for a, b in zip(n_s.tolist(), n_p.tolist())]


def relative_shifts(n_shift: int = 8) -> list:
    """Shifts 10^-4 .. 10^-1, log-spaced, relative to mean(diag S) of each system."""
    if n_shift == 1:
        return [1e-4]
    return [10.0 ** (-4.0 + 3.0 * i / (n_shift - 1)) for i in range(n_shift)]


def cps_index_inputs(n_s: int, n_corr: int, n_states: int, n_dense: int, seed: int, device="cpu",
                     dense_dtype=torch.float64, dense_var: float = 0.2, row_chunk: int = 4096):
    """The matrix of cps_inputs (same seed, the same random draws in the same order) in
    index-coded form, without building the n_s x n_p matrix:

      idx   (n_corr, ld) uint8, correlator-major, ld = n_s rounded up to 16 (the padding
            holds 0xFF, a state that selects no column); idx[p, k] = s_kp
      val   (n_corr * n_states,) float64, 1/c_{p,s}
      dense (n_s, n_dense) in dense_dtype (None when n_dense = 0)
      E     (n_s,) float64 by the same recipe, O_k . u summed over the sample's states
            and the dense block in float64 (equal to cps_inputs' E up to rounding order)

    Returns dict(idx, val, dense, E, c, n_states).  Requires n_states <= 256.
    """
    if n_states > 256:
        raise ValueError("index-coded storage holds at most 256 states per correlator")
    gen = _gen(seed, device)
    n_sparse = n_corr * n_states
    n_p = n_sparse + n_dense
    c = 0.5 + torch.rand(n_corr, n_states, generator=gen, device=device, dtype=torch.float64)
    val = (1.0 / c).reshape(-1)
    ld = ((n_s + 15) // 16) * 16
    idx = torch.full((n_corr, ld), 255, dtype=torch.uint8, device=device)
    dense = torch.empty(n_s, n_dense, dtype=dense_dtype, device=device) if n_dense else None
    states = []
    for r0 in range(0, n_s, row_chunk):
        r1 = min(n_s, r0 + row_chunk)
        st = torch.randint(0, n_states, (r1 - r0, n_corr), generator=gen, device=device)
        idx[:, r0:r1] = st.t().to(torch.uint8)
        states.append((r0, r1, st))
        if n_dense:
            d = torch.randn(r1 - r0, n_dense, generator=gen, device=device, dtype=torch.float64)
            dense[r0:r1] = (d * math.sqrt(dense_var)).to(dense_dtype)
            del d
    u = torch.randn(n_p, generator=gen, device=device, dtype=torch.float64) * math.sqrt(1.0 / n_p)
    noise = torch.randn(n_s, generator=gen, device=device, dtype=torch.float64)
    vu = val * u[:n_sparse]
    pcols = (torch.arange(n_corr, device=device, dtype=torch.int64) * n_states)[None, :]
    ou = torch.empty(n_s, dtype=torch.float64, device=device)
    for r0, r1, st in states:
        ou[r0:r1] = vu[pcols + st].sum(dim=1)
        if n_dense:
            ou[r0:r1] += dense[r0:r1].to(torch.float64) @ u[n_sparse:]
    E = -20.0 + 0.3 * ou + noise
    return {"idx": idx[:, :n_s], "val": val, "dense": dense, "E": E, "c": c, "n_states": n_states}


def cps_stream_layout(n_corr: int, n_states: int, n_dense: int, seed: int, device="cpu") -> dict:
    """The fixed part of a streamed CPS sample set: the correlator values val = 1/c (c ~
    U[0.5, 1.5] once per column) and the energy recipe's u ~ N(0, 1/N_p)."""
    gen = _gen(seed, device)
    n_p = n_corr * n_states + n_dense
    c = 0.5 + torch.rand(n_corr, n_states, generator=gen, device=device, dtype=torch.float64)
    u = torch.randn(n_p, generator=gen, device=device, dtype=torch.float64) * math.sqrt(1.0 / n_p)
    return {"n_corr": n_corr, "n_states": n_states, "n_dense": n_dense, "seed": seed, "c": c,
            "val": (1.0 / c).reshape(-1), "u": u}


def cps_stream_batch(layout: dict, batch: int, n_rows: int, device="cpu", dense_dtype=torch.float64,
                     dense_var: float = 0.2) -> dict:
    """Batch `batch` of a streamed CPS sample set (a stand-in for the rows a sampler produces
    one configuration at a time): n_rows samples, each in a uniform state of every correlator
    plus N(0, dense_var) pairing derivatives, and E by the recipe of this module.  The batch is
    a function of (layout seed, batch) alone, so it can be produced again instead of stored.
    Returns dict(idx (n_corr, n_rows) uint8 correlator-major, dense (n_rows, n_dense), E)."""
    n_corr, ns, nd = layout["n_corr"], layout["n_states"], layout["n_dense"]
    gen = _gen(layout["seed"] * 1000003 + 7919 * (batch + 1), device)
    ld = ((n_rows + 15) // 16) * 16
    idx = torch.full((n_corr, ld), 255, dtype=torch.uint8, device=device)
    st = torch.randint(0, ns, (n_rows, n_corr), generator=gen, device=device)
    idx[:, :n_rows] = st.t().to(torch.uint8)
    dense = None
    u = layout["u"]
    n_sparse = n_corr * ns
    ou = torch.zeros(n_rows, dtype=torch.float64, device=device)
    if n_corr:
        pcols = (torch.arange(n_corr, device=device, dtype=torch.int64) * ns)[None, :]
        ou += (layout["val"] * u[:n_sparse])[pcols + st].sum(dim=1)
    if nd:
        d = torch.randn(n_rows, nd, generator=gen, device=device, dtype=torch.float64) * math.sqrt(dense_var)
        dense = d.to(dense_dtype)
        ou += dense.to(torch.float64) @ u[n_sparse:]
    E = -20.0 + 0.3 * ou + torch.randn(n_rows, generator=gen, device=device, dtype=torch.float64)
    return {"idx": idx[:, :n_rows], "dense": dense, "E": E}
