"""torch.autograd wrapper of the SR solve with the implicit-adjoint backward.

    x = SRSolve.apply(O, E, eps, rtol, refresh_every, precond)

solves (S + eps I) x = g with S and g sampled from O (float64 or float32, n_s x n_p) and
the local energies E (float64, n_s) (Sec. II.A, Eq. sr_lin_eq in its centred form).
Backward, for an incoming dL/dx:
    lambda = (S + eps I)^{-1} dL/dx          (a second CG solve, the same kernel)
    dL/dO, dL/dE                             (sr_adjoint: one read of O, one rank-2 write)
    dL/deps = -lambda . x                    (when eps is a tensor that requires grad)
Both solves take the same options (precond: Jacobi-preconditioned CG).  Everything runs
in libsr on the device; this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import sr


class SRSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, O: torch.Tensor, E: torch.Tensor, eps, rtol: float = 1e-10, refresh_every: int = 20,
                precond: bool = False):
        if O.dtype not in (torch.float64, torch.float32) or O.dim() != 2:
            raise ValueError("SRSolve: O must be a 2-D float64 or float32 tensor")
        eps_val = float(eps.detach()) if torch.is_tensor(eps) else float(eps)
        M = sr.as_matrix(O.detach())
        st = sr.sr_grad(M, E.detach())
        M.mean = st["mean"]
        x, info = sr.sr_cg_solve(M, st["g"], eps_val, rtol=rtol, refresh_every=refresh_every, precond=precond)
        if info["status"] != sr.SR_OK:
            raise RuntimeError(f"SRSolve: CG did not converge: {info}")
        ctx.save_for_backward(O, E, x, st["mean"])
        ctx.M = M
        ctx.eps_val = eps_val
        ctx.eps_is_tensor = torch.is_tensor(eps)
        ctx.rtol = rtol
        ctx.refresh_every = refresh_every
        ctx.precond = precond
        return x

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        O, E, x, mean = ctx.saved_tensors
        M = ctx.M
        M.mean = mean
        lam, info = sr.sr_cg_solve(M, gx.detach().to(torch.float64).contiguous(), ctx.eps_val, rtol=ctx.rtol,
                                   refresh_every=ctx.refresh_every, precond=ctx.precond)
        if info["status"] != sr.SR_OK:
            raise RuntimeError(f"SRSolve backward: CG did not converge: {info}")
        need_O, need_E = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        need_eps = ctx.needs_input_grad[2] and ctx.eps_is_tensor
        dO = dE = deps = None
        if need_O or need_E or need_eps:
            dO, dE, _, deps = sr.sr_adjoint(M, E.detach(), x, lam, dO_dtype=O.dtype if need_O else None,
                                            want_dE=need_E, want_deps=True)
            if dO is not None and dO.stride(0) != dO.shape[1]:
                dO = dO.contiguous()
            if not need_eps:
                deps = None
        return dO, dE, deps, None, None, None


def sr_solve(O: torch.Tensor, E: torch.Tensor, eps, rtol: float = 1e-10, refresh_every: int = 20,
             precond: bool = False) -> torch.Tensor:
    """Differentiable SR solve x = (S + eps I)^{-1} g (see SRSolve)."""
    return SRSolve.apply(O, E, eps, rtol, refresh_every, precond)
