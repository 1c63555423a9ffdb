"""torch.autograd.Function over the HIP forward and adjoint kernels.

AicaLJ.apply(x, eps, sigma, dil, species, precision) -> (F, U)
  x: [n,3] device positions (requires_grad allowed); eps, sigma: [n_species]
  tensors (any device, float64 recommended).  The backward pass calls the
  hand-written adjoint with G = dL/dF and gamma = dL/dU, recomputing every pair
  term instead of storing them.
"""
from __future__ import annotations

import torch


class AicaLJ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, eps, sigma, dil, species=None, precision="fp32"):
        from . import aica_bin, aica_forces
        xd = x.detach().contiguous()
        aica_bin(dil, xd)
        e = eps.detach().cpu().double().numpy()
        s = sigma.detach().cpu().double().numpy()
        F, uw, _ = aica_forces(dil, xd, species, e, s, precision=precision)
        ctx.dil, ctx.species, ctx.precision = dil, species, precision
        ctx.save_for_backward(xd, eps, sigma)
        U = uw[0].to(F.dtype)
        return F, U

    @staticmethod
    def backward(ctx, gF, gU):
        from . import aica_bin, aica_forces_adjoint
        xd, eps, sigma = ctx.saved_tensors
        if gF is None:
            gF = torch.zeros((xd.shape[0], 3), dtype=torch.float32 if ctx.precision == "fp32" else torch.float64,
                             device=xd.device)
        gamma = 0.0 if gU is None else float(gU.detach().double().cpu())
        if ctx.dil._pos is not xd:
            aica_bin(ctx.dil, xd)
        e = eps.detach().cpu().double().numpy()
        s = sigma.detach().cpu().double().numpy()
        gx, ge, gs = aica_forces_adjoint(ctx.dil, xd, gF.contiguous(), gamma, ctx.species, e, s,
                                         precision=ctx.precision)
        return (gx.to(xd.dtype), ge.to(device=eps.device, dtype=eps.dtype), gs.to(device=sigma.device,
                dtype=sigma.dtype), None, None, None)
