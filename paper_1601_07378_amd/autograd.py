"""Differentiable local-potential energy on top of libvloc.

E = sum_n w_n Re <c_n | V c_n>, the energy of weighted bands in the local
potential (Sec. 2: the action of the diagonal V through the two transforms).

* forward: out = V_loc c (vloc_apply), e_n = Re <c_n|out_n> and E = sum w_n e_n,
  both reduced in FP64 on the GPU;
* backward: dE/dc_n = 2 w_n out_n (V_loc is Hermitian; this is
  dE/d(Re c) + i dE/d(Im c), the convention torch uses for real losses of
  complex inputs), dE/dV(j) = (1/N) sum_n w_n |psi_n(j)|^2 and dE/dw_n = e_n.
  The real-space psi_n is never stored.  With the whole-plane layout of the
  plane kernel, the forward pass accumulates the weighted density from the
  psi_n it computes for the application anyway (vloc_apply_density, band chunk
  by band chunk) and the backward pass only scales it by the upstream
  gradient; with the row-buffer layout (where the whole plane does not fit in
  LDS, e.g. 128^3 in FP64) the backward pass recomputes psi_n band chunk by
  band chunk in a density pass (vloc_density), which measured faster there
  than the fused pass.

Every arithmetic step runs in libvloc's kernels; torch holds the tensors.
"""
from __future__ import annotations

import torch

from .vloc import Plan


class LocalEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, V, w, plan: Plan):
        if ctx.needs_input_grad[1] and plan.whole_plane:
            out, rho = plan.apply_density(c, V, w)
        else:
            out, rho = plan.apply(c, V), None
        e = plan.band_dot(c, out)
        E = plan.weighted_sum(e, w)
        ctx.plan = plan
        ctx.V_dtype = V.dtype
        ctx.rho = rho
        ctx.save_for_backward(c, w, out, e)
        return E

    @staticmethod
    def backward(ctx, gE):
        c, w, out, e = ctx.saved_tensors
        plan: Plan = ctx.plan
        g = gE.detach().to(torch.float64).reshape(1).contiguous()
        grad_c = grad_V = grad_w = None
        if ctx.needs_input_grad[0]:
            grad_c = plan.scale_bands(out, w, g, factor=2.0)
        if ctx.needs_input_grad[1]:
            if ctx.rho is not None:
                grad_V = plan.scale_real(ctx.rho, g).to(ctx.V_dtype)
            else:
                grad_V = plan.density(c, w, scale=g).to(ctx.V_dtype)
            ctx.rho = None
        if ctx.needs_input_grad[2]:
            grad_w = e * g
        return grad_c, grad_V, grad_w, None


def local_energy(plan: Plan, c, V, w):
    """E = sum_n w_n Re <c_n | V c_n> with autograd support for c, V and w."""
    return LocalEnergy.apply(c, V, w, plan)
