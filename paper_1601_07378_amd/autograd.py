"""Differentiable local-potential energy on top of libvloc.

E = sum_n w_n Re <c_n | V c_n>, the energy of weighted bands in the local
potential (Sec. 2: the action of the diagonal V through the two transforms).

* forward: out = V_loc c (vloc_apply), e_n = Re <c_n|out_n> and E = sum w_n e_n,
  both reduced in FP64 on the GPU;
* backward: dE/dc_n = 2 w_n out_n (V_loc is Hermitian; this is
  dE/d(Re c) + i dE/d(Im c), the convention torch uses for real losses of
  complex inputs), dE/dV(j) = (1/N) sum_n w_n |psi_n(j)|^2 computed by the
  density pass, which recomputes psi_n band chunk by band chunk instead of
  storing it, and dE/dw_n = e_n.

Every arithmetic step runs in libvloc's kernels; torch holds the tensors.
"""
from __future__ import annotations

import torch

from .vloc import Plan


class LocalEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, V, w, plan: Plan):
        out = plan.apply(c, V)
        e = plan.band_dot(c, out)
        E = plan.weighted_sum(e, w)
        ctx.plan = plan
        ctx.V_dtype = V.dtype
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
            grad_V = plan.density(c, w, scale=g).to(ctx.V_dtype)
        if ctx.needs_input_grad[2]:
            grad_w = e * g
        return grad_c, grad_V, grad_w, None


def local_energy(plan: Plan, c, V, w):
    """E = sum_n w_n Re <c_n | V c_n> with autograd support for c, V and w."""
    return LocalEnergy.apply(c, V, w, plan)
