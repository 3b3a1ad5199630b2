"""torch.autograd.Function around the long-range step.

forward returns E (a 0-d float64 device tensor); backward returns dE/dr for
ions and for Wannier centroids computed by the library (-g * F).  The WC part
is the gradient a Deep Wannier model chains back to the atoms through
W_n = R_i + Delta_n (the force chain-rule equations of the DPLR background
section).  Charges are treated as constants (no gradient)."""
from __future__ import annotations

import torch


class DPLRLongRange(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ion_pos, wc_pos, ion_q, wc_q, plan):
        energy, f_ion, f_wc, virial = plan.compute(ion_pos.detach().contiguous(), ion_q.detach().contiguous(),
                                                   wc_pos.detach().contiguous(), wc_q.detach().contiguous())
        plan.last_virial = virial
        ctx.plan = plan
        ctx.save_for_backward(f_ion, f_wc)
        ctx.mark_non_differentiable(virial)
        return energy

    @staticmethod
    def backward(ctx, grad_energy):
        f_ion, f_wc = ctx.saved_tensors
        g_ion, g_wc = ctx.plan.scale_grad(grad_energy.reshape(()), f_ion, f_wc)
        return g_ion, g_wc, None, None, None


def dplr_long_range(ion_pos, wc_pos, ion_q, wc_q, plan):
    """E_Gt of the given ions and WCs with autograd support on both position sets."""
    return DPLRLongRange.apply(ion_pos, wc_pos, ion_q, wc_q, plan)
