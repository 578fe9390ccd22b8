"""torch.autograd.Function over the iFCI energy.

Forward: embed, solve every increment and assemble E_iFCI on the GPU.
Backward: the adjoint is the weighted density matrices (Hellmann-Feynman),
dE/dh = gamma_w and dE/d(pq|rs) = Gamma_w / 2, computed by the HIP RDM
kernels from the converged vectors."""
from __future__ import annotations

import torch

from . import ifci


class IFCIEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, eri, problem, precision=ifci.FP64, opts=None):
        opts = opts or {}
        q = type(problem)(h.detach().cpu().numpy(), eri.detach().cpu().numpy(), problem.bodies,
                          problem.nocc, problem.order, getattr(problem, "e_const", 0.0))
        plan = ifci.Plan(q, precision=precision, device=h.device.index or 0, **opts)
        plan.attach(h.detach(), eri.detach())
        e, st, _, _ = plan.davidson()
        en = plan.energy(e, st)
        ctx.plan = plan
        return torch.tensor(en["total"], dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(ctx, grad):
        dh, dg = ctx.plan.rdm()
        ctx.plan.close()
        return grad * dh, grad * dg, None, None, None


def ifci_energy(h, eri, problem, precision=ifci.FP64, **opts):
    return IFCIEnergy.apply(h, eri, problem, precision, opts)
