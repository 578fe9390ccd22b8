"""torch.autograd.Function over the iFCI energy.

Forward: embed, solve every increment and assemble E_iFCI on the GPU.
Backward: the adjoint is the weighted density matrices (Hellmann-Feynman),
dE/dh = gamma_w and dE/d(pq|rs) = Gamma_w / 2, computed by the HIP RDM
kernels from the converged vectors."""
from __future__ import annotations

from types import SimpleNamespace

import torch

from . import ifci


class IFCIEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, eri, problem, precision=ifci.FP64, opts=None):
        opts = opts or {}
        # the plan needs only the partition and the order; the integrals stay
        # on the device
        shape = SimpleNamespace(n_orb=int(h.shape[0]), bodies=problem.bodies, nocc=problem.nocc,
                                order=problem.order, e_const=getattr(problem, "e_const", 0.0))
        plan = ifci.Plan(shape, precision=precision, device=h.device.index or 0, **opts)
        plan.attach(h.detach(), eri.detach())
        e, st, _, _ = plan.davidson()
        en = plan.energy(e, st)
        if not en["converged"]:
            n_bad = int((st != ifci.INC_DONE).sum())
            plan.close()
            raise RuntimeError(f"iFCI energy: {n_bad} increments did not converge; the energy and its "
                               "Hellmann-Feynman gradient would not be those of the eigenstates")
        # the plan (with its converged vectors) lives as long as the graph node
        ctx.plan = plan
        return torch.tensor(en["total"], dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(ctx, grad):
        dh, dg = ctx.plan.rdm()
        return grad * dh, grad * dg, None, None, None


def ifci_energy(h, eri, problem, precision=ifci.FP64, **opts):
    return IFCIEnergy.apply(h, eri, problem, precision, opts)
