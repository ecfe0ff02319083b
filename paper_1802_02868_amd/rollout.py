"""Differentiable FP64 rollouts: torch.autograd.Function over the library.

Forward: Step 1 from phi0, then `nsteps` steps on the fused kernel, keeping
the populations every `every` steps as checkpoints.  Backward: the library's
adjoint walks the checkpoints in reverse (each segment recomputed from its
checkpoint) and through Step 1, giving dJ/d(phi0), dJ/d(kappa) (at fixed
beta) and dJ/d(gx, gy) for any scalar J of the final populations.
Argument marshalling only: all arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

import torch

from . import dugks2p as D


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, kappa, g, case, nsteps, every):
        params = dict(case.params)
        params["kappa"] = float(kappa)
        params["gx"], params["gy"] = (float(v) for v in g.detach().cpu())
        params.pop("precision", None)
        params.pop("kernel", None)
        dev = phi0.device
        u0 = [torch.as_tensor(a, dtype=torch.float64, device=dev) for a in (case.ux0, case.uy0, case.p0)]
        sim = D.Simulation(params, case.x_faces, case.y_faces, phi0.detach(), *u0,
                           precision=D.FP64, kernel=D.KERNEL_AUTO)
        ckpts = []
        done = 0
        while done < nsteps:
            ckpts.append(sim.populations())
            n = min(every, nsteps - done)
            sim.step(n)
            done += n
        out = sim.populations()
        sim.close()
        ctx.params, ctx.case, ctx.nsteps, ctx.every = params, case, int(nsteps), int(every)
        ctx.ckpts = ckpts
        ctx.save_for_backward(phi0.detach(), *u0)
        return out

    @staticmethod
    def backward(ctx, grad_pops):
        phi0, ux0, uy0, p0 = ctx.saved_tensors
        case = ctx.case
        adj = D.Adjoint(ctx.params, case.x_faces, case.y_faces, max_segment=max(ctx.every, 1))
        pg = torch.zeros(3, dtype=torch.float64, device=phi0.device)
        lam = grad_pops.detach().to(torch.float64).contiguous()
        for k in range(len(ctx.ckpts) - 1, -1, -1):
            n = min(ctx.every, ctx.nsteps - k * ctx.every)
            lam = adj.segment(ctx.ckpts[k], n, lam, pg)
        phi0_grad = adj.initial(phi0, ux0, uy0, p0, lam, pg)
        adj.close()
        ctx.ckpts = None
        return phi0_grad, pg[0].clone(), pg[1:3].clone(), None, None, None


def rollout(phi0, kappa, g, case, nsteps, every=50):
    """Final populations [18, ny, nx] after Step 1 and `nsteps` steps.

    phi0: float64 CUDA [ny, nx]; kappa: float64 0-d tensor; g: float64
    tensor [2] = (gx, gy); the other parameters, the mesh and u0, p0 come
    from `case` (workloads.Case)."""
    return Rollout.apply(phi0, kappa, g, case, int(nsteps), int(every))
