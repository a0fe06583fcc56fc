"""torch.autograd.Function over the library's transient loss and its reverse-time adjoint.

``SoftplusDropLoss.apply(C, gE, gN, ctx, grid, nsteps, ckpt_every, margin, tol_adj)`` returns the
scalar J = sum_k sum_i softplus(Vdd - v_k,i - margin)^2 of a backward-Euler transient run by the
HIP library from t = 0, with the node capacitances C [nl,ny,nx] and segment conductances
gE [nl,ny,nx-1], gN [nl,ny-1,nx] taken from the tensors; backward() returns dJ/dC, dJ/dgE,
dJ/dgN computed on the GPU by the adjoint (`pg_loss_backward_dev`).  The tensors are float64,
on the context's GPU (the coefficients are then rebuilt on the device from their memory,
`pg_update_mesh_values_dev`) or on the CPU (`pg_update_mesh_values`).
"""
from __future__ import annotations

import torch


class SoftplusDropLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, C, gE, gN, ctx, grid=0, nsteps=200, ckpt_every=20, margin=0.05, tol_adj=1e-9):
        if C.is_cuda and gE.is_cuda and gN.is_cuda:
            ctx.update_mesh_values_dev(grid, gE.detach().double().contiguous(), gN.detach().double().contiguous(),
                                       C.detach().double().contiguous())
        else:
            ctx.update_mesh_values(grid, gE.detach().cpu().double().numpy(), gN.detach().cpu().double().numpy(),
                                   C.detach().cpu().double().numpy())
        ctx.reset()
        J = ctx.loss_forward(grid, 0, nsteps, ckpt_every, margin)
        fctx.pg = ctx
        fctx.tol_adj = tol_adj
        fctx.shapes = (C.shape, gE.shape, gN.shape)
        fctx.devices = (C.device, gE.device, gN.device)
        return torch.tensor(J, dtype=torch.float64, device=C.device)

    @staticmethod
    def backward(fctx, gout):
        dev = torch.device("cuda", torch.cuda.current_device())
        dC = torch.empty(fctx.shapes[0], dtype=torch.float64, device=dev)
        dE = torch.empty(fctx.shapes[1], dtype=torch.float64, device=dev)
        dN = torch.empty(fctx.shapes[2], dtype=torch.float64, device=dev)
        fctx.pg.loss_backward_dev(fctx.tol_adj, dC, dE, dN)
        torch.cuda.current_stream().synchronize()
        g = gout.to(dev)
        return ((g * dC).to(fctx.devices[0]), (g * dE).to(fctx.devices[1]), (g * dN).to(fctx.devices[2]),
                None, None, None, None, None, None)


def softplus_drop_loss(C, gE, gN, ctx, grid=0, nsteps=200, ckpt_every=20, margin=0.05, tol_adj=1e-9):
    return SoftplusDropLoss.apply(C, gE, gN, ctx, grid, nsteps, ckpt_every, margin, tol_adj)
