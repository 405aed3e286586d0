"""torch.autograd.Function around the POD energy (argument marshalling only).

Forward calls pod_energy_forces (one launch of the per-atom kernel plus the
finalize kernel); the adjoint it already evaluates gives the gradients:
dE/dpos = -F (Sec. II.G, eqs. (26c), (24c)) and dE/dc = G (eq. (58a)).
The virial is returned beside the energy as a non-differentiable output.
"""
from __future__ import annotations

import torch

from . import pod


class PodEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, c, model: "pod.PodModel", nbrs: "pod.DeviceNeighbors", cell):
        N = nbrs.N
        dev = model.device
        tdt = model.torch_dtype
        pos_c = pos.detach().to(device=dev, dtype=tdt).contiguous()
        c_c = c.detach().to(device=dev, dtype=tdt).contiguous()
        E = torch.empty(1, dtype=torch.float64, device=dev)
        F = torch.empty((N, 3), dtype=tdt, device=dev)
        W = torch.empty((3, 3), dtype=torch.float64, device=dev)
        G = torch.empty(model.M, dtype=torch.float64, device=dev)
        pod.pod_energy_forces(model.h, N, nbrs.P, pos_c, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, c_c,
                              None, E, F, W, G, rev=nbrs.rev)
        ctx.save_for_backward(F, G)
        ctx.pos_dtype = pos.dtype
        ctx.c_dtype = c.dtype
        ctx.mark_non_differentiable(W)
        return E.to(pos.dtype)[0], W

    @staticmethod
    def backward(ctx, gE, gW):
        F, G = ctx.saved_tensors
        g_pos = g_c = None
        if ctx.needs_input_grad[0]:
            g_pos = (-F.to(ctx.pos_dtype)) * gE
        if ctx.needs_input_grad[1]:
            g_c = G.to(ctx.c_dtype) * gE
        return g_pos, g_c, None, None, None


def pod_energy(pos, c, model, nbrs, cell):
    """Total POD energy (differentiable in pos and c) and the virial."""
    return PodEnergy.apply(pos, c, model, nbrs, cell)
