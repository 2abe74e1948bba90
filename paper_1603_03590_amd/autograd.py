"""``torch.autograd.Function`` over the C entry points: the forward calls
dis_compute_flow, the backward dis_flow_backward (the hand-written adjoint of
Alg. 1 with per-scale recomputation).  Marshalling only."""
from __future__ import annotations

import torch


class DISFlow(torch.autograd.Function):
    """flow = DIS(I0, I1); backward gives dL/dI0 and dL/dI1."""

    @staticmethod
    def forward(ctx, I0, I1, dis):
        flow = dis.flow(I0, I1)
        ctx.dis = dis
        ctx.generation = dis._generation
        ctx.shape = tuple(I0.shape)
        return flow

    @staticmethod
    def backward(ctx, grad_flow):
        dis = ctx.dis
        if getattr(dis, "_generation", None) != ctx.generation:
            raise RuntimeError("DIS backward needs the handle's most recent forward; run backward before the next "
                               "forward on the same handle, or use one handle per pending result")
        g0, g1 = dis.backward(grad_flow.to(dis.dtype), ctx.shape)
        return g0, g1, None
