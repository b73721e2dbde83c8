"""``torch.autograd`` wrapper of the forward map and its exact adjoint.

``WaveOperator(plan)`` owns one workspace; ``op(p0, c)`` returns the sensor
traces f(p0, c) of eq. (2) (HIP forward solve, recorded), and backpropagating a
gradient ``dL/d data`` through it runs the HIP adjoint (eqs. (5)-(9)) with
``resid = dL/d data``, giving ``dL/dp0`` for every dataset and ``dL/dc``.

Only one recorded forward per operator can be pending: a second forward before
the first one's backward overwrites the recorded history, and that backward
then raises (the library reports ``PAT_EWORKSPACE``).
"""
from __future__ import annotations

import torch

from . import pat


class _PATForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0, c, op):
        if p0.dtype != torch.float32 or c.dtype != torch.float32:
            raise ValueError("p0 and c must be float32")
        p0 = p0.contiguous()
        c = c.contiguous()
        data = torch.empty(op.plan.data_shape, dtype=torch.float32, device=p0.device)
        op.plan.forward(c, p0, data, op.ws, ckpt_every=op.ckpt_every, record=True)
        ctx.op = op
        ctx.save_for_backward(p0, c)
        return data

    @staticmethod
    def backward(ctx, grad_data):
        p0, c = ctx.saved_tensors
        op = ctx.op
        g_p0 = torch.empty_like(p0)
        g_c = torch.empty_like(c)
        op.plan.adjoint_gradient(c, p0, grad_data.contiguous().float(), g_p0, g_c, op.ws)
        return g_p0, g_c, None


class WaveOperator(torch.nn.Module):
    """f(p0, c) for the K datasets of ``plan`` (a :class:`pat.Plan`)."""

    def __init__(self, plan: "pat.Plan", ckpt_every: int = 0, device="cuda"):
        super().__init__()
        self.plan = plan
        self.ckpt_every = int(ckpt_every)
        self.ws = plan.workspace(self.ckpt_every, device=device)

    def forward(self, p0: torch.Tensor, c: torch.Tensor) -> torch.Tensor:
        return _PATForward.apply(p0, c, self)
