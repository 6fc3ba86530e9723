"""Differentiation wrapper: the fused objective kernel is the forward of a
torch.autograd.Function and the gradient kernel is its adjoint.

forward  runs gcp_loss_grad for the objective only; the model values are not
         kept (only the input tensors are saved).
backward runs the gradient kernel again, recomputing the model (checkpointing)
         and multiplying by the incoming gradient on the device
         (gcp_loss_grad_scaled); the adjoint of the objective with respect to
         A^(k) and s_t is the MTTKRP of eqs. gcp_grad_A / gcp_grad_lambda.
The slice X_t and the window are held by the stream handle and are not
differentiated.
"""
from __future__ import annotations

import torch

from .stream import Stream


class GcpLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, stream: Stream, X_t: torch.Tensor, A1, A2, A3, s_t):
        A = [A1.detach(), A2.detach(), A3.detach()]
        loss, _, _ = stream.loss_grad(X_t, A, s_t.detach(), want_loss=True, want_grad=False)
        ctx.stream = stream
        ctx.X_t = X_t
        ctx.save_for_backward(A1, A2, A3, s_t)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        A1, A2, A3, s_t = ctx.saved_tensors
        scale = grad_out.detach().reshape(1).to(dtype=A1.dtype).contiguous()
        _, G, g_s = ctx.stream.loss_grad(ctx.X_t, [A1.detach(), A2.detach(), A3.detach()],
                                         s_t.detach(), want_loss=False, want_grad=True,
                                         grad_scale=scale)
        return None, None, G[0], G[1], G[2], g_s


def gcp_loss(stream: Stream, X_t: torch.Tensor, A, s_t: torch.Tensor) -> torch.Tensor:
    """Differentiable objective F(A^(1..3), s_t) over X_t and the stream's window."""
    return GcpLoss.apply(stream, X_t, A[0], A[1], A[2], s_t)
