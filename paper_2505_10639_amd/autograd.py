"""torch.autograd.Function over momfbd_loss_grad.

Forward returns the summed patch loss sum_p L_p (float64 scalar); backward
returns grad_out * dL/dalpha computed by the library's adjoint kernels in
the same call as the loss.
"""

from __future__ import annotations

import torch


class MomfbdLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, plan, D, gamma=1e-3, weights=None):
        loss, grad = plan.loss_grad(alpha.detach().contiguous(), D, gamma, weights,
                                    want_grad=alpha.requires_grad)
        ctx.save_for_backward(grad if grad is not None else torch.empty(0))
        return loss.sum()

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return (grad_out.to(grad.dtype) * grad, None, None, None, None)


def momfbd_loss(alpha, plan, D, gamma=1e-3, weights=None):
    return MomfbdLoss.apply(alpha, plan, D, gamma, weights)
