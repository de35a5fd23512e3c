"""Differentiable sparse CP model: loss over the stored entries.

    L(A_0, ..., A_{N-1}) = sum_k (x_k - sum_r prod_w A_w[i_w(k), r])^2

(the CP model of Sec. 2.1 evaluated at the nonzeros).  dL/dA_d =
-2 * MTTKRP_d(E) for the sparse residual tensor E, computed by the fused
residual + MTTKRP kernel, which recomputes every residual from the factor
rows: nothing per nonzero is kept between the passes.

``SparseCPLoss`` evaluates the loss alone in its forward pass
(``amped_cp_loss``) and every needed gradient in backward (``amped_cp_grad``
with scale = -2 * grad_output).  ``sparse_cp_loss`` picks, when autograd will
need gradients, ``SparseCPLossFused``: its forward pass runs
``amped_cp_loss_grad``, which yields the loss and the first needed mode's
gradient (unscaled by grad_output) in one pass, and keeps that gradient until
backward (one factor-sized buffer), so a loss + all-gradients step reads the
tensor N times instead of N + 1.
"""
import torch

from . import api


class SparseCPLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tensor: "api.Tensor", *factors):
        ctx.tensor = tensor
        ctx.early = None
        ctx.save_for_backward(*factors)
        return api.cp_loss(tensor, [f.detach() for f in factors])

    @staticmethod
    def backward(ctx, grad_out):
        factors = [f.detach() for f in ctx.saved_tensors]
        t = ctx.tensor
        early = ctx.early
        ctx.early = None
        scale = None
        grads = [None]
        for d in range(len(factors)):
            if not ctx.needs_input_grad[d + 1]:
                grads.append(None)
            elif early is not None and early[0] == d:
                # -2 * MTTKRP_d(E) from the forward pass, times dL_out on the device
                grads.append(early[1].mul_(grad_out))
            else:
                if scale is None:
                    # the loss is float64 on the device; the gradient scale is read once
                    scale = -2.0 * float(grad_out)
                grads.append(api.cp_grad(t, d, factors, scale))
        return tuple(grads)


class SparseCPLossFused(SparseCPLoss):
    @staticmethod
    def forward(ctx, tensor: "api.Tensor", *factors):
        ctx.tensor = tensor
        ctx.save_for_backward(*factors)
        need = [d for d in range(len(factors)) if ctx.needs_input_grad[d + 1]]
        if not need:
            ctx.early = None
            return api.cp_loss(tensor, [f.detach() for f in factors])
        loss, grad = api.cp_loss_grad(tensor, need[0], [f.detach() for f in factors], -2.0)
        ctx.early = (need[0], grad)
        return loss


def sparse_cp_loss(tensor: "api.Tensor", *factors):
    """The sparse CP loss as a differentiable 0-dim float64 tensor; when a
    gradient will be taken, its forward pass also computes one mode's
    gradient (SparseCPLossFused)."""
    if torch.is_grad_enabled() and any(f.requires_grad for f in factors):
        return SparseCPLossFused.apply(tensor, *factors)
    return SparseCPLoss.apply(tensor, *factors)
