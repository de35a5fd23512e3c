"""Differentiable sparse CP model: loss over the stored entries.

    L(A_0, ..., A_{N-1}) = sum_k (x_k - sum_r prod_w A_w[i_w(k), r])^2

(the CP model of Sec. 2.1 evaluated at the nonzeros).  The forward pass is one
kernel (``amped_cp_loss``); the backward pass calls, for every factor that
needs a gradient, the fused residual + MTTKRP kernel (``amped_cp_grad``) with
scale = -2 * grad_output, because dL/dA_d = -2 * MTTKRP_d(E) for the sparse
residual tensor E.  Nothing per nonzero is saved between the passes: the
residuals are recomputed inside the gradient kernel.
"""
import torch

from . import api


class SparseCPLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tensor: "api.Tensor", *factors):
        ctx.tensor = tensor
        ctx.save_for_backward(*factors)
        return api.cp_loss(tensor, [f.detach() for f in factors])

    @staticmethod
    def backward(ctx, grad_out):
        factors = [f.detach() for f in ctx.saved_tensors]
        t = ctx.tensor
        # the loss is float64 on the device; the gradient scale is read once
        scale = -2.0 * float(grad_out)
        grads = [None]
        for d, f in enumerate(factors):
            if ctx.needs_input_grad[d + 1]:
                grads.append(api.cp_grad(t, d, factors, scale))
            else:
                grads.append(None)
        return tuple(grads)


def sparse_cp_loss(tensor: "api.Tensor", *factors):
    return SparseCPLoss.apply(tensor, *factors)
