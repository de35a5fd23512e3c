"""MI355X (gfx950) sparse MTTKRP after AMPED (arXiv 2507.15121).

``api``      -- binding of the C ABI (include/amped.h): Tensor, mttkrp,
                mttkrp_bf16, cp_loss, cp_grad, cp_loss_grad, gram,
                cp_als_sweep, layout_host.
``autograd`` -- SparseCPLoss / sparse_cp_loss, the differentiable sparse CP
                loss.
``synth``    -- seeded synthetic tensors (input generation only).
``build``    -- in-tree build of the native libraries.
"""
from .api import (AmpedError, Tensor, cp_grad, cp_loss, cp_loss_grad, layout_host, lib, mttkrp,  # noqa: F401
                  mttkrp_bf16, version)


def __getattr__(name):
    if name in ("SparseCPLoss", "SparseCPLossFused", "sparse_cp_loss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
