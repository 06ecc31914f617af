"""torch.autograd binding of the device log-likelihood and its adjoint gradient.

SBVLogLik.apply(theta, sets, two_nu, prec) returns the SBV log-likelihood of
each dataset (a CUDA float64 tensor of n_sets values) and records the gradient
that sbv_loglik_grad_dev computes alongside it (the library's adjoint kernels);
backward scales that saved gradient by the incoming gradient of each set.  All
arithmetic of the value and the gradient happens in libsbv.so; this module
only moves device pointers and the stream handle, and multiplies by
grad_output as the chain rule asks.
"""
import numpy as np
import torch

from . import sbv


class SBVLogLik(torch.autograd.Function):
    """l(theta) per dataset with d/dtheta from the library's adjoint.

    theta: CUDA float64 tensor with the packed log-parameters of every set
    ([log beta_1..d, log sigma^2, log tau^2] per set, sets in order).
    sets: one sbv.Blocks handle or a list of them; two_nu: int or one per set;
    prec: sbv.SBV_FP64 or sbv.SBV_FP32.
    """

    @staticmethod
    def forward(ctx, theta, sets, two_nu, prec=sbv.SBV_FP64):
        if not (theta.is_cuda and theta.dtype == torch.float64):
            raise TypeError("theta must be a CUDA float64 tensor")
        hs = [sets] if isinstance(sets, sbv.Blocks) else list(sets)
        th = theta.detach().contiguous()
        out = torch.empty(len(hs), dtype=torch.float64, device=theta.device)
        grad = torch.empty_like(th)
        sbv.sbv_loglik_grad_dev(hs, th, two_nu, out, grad, prec=prec, stream=torch.cuda.current_stream())
        # per-parameter index of the set it belongs to, for the backward scaling
        owner = np.repeat(np.arange(len(hs)), [h.d + 2 for h in hs])
        ctx.save_for_backward(grad, torch.as_tensor(owner, device=theta.device))
        return out

    @staticmethod
    def backward(ctx, grad_out):
        grad, owner = ctx.saved_tensors
        return grad_out[owner] * grad, None, None, None


def loglik(theta, sets, two_nu, prec=sbv.SBV_FP64):
    """Differentiable SBV log-likelihood (see SBVLogLik)."""
    return SBVLogLik.apply(theta, sets, two_nu, prec)
