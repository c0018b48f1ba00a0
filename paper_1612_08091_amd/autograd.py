"""<H> of a parametrised circuit as a differentiable torch function.

The forward runs the library's adjoint routine, which returns the value and
the whole gradient in one call (forward sweep, H psi, reverse sweep); the
backward multiplies the stored gradient by the incoming gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import qsv as Q


class QsvExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, sim, circuit, ham):
        th = theta.detach().to("cpu", torch.float64).numpy()
        value, grad = Q.adjoint_gradient(sim, circuit, ham, th)
        ctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(grad)).to(theta.device,
                                                                             theta.dtype))
        return theta.new_tensor(value)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None, None, None


def expectation(theta: torch.Tensor, sim, circuit, ham) -> torch.Tensor:
    """<0|U(theta)^dag H U(theta)|0> with d/dtheta by adjoint differentiation.
    ``circuit`` is a workloads.Circuit whose rotation gates index ``theta``."""
    return QsvExpectation.apply(theta, sim, circuit, ham)
