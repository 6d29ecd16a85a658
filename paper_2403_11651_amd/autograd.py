"""torch.autograd.Function around the HIP rate-distortion pass.

CoolChicFn.apply(problem, img, u, y, arm_w, ups_w, syn_w) returns the loss of
Eq. (1), D + lambda R / (H W), as a 0-d device tensor.  Its forward is one
coolchic_forward call and its backward one coolchic_backward call, which
recomputes the forward pass on the device (nothing but the inputs is kept
between the two) and returns the gradients with respect to the latents and
every parameter block (Section IV-A: the backward pass takes the gradient of
the loss with respect to the layer weights and the layer inputs).  The
quantiser is the problem's: rounding with the straight-through gradient, or
the additive noise u (both have the identity as the gradient of y_hat with
respect to y).  torch only allocates the tensors; all arithmetic runs in the
library's kernels.  The image and the noise get no gradient.

The backward reads the incoming gradient of the loss (a scalar) on the host
to pass it as the pass's dloss argument, which synchronises the stream once
per backward call; training loops that need no autograd graph call
coolchic_train_step instead.
"""
from __future__ import annotations

import torch

from . import binding as B


def _f32(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 GPU tensor")
    return t.contiguous()


class CoolChicFn(torch.autograd.Function):
    """Loss of Eq. (1) with the hand-written adjoint as its backward."""

    @staticmethod
    def forward(ctx, problem, img, u, y, arm_w, ups_w, syn_w):
        img, y, arm_w, ups_w, syn_w = (_f32(t, n) for t, n in
                                       ((img, "img"), (y, "y"), (arm_w, "arm_w"), (ups_w, "ups_w"),
                                        (syn_w, "syn_w")))
        if problem.quant == B.CC_QUANT_NOISE:
            u = _f32(u, "u")
        else:
            u = None
        loss4 = torch.empty(4, dtype=y.dtype, device=y.device)
        B.coolchic_forward(problem, img, y, u, arm_w, ups_w, syn_w, loss4)
        ctx.problem = problem
        ctx.save_for_backward(img, y, arm_w, ups_w, syn_w, *(() if u is None else (u,)))
        ctx.loss4 = loss4
        return loss4[0].clone()

    @staticmethod
    def backward(ctx, g_loss):
        img, y, arm_w, ups_w, syn_w, *rest = ctx.saved_tensors
        u = rest[0] if rest else None
        p = ctx.problem
        dloss = float(g_loss)
        loss4 = torch.empty(4, dtype=y.dtype, device=y.device)
        g_y, g_arm, g_ups, g_syn = (torch.empty_like(t) for t in (y, arm_w, ups_w, syn_w))
        B.coolchic_backward(p, img, y, u, arm_w, ups_w, syn_w, dloss, loss4, g_y, g_arm, g_ups, g_syn)
        return None, None, None, g_y, g_arm, g_ups, g_syn


def coolchic_loss(problem, img, y, arm_w, ups_w, syn_w, u=None):
    """The loss of Eq. (1) as a differentiable 0-d tensor (see CoolChicFn)."""
    return CoolChicFn.apply(problem, img, u, y, arm_w, ups_w, syn_w)
