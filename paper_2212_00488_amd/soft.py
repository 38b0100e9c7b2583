"""torch.autograd front end of the soft-argmin head (include/stereo.h,
stereo_soft_*).  Forward and backward both run in the library's kernels;
these classes only route tensors and the upstream gradient.

    ctx = Stereo(0)
    d_hat = soft_disparity(ctx, left, right, lambdas, dmax)        # [n][Y][X]
    loss = l1_loss(ctx, d_hat, gt, nonocc)                          # [1]
    loss.backward()   # gradients in left.grad, right.grad, lambdas.grad

left, right: float32 [n][H][W][3] in [0, 1] on the device; lambdas: float32
[2] = (lambda_AD, lambda_census) on the device; gt: int16 [n][H][W]; nonocc:
uint8 [n][H][W].
"""

from __future__ import annotations

import torch

from .binding import SOFT_F_REUSE_FEATURES, SOFT_F_SAVE_WEIGHTS, SoftParams, soft_default_params


def _with_flags(params: SoftParams | None, flags: int) -> SoftParams:
    p = soft_default_params() if params is None else SoftParams.from_buffer_copy(params)
    p.flags |= flags
    return p


def _reusing(params: SoftParams | None) -> SoftParams:
    """params (defaults when None) with REUSE_FEATURES set: the backward
    gets the forward's saved inputs, which autograd keeps unchanged, so the
    forward's features, and its softmax weights when it saved them, are
    reused whenever the plan still holds them (the library checks that the
    last forward was for the same tensors)."""
    return _with_flags(params, SOFT_F_REUSE_FEATURES)


class SoftArgmin(torch.autograd.Function):
    @staticmethod
    def forward(fctx, left, right, lambdas, dmax, params, fwd_params, stereo):
        left, right, lambdas = left.contiguous(), right.contiguous(), lambdas.contiguous()
        d_hat, lse2 = stereo.soft_forward(left, right, lambdas, dmax, fwd_params)
        fctx.save_for_backward(left, right, lambdas, d_hat, lse2)
        fctx.dmax, fctx.params, fctx.stereo = dmax, params, stereo
        fctx.mark_non_differentiable(lse2)
        # lse2 takes no gradient: no zero tensor is made for it
        fctx.set_materialize_grads(False)
        return d_hat, lse2

    @staticmethod
    def backward(fctx, g_dhat, _g_lse):
        left, right, lambdas, d_hat, lse2 = fctx.saved_tensors
        if g_dhat is None:  # nothing flows back (possible without materialised grads)
            return None, None, None, None, None, None, None
        g_left, g_right, g_lam = fctx.stereo.soft_backward(
            left, right, lambdas, fctx.dmax, d_hat, lse2, g_dhat.contiguous(),
            _reusing(fctx.params))
        return g_left, g_right, g_lam, None, None, None, None


class L1Loss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, d_hat, gt, nonocc, stereo):
        d_hat = d_hat.contiguous()
        fctx.save_for_backward(d_hat, gt, nonocc)
        fctx.stereo = stereo
        return stereo.l1_loss(d_hat, gt, nonocc)

    @staticmethod
    def backward(fctx, g_loss):
        d_hat, gt, nonocc = fctx.saved_tensors
        g = fctx.stereo.l1_grad(d_hat, gt, nonocc, g_loss.contiguous().to(torch.float32))
        return g, None, None, None


def soft_disparity(stereo, left, right, lambdas, dmax: int, params: SoftParams | None = None):
    """Half-resolution soft-argmin disparity [n][Y][X] (differentiable).  When a
    backward can follow (grad mode on and an input that requires grad), the
    forward keeps its softmax weights for it (SAVE_WEIGHTS)."""
    grad = torch.is_grad_enabled() and any(t.requires_grad for t in (left, right, lambdas))
    fwd_params = _with_flags(params, SOFT_F_SAVE_WEIGHTS) if grad else params
    d_hat, _ = SoftArgmin.apply(left, right, lambdas, dmax, params, fwd_params, stereo)
    return d_hat


def l1_loss(stereo, d_hat, gt, nonocc):
    """Mean over pairs of the mean |2 d_hat - GT(2x,2y)| on non-occluded pixels."""
    return L1Loss.apply(d_hat, gt, nonocc, stereo)
