"""torch.autograd.Function around the library's forward and hand-written backward.

    C, power = rx_render(renderer, means, log_scales, quats, logits,
                         features_or_radiance, mlp_params, rx, tx=..., mode="tx")

The forward copies the (possibly updated) scene and MLP into the renderer,
renders with a saved state, and keeps it for the backward; the backward calls
rxgs_render_backward with dL/dC and dL/dpower and returns gradients for the
means, log-scales, quaternions, opacity logits, features or direct radiance,
and the flat MLP parameter vector.  Receiver and transmitter positions get no
gradient.
"""
from __future__ import annotations

import torch

from . import rxgs


class RxRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, mode, rx_off, means, log_scales, quats, logits, feat_or_rad, mlp, rx, tx):
        use_mlp = mlp is not None
        if use_mlp:
            renderer.upload_scene(means.detach(), log_scales.detach(), quats.detach(), logits.detach(),
                                  features=feat_or_rad.detach())
            renderer.upload_mlp(mlp.detach())
        else:
            renderer.upload_scene(means.detach(), log_scales.detach(), quats.detach(), logits.detach(),
                                  radiance=feat_or_rad.detach())
        saved = rxgs.Saved(renderer)
        C, P, _ = renderer.render(rx.detach(), tx=None if tx is None else tx.detach(), rx_off=rx_off, mode=mode,
                                  saved=saved)
        ctx.renderer = renderer
        ctx.saved_state = saved
        ctx.use_mlp = use_mlp
        ctx.save_for_backward(C)
        ctx.mark_non_differentiable()
        return C, P

    @staticmethod
    def backward(ctx, gC, gP):
        (C,) = ctx.saved_tensors
        r = ctx.renderer
        if gC is None:
            gC = torch.zeros_like(C)
        g = r.backward(ctx.saved_state, C, gC.contiguous(), None if gP is None else gP.contiguous())
        ctx.saved_state.close()
        fr = g["features"] if ctx.use_mlp else g["radiance"]
        gm = g["mlp"] if ctx.use_mlp else None
        return (None, None, None, g["means"], g["log_scales"], g["quats"], g["logits"], fr, gm, None, None)


def rx_render(renderer, means, log_scales, quats, logits, feat_or_rad, mlp, rx, tx=None, mode="tx", rx_off=None):
    """Differentiable multi-receiver render; returns (C (N,2,H,W), power (N))."""
    return RxRenderFn.apply(renderer, mode, rx_off, means, log_scales, quats, logits, feat_or_rad, mlp, rx, tx)
