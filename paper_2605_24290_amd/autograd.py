"""torch.autograd.Function around the library's forward and hand-written backward.

    C, power = rx_render(renderer, means, log_scales, quats, logits,
                         features_or_radiance, mlp_params, rx, tx=..., mode="tx")

The forward copies the scene and MLP into the renderer when they differ from
what it holds (another tensor, or the same tensor modified in place since),
renders with a saved state, and keeps it for the backward; the backward calls
rxgs_render_backward with dL/dC and dL/dpower and returns gradients for the
means, log-scales, quaternions, opacity logits, features or direct radiance,
and the flat MLP parameter vector.  Receiver and transmitter positions get no
gradient.  Several renders of one unchanged scene may share a graph (a loss
summed over transmitters): each keeps its own saved state.  Changing the scene
between such renders invalidates the earlier ones' saved states, and their
backward then raises RxgsError (E_STATE).
"""
from __future__ import annotations

import torch

from . import rxgs


def _stamp(tensors):
    """Identity of the tensors' contents: storage, shape and in-place version."""
    return tuple(None if t is None else (t.data_ptr(), tuple(t.shape), t.dtype, t.device, t._version)
                 for t in tensors)


class RxRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, mode, rx_off, means, log_scales, quats, logits, feat_or_rad, mlp, rx, tx):
        use_mlp = mlp is not None
        scene = (means, log_scales, quats, logits, feat_or_rad, use_mlp)
        stamp = _stamp(scene[:5]) + (use_mlp,)
        if getattr(renderer, "_autograd_scene", None) != stamp:
            if use_mlp:
                renderer.upload_scene(means.detach(), log_scales.detach(), quats.detach(), logits.detach(),
                                      features=feat_or_rad.detach())
            else:
                renderer.upload_scene(means.detach(), log_scales.detach(), quats.detach(), logits.detach(),
                                      radiance=feat_or_rad.detach())
            renderer._autograd_scene = stamp
            renderer._autograd_mlp = None
            # (held so that their storage cannot be reused under an equal stamp)
            renderer._autograd_keep = scene[:5]
        if use_mlp:
            mstamp = _stamp((mlp,))
            if getattr(renderer, "_autograd_mlp", None) != mstamp:
                renderer.upload_mlp(mlp.detach())
                renderer._autograd_mlp = mstamp
                renderer._autograd_keep_mlp = mlp
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
