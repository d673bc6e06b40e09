"""torch.autograd.Function over hair_render / hair_render_backward.

The differentiable inputs are a thick-hair level's fitted parameters (Sec. 4 quantities):
per cluster segment the ellipse semi-axes (|a|, |b|), per cluster the hair radius r and the
absorption sigma_a.  Forward uploads them (device-to-device) and renders; backward runs the
library's hand-written adjoint, which recomputes the fragment lists instead of storing them.
"""
from __future__ import annotations

import torch

from . import binding as B


class HairLoDRender(torch.autograd.Function):
    @staticmethod
    def forward(fctx, axes, r, sigma_a, hctx: B.Context, asset: int, level: int, cam, lights, ws):
        axes_c, r_c, sig_c = axes.detach().contiguous(), r.detach().contiguous(), sigma_a.detach().contiguous()
        hctx.set_cluster_params(asset, level, axes_c, r_c, sig_c)
        img, _, _ = hctx.render(asset, level, cam, lights, ws=ws)
        fctx.save_for_backward(axes_c, r_c, sig_c)
        fctx.args = (hctx, asset, level, cam, lights, ws)
        return img

    @staticmethod
    def backward(fctx, d_img):
        axes_c, r_c, sig_c = fctx.saved_tensors
        hctx, asset, level, cam, lights, ws = fctx.args
        hctx.set_cluster_params(asset, level, axes_c, r_c, sig_c)
        d_axes = torch.empty_like(axes_c)
        d_r = torch.empty_like(r_c)
        d_sig = torch.empty_like(sig_c)
        hctx.render_backward(asset, level, cam, lights, d_img.contiguous(), d_axes, d_r, d_sig, ws=ws)
        return d_axes, d_r, d_sig, None, None, None, None, None, None


def render_lod(axes, r, sigma_a, hctx, asset, level, cam, lights, ws=None):
    """Differentiable render of a thick-hair level: float32 [H, W, 4] on the device."""
    return HairLoDRender.apply(axes, r, sigma_a, hctx, asset, level, cam, lights, ws)
