"""LoD fitting: adjust a thick-hair level so its render matches the strand render.

Parameters live in log space (|a|, |b| per cluster segment, r and sigma_a per cluster) so they
stay positive; Adam on the mean squared RGB difference over a set of views.  The gradient is
the library's adjoint (autograd.HairLoDRender).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from . import binding as B
from .autograd import render_lod


@dataclass
class FitResult:
    loss_history: list = field(default_factory=list)
    seconds: float = 0.0
    axes: torch.Tensor = None
    r: torch.Tensor = None
    sigma_a: torch.Tensor = None


def strand_targets(hctx: B.Context, asset: int, cams, lights, ws=None):
    """Strand-level renders (level 0) of every view, the fitting targets."""
    return [hctx.render(asset, 0, cam, lights, ws=ws)[0].clone() for cam in cams]


def lod_loss(hctx, asset, level, cams, lights, targets, axes, r, sigma_a, ws=None):
    """Mean over views, pixels and RGB of (C_lod - C_strand)^2."""
    total = 0.0
    for cam, tgt in zip(cams, targets):
        img = render_lod(axes, r, sigma_a, hctx, asset, level, cam, lights, ws)
        total = total + ((img[..., :3] - tgt[..., :3]) ** 2).mean()
    return total / len(cams)


def fit_level(hctx: B.Context, asset: int, level: int, cams, lights, iters: int = 200, lr: float = 1e-2,
              ws=None, targets=None, log_every: int = 0) -> FitResult:
    dev = torch.device(f"cuda:{hctx.device}")
    lod = hctx.get_lod(asset, level)
    la = torch.tensor(lod.axes, device=dev).log().requires_grad_(True)
    lr_ = torch.tensor(lod.r, device=dev).log().requires_grad_(True)
    ls = torch.tensor(lod.sigma_a, device=dev).clamp_min(1e-6).log().requires_grad_(True)
    if targets is None:
        targets = strand_targets(hctx, asset, cams, lights, ws)
    opt = torch.optim.Adam([la, lr_, ls], lr=lr)
    res = FitResult()
    t0 = time.perf_counter()
    for it in range(iters + 1):
        opt.zero_grad()
        loss = lod_loss(hctx, asset, level, cams, lights, targets, la.exp(), lr_.exp(), ls.exp(), ws)
        res.loss_history.append(float(loss))
        if log_every and it % log_every == 0:
            print(f"fit iter {it}: loss {float(loss):.6e}", flush=True)
        if it == iters:
            break
        loss.backward()
        opt.step()
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    res.axes, res.r, res.sigma_a = la.detach().exp(), lr_.detach().exp(), ls.detach().exp()
    hctx.set_cluster_params(asset, level, res.axes.contiguous(), res.r.contiguous(), res.sigma_a.contiguous())
    return res
