"""LoD fitting: adjust a thick-hair level so its render matches the strand render.

Parameters live in log space (|a|, |b| per cluster segment, r and sigma_a per cluster) so they
stay positive; Adam on the mean squared RGB difference over a set of views.  The gradient is
the library's adjoint (autograd.HairLoDRender).

A fit can be checkpointed and resumed: a checkpoint holds the log parameters, Adam's state
(moments and step counts), the number of steps taken, the loss history and the level it
belongs to, as plain tensors and numbers (torch.save; read back with weights_only=True).
Resuming continues the step sequence where it stopped.
"""
from __future__ import annotations

import os
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


CHECKPOINT_VERSION = 1
PARAM_NAMES = ("log_axes", "log_r", "log_sigma_a")


def save_checkpoint(path: str, level: int, params, opt: torch.optim.Optimizer, steps: int, loss_history,
                    lr: float) -> None:
    """Write a fit's state (params: the log-parameter tensors in PARAM_NAMES order; steps: the
    optimizer steps taken) to path, atomically (a temporary file renamed over it)."""
    state = {
        "version": CHECKPOINT_VERSION,
        "level": int(level),
        "steps": int(steps),
        "lr": float(lr),
        "loss_history": torch.tensor(list(loss_history), dtype=torch.float64),
        "params": {k: p.detach().cpu().clone() for k, p in zip(PARAM_NAMES, params)},
        "adam": opt.state_dict(),
    }
    tmp = f"{path}.tmp{os.getpid()}"
    torch.save(state, tmp)
    os.replace(tmp, path)


def load_checkpoint(path: str) -> dict:
    """A checkpoint written by save_checkpoint (loaded with weights_only=True)."""
    state = torch.load(path, map_location="cpu", weights_only=True)
    if state.get("version") != CHECKPOINT_VERSION:
        raise ValueError(f"{path}: checkpoint version {state.get('version')} (expected {CHECKPOINT_VERSION})")
    missing = [k for k in PARAM_NAMES if k not in state["params"]]
    if missing:
        raise ValueError(f"{path}: checkpoint lacks {missing}")
    return state


def restore(state: dict, params, opt: torch.optim.Optimizer):
    """Copy a checkpoint's parameters into params (same shapes) and its Adam state into opt;
    returns (steps taken, loss history)."""
    with torch.no_grad():
        for k, p in zip(PARAM_NAMES, params):
            src = state["params"][k]
            if tuple(src.shape) != tuple(p.shape):
                raise ValueError(f"checkpoint {k} has shape {tuple(src.shape)}, the level {tuple(p.shape)}")
            p.copy_(src.to(p.device))
    opt.load_state_dict(state["adam"])
    return int(state["steps"]), [float(v) for v in state["loss_history"]]


def fit_level(hctx: B.Context, asset: int, level: int, cams, lights, iters: int = 200, lr: float = 1e-2,
              ws=None, targets=None, log_every: int = 0, checkpoint: str | None = None, save_every: int = 0,
              resume: str | None = None) -> FitResult:
    """Adam for `iters` steps in total.  checkpoint + save_every: write a checkpoint every
    save_every steps (and after the last); resume: continue from a checkpoint of this level
    (its steps count toward iters)."""
    dev = torch.device(f"cuda:{hctx.device}")
    lod = hctx.get_lod(asset, level)
    la = torch.tensor(lod.axes, device=dev).log().requires_grad_(True)
    lr_ = torch.tensor(lod.r, device=dev).log().requires_grad_(True)
    ls = torch.tensor(lod.sigma_a, device=dev).clamp_min(1e-6).log().requires_grad_(True)
    if targets is None:
        targets = strand_targets(hctx, asset, cams, lights, ws)
    opt = torch.optim.Adam([la, lr_, ls], lr=lr)
    res = FitResult()
    start = 0
    if resume is not None:
        state = load_checkpoint(resume)
        if state["level"] != level:
            raise ValueError(f"{resume}: a checkpoint of level {state['level']}, not {level}")
        start, res.loss_history = restore(state, (la, lr_, ls), opt)
    t0 = time.perf_counter()
    for it in range(start, iters + 1):
        opt.zero_grad()
        loss = lod_loss(hctx, asset, level, cams, lights, targets, la.exp(), lr_.exp(), ls.exp(), ws)
        res.loss_history.append(float(loss.detach()))
        if log_every and it % log_every == 0:
            print(f"fit iter {it}: loss {float(loss):.6e}", flush=True)
        if it == iters:
            break
        loss.backward()
        opt.step()
        if checkpoint and save_every and ((it + 1) % save_every == 0 or it + 1 == iters):
            save_checkpoint(checkpoint, level, (la, lr_, ls), opt, it + 1, res.loss_history, lr)
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    res.axes, res.r, res.sigma_a = la.detach().exp(), lr_.detach().exp(), ls.detach().exp()
    hctx.set_cluster_params(asset, level, res.axes.contiguous(), res.r.contiguous(), res.sigma_a.contiguous())
    return res
