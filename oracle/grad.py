"""Gradient of a thick-hair render with respect to the per-cluster parameters (oracle).

The LoD fitting adjusts, per cluster, the ellipse semi-axes |a|, |b| of every segment, the
single-hair radius r and the absorption sigma_a so that the coarse render matches the strand
render.  Those are exactly the quantities the aggregated model reads (Sec. 4: rho and the
hair count from n_total, r, |a|, |b|; the lobes from sigma_a) plus the screen half-width the
thick hair is drawn with (Sec. 5.2, hair width calculation).

This module gives the vector-Jacobian product  d/dtheta sum(d_rgba * rgba(theta))  by torch
autograd in float64, with the fragment set held fixed at the one the stored parameters
produce (coverage is piecewise constant in theta; alpha, h and the radiance are smooth
inside a piece).  The half-width is recomputed differentiably from |a|, |b| with the same
formula the float32 coverage radius uses.
"""
from __future__ import annotations

import numpy as np
import torch

from . import raster as rs
from .render import DT, LevelGeom, composite, fragment_radiance, rasterize, split_long


def _midpoint_yhat(geom: LevelGeom, cam):
    """y^ at each segment midpoint (float64), the direction the support width is taken along."""
    A = geom.pA.astype(np.float64)
    B = geom.pB.astype(np.float64)
    t = B - A
    u = t / np.linalg.norm(t, axis=0)
    m = 0.5 * (A + B)
    w = np.asarray(cam.pos, dtype=np.float64)[:, None] - m
    w = w / np.linalg.norm(w, axis=0)
    wp = w - (w * u).sum(0) * u
    nrm = np.linalg.norm(wp, axis=0)
    xh = wp / np.where(nrm > 0, nrm, 1.0)
    yh = np.cross(u.T, xh.T).T
    bh = np.cross(u.T, geom.ahat.astype(np.float64).T).T
    return yh, bh, nrm > 1e-7


def halfwidth_torch(geom: LevelGeom, ras, cam, a_len, b_len):
    """Differentiable hw (pixels) of each thick-hair segment."""
    yh, bh, ok = _midpoint_yhat(geom, cam)
    pa = a_len * torch.as_tensor((geom.ahat.astype(np.float64) * yh).sum(0))
    pb = b_len * torch.as_tensor((bh * yh).sum(0))
    W = torch.sqrt(pa * pa + pb * pb)
    W = torch.where(torch.as_tensor(ok), W, torch.maximum(a_len, b_len))
    c = rs.cam_arrays(cam)
    _, _, zA, _, _ = rs.project_points(geom.pA, c)
    _, _, zB, _, _ = rs.project_points(geom.pB, c)
    zm = 0.5 * (torch.as_tensor(zA.astype(np.float64)) + torch.as_tensor(zB.astype(np.float64)))
    return W * float(c["fy"]) / zm


def cluster_vjp(geom: LevelGeom, cam, lights, mat, d_rgba, K: int, S: int, ras=None):
    """(d_axes [K, S, 2], d_r [K], d_sigma_a [3, K], rgba) for the loss sum(d_rgba * rgba).
    The camera raster draws long segments as pieces (render.split_long); a piece's parameters
    are its segment's.  A given ras must come from split_long(geom, cam)."""
    base = geom
    geom = split_long(geom, cam)
    if ras is None:
        ras = rasterize(geom, cam)
    axes = torch.tensor(np.stack([base.a_len.reshape(K, S), base.b_len.reshape(K, S)], -1),
                        dtype=DT, requires_grad=True)
    r = torch.tensor(base.r.reshape(K, S)[:, 0], dtype=DT, requires_grad=True)
    sig = torch.tensor(base.sigma_a.reshape(K, S, 3)[:, 0, :].T.copy(), dtype=DT, requires_grad=True)
    rows = torch.as_tensor(geom.parent if geom.parent is not None else np.arange(K * S), dtype=torch.int64)
    a_len = axes[..., 0].reshape(-1)[rows]
    b_len = axes[..., 1].reshape(-1)[rows]
    params = dict(a_len=a_len, b_len=b_len,
                  r=r.repeat_interleave(S)[rows], sigma_a=sig.T.repeat_interleave(S, dim=0)[rows],
                  hw=halfwidth_torch(geom, ras, cam, a_len, b_len))
    alpha, L = fragment_radiance(geom, ras, cam, lights, mat, params=params)
    rgba = composite(ras, alpha, L)
    loss = (rgba * torch.as_tensor(np.asarray(d_rgba, dtype=np.float64))).sum()
    g_axes, g_r, g_sig = torch.autograd.grad(loss, (axes, r, sig), allow_unused=True)
    z = lambda g, ref: torch.zeros_like(ref) if g is None else g
    return (z(g_axes, axes).numpy(), z(g_r, r).numpy(), z(g_sig, sig).numpy(), rgba.detach().numpy())


def cluster_render_with(geom: LevelGeom, cam, lights, mat, K, S, axes, r, sigma_a, ras):
    """Render with substituted parameters on a fixed fragment set (for finite differences)."""
    a_len = torch.as_tensor(axes[..., 0].reshape(-1), dtype=DT)
    b_len = torch.as_tensor(axes[..., 1].reshape(-1), dtype=DT)
    params = dict(a_len=a_len, b_len=b_len, r=torch.as_tensor(np.repeat(r, S), dtype=DT),
                  sigma_a=torch.as_tensor(np.repeat(np.asarray(sigma_a).T, S, axis=0), dtype=DT),
                  hw=halfwidth_torch(geom, ras, cam, a_len, b_len))
    alpha, L = fragment_radiance(geom, ras, cam, lights, mat, params=params)
    return composite(ras, alpha, L).numpy()
