"""Shadow pass: deep opacity map (DOM) of the hair toward each directional light (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper renders the hair into a deep opacity map in its shadow pass (Sec. 5.2, runtime
pipeline) and defers the use of it to dual scattering: the number n of hairs a light path
crosses before it reaches a shading point scales the forward-scattered light by a_F^n and
widens it by n sigma_f^2 (Sec. 3.2).  Readings taken here (the paper prints no DOM details):

  * Light frame.  omega = the unit direction toward the light; e1 = normalize((0, 1, 0) x
    omega) (or (1, 0, 0) x omega when |omega_y| >= 0.9), e2 = omega x e1, depth axis
    d = -omega (increasing away from the light).  Computed in float64, stored as float32.
  * Grid.  R x R square texels over the hair: u = p . e1, v = p . e2, z = p . d per segment
    endpoint (float32, rows summed left to right), widened by the segment's half-width
    (strands w / 2, thick hairs max(|a|, |b|)); extent = max(u range, v range) (at least
    1e-6), texel size s = extent / (R - 2), origin one texel below the minima; z_ref =
    z_max + 1 so that iz = z_ref - z >= 1 orders fragments like an inverse depth.
  * Light-view records: the camera raster's integer predicate on texels.  X = rint((u - u0)
    (16 / s)), Y likewise, iz = z_ref - z; half-width in texels (w / 2) / s for strands and,
    for thick hairs, the ellipse's support half-width across the light direction divided by
    s.  Every fragment (texel, segment) comes from the same coverage rule as the camera pass.
  * Texel content: iz0 = the largest iz of its fragments (the first hair the light meets);
    K layers of depth Delta from there: fragment layer k = min(K - 1, floor((iz0 - iz) /
    Delta)).  A fragment adds its expected hair count: a strand its box coverage alpha, a
    thick hair alpha rho kappa l with l = l_max sqrt(1 - h^2) the chord along the light at
    the texel's offset h = min(delta / hw, 1) and l_max = 2 |a||b| / W (Sec. 4, hair number).
    C_k = cumulative count through layer k.
  * Lookup at a world point x (float32: the fragment's point on the centre line from the
    integer raster parameter t, without fused operations): x = (iz0 - iz(x)) / Delta - 1
    layers behind the first hit (one layer of bias so that a hair never shadows itself; the
    hairs inside a thick hair toward the light are its own n_F), n = 0 for x < 0, C_{K-1}
    for x >= K, else C_{j-1} + (x - j)(C_j - C_{j-1}) with j = floor(x); bilinear between
    the four nearest texel centres, texels outside the grid or without hair count 0.
  * Shading (Sec. 4 with the path's n): n_s hairs in front of the fragment add to the
    forward count: a strand is shaded by f_ours with n_total = 1 and n_F = 1 + n_s, a thick
    hair by f_ours with n_F + n_s.  Only directional lights have a DOM; point lights are
    unshadowed.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import raster as rs
from .render import DT, LevelGeom, fragment_alpha_h

F32 = np.float32


def light_basis(omega):
    """(e1, e2, d, omega) as float32 arrays from the toward-light vector (float64 math)."""
    w = np.asarray(omega, dtype=np.float64)
    w = w / math.sqrt(float(w @ w))
    a = np.array([0.0, 1.0, 0.0]) if abs(w[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(a, w)
    e1 = e1 / math.sqrt(float(e1 @ e1))
    e2 = np.cross(w, e1)
    return e1.astype(F32), e2.astype(F32), (-w).astype(F32), w.astype(F32)


def _proj(p, e):
    """p . e in float32, summed left to right.  p: [3, N] float32."""
    return (p[0] * e[0] + p[1] * e[1]) + p[2] * e[2]


def _thick(geom: LevelGeom):
    n = geom.pA.shape[1]
    if geom.kind == "strand":
        return np.zeros(n, dtype=bool)
    if geom.kind == "cluster":
        return np.ones(n, dtype=bool)
    return np.asarray(geom.thick, dtype=bool)


def segment_halfwidth_world(geom: LevelGeom):
    """Per-segment world half-width used to pad the grid."""
    t = _thick(geom)
    hw = np.zeros(geom.pA.shape[1], dtype=F32)
    if (~t).any():
        hw[~t] = F32(0.5) * geom.width[~t]
    if t.any():
        hw[t] = np.maximum(geom.a_len[t], geom.b_len[t])
    return hw


def dom_grid(geom: LevelGeom, omega, R: int):
    """Grid of the level toward the light: dict of float32 parameters."""
    e1, e2, d, w = light_basis(omega)
    hw = segment_halfwidth_world(geom)
    uA, uB = _proj(geom.pA, e1), _proj(geom.pB, e1)
    vA, vB = _proj(geom.pA, e2), _proj(geom.pB, e2)
    zA, zB = _proj(geom.pA, d), _proj(geom.pB, d)
    umin = min(np.min(uA - hw), np.min(uB - hw))
    umax = max(np.max(uA + hw), np.max(uB + hw))
    vmin = min(np.min(vA - hw), np.min(vB - hw))
    vmax = max(np.max(vA + hw), np.max(vB + hw))
    zmax = max(np.max(zA), np.max(zB))
    ext = max(F32(umax - umin), F32(vmax - vmin), F32(1e-6))
    s = F32(ext / F32(R - 2))
    return dict(e1=e1, e2=e2, d=d, omega=w, u0=F32(umin - s), v0=F32(vmin - s), s=s,
                k16=F32(F32(16.0) / s), z_ref=F32(zmax + F32(1.0)), R=int(R))


def light_records(geom: LevelGeom, g):
    """(XA, YA, XB, YB, izA, izB, hw, hw_fx, vis) of the light view (float32 decisions)."""
    uA, uB = _proj(geom.pA, g["e1"]), _proj(geom.pB, g["e1"])
    vA, vB = _proj(geom.pA, g["e2"]), _proj(geom.pB, g["e2"])
    zA, zB = _proj(geom.pA, g["d"]), _proj(geom.pB, g["d"])
    XA = np.rint((uA - g["u0"]) * g["k16"]).astype(np.int64)
    YA = np.rint((vA - g["v0"]) * g["k16"]).astype(np.int64)
    XB = np.rint((uB - g["u0"]) * g["k16"]).astype(np.int64)
    YB = np.rint((vB - g["v0"]) * g["k16"]).astype(np.int64)
    izA = (g["z_ref"] - zA).astype(F32)
    izB = (g["z_ref"] - zB).astype(F32)
    t = _thick(geom)
    hw = np.zeros(XA.shape, dtype=F32)
    if (~t).any():
        hw[~t] = (F32(0.5) * geom.width[~t]) / g["s"]
    if t.any():
        hw[t] = support_width(geom, g["omega"], t) / g["s"]
    ok = np.ones(XA.shape, dtype=bool)
    hw_fx, vis = rs.finalize_segments(XA, YA, XB, YB, ok, ok, hw)
    return XA, YA, XB, YB, izA, izB, hw, hw_fx, vis


def support_width(geom: LevelGeom, omega, rows):
    """Ellipse support half-width W across the light direction (float32, the same operation
    order as the camera's: x^ = normalize(w - (w.u) u) with w = omega, y^ = u x x^)."""
    pA, pB = geom.pA[:, rows], geom.pB[:, rows]
    a_len, b_len, ah = geom.a_len[rows], geom.b_len[rows], geom.ahat[:, rows]
    t = [pB[i] - pA[i] for i in range(3)]
    tl = rs._norm3(*t)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = [t[i] / tl for i in range(3)]
        w = [np.full_like(tl, omega[i]) for i in range(3)]
        dwu = rs._dot(w, u)
        wp = [w[i] - dwu * u[i] for i in range(3)]
        wpl = rs._norm3(*wp)
        xh = [wp[i] / wpl for i in range(3)]
        yh = rs._cross(u, xh)
        bh = rs._cross(u, ah)
        pa = a_len * rs._dot(ah, yh)
        pb = b_len * rs._dot(bh, yh)
        W = np.sqrt(pa * pa + pb * pb)
        return np.where(wpl > F32(1e-7), W, np.maximum(a_len, b_len)).astype(F32)


class Dom:
    """iz0 [R*R] float32 (0 = no hair), C [R*R, K] float64 cumulative counts."""

    def __init__(self, grid, K, delta, iz0, C):
        self.grid, self.K, self.delta, self.iz0, self.C = grid, K, F32(delta), iz0, C


def build_dom(geom: LevelGeom, omega, R: int, K: int, delta: float) -> Dom:
    g = dom_grid(geom, omega, R)
    XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = light_records(geom, g)
    seg, pi, pj = rs.candidate_pixels(XA, YA, XB, YB, hw_fx, vis, R, R)
    ok, t_num, t_den, cross = rs.coverage(XA, YA, XB, YB, hw_fx, seg, pi, pj)
    seg, pi, pj, t_num, t_den, cross = seg[ok], pi[ok], pj[ok], t_num[ok], t_den[ok], cross[ok]
    key, _, _ = rs.depth_key(t_num, t_den, izA[seg], izB[seg])
    iz = (np.uint32(0xFFFFFFFF) - key.astype(np.uint32)).view(F32)
    pix = pj * R + pi
    iz0 = np.zeros(R * R, dtype=F32)
    np.maximum.at(iz0, pix, iz)
    layer = np.minimum(K - 1, np.floor((iz0[pix] - iz) / F32(delta)).astype(np.int64))
    # expected hair count of each fragment (float64)
    ras = type("Ras", (), {})()
    ras.cross, ras.t_den, ras.seg = cross, t_den, seg
    ras.sign = np.ones(len(XA))
    hw_t = torch.as_tensor(hw[seg].astype(np.float64), dtype=DT)
    alpha, _ = fragment_alpha_h(ras, hw_t)
    cnt = alpha.numpy()
    th = _thick(geom)[seg]
    if th.any():
        sg = seg[th]
        delta_px = np.abs(cross[th].astype(np.float64)) / np.sqrt(t_den[th].astype(np.float64)) / 16.0
        h = np.minimum(delta_px / hw[sg].astype(np.float64), 1.0)
        a = geom.a_len[sg].astype(np.float64)
        b = geom.b_len[sg].astype(np.float64)
        n_total = geom.n_total[sg].astype(np.float64)
        r = geom.r[sg].astype(np.float64)
        W = hw[sg].astype(np.float64) * float(g["s"])
        rho = np.clip(n_total * r * r / (a * b), 0.0, 1.0)
        kappa = np.sqrt(n_total / (math.pi * a * b))
        with np.errstate(divide="ignore", invalid="ignore"):
            c = cnt[th] * rho * kappa * (2.0 * a * b / W) * np.sqrt(1.0 - h * h)
        cnt[th] = np.where(W > 0, c, 0.0)     # a zero-width thick hair holds no hairs across the light
    S = np.zeros((R * R, K))
    np.add.at(S, (pix, layer), cnt)
    return Dom(g, K, delta, iz0, np.cumsum(S, axis=1))


def lookup_point(geom: LevelGeom, ras, cam):
    """Float32 world point of every camera fragment on its centre line, as the kernel forms it
    for the DOM lookup: t = float(t_num) / float(t_den), iz = izA + t (izB - izA),
    t_w = (t izB) / iz, x = pA + t_w (pB - pA); every operation rounded once."""
    s = ras.seg
    t = ras.t_num.astype(F32) / ras.t_den.astype(F32)
    izA, izB = ras.izA[s], ras.izB[s]
    iz = izA + t * (izB - izA)
    tw = (t * izB) / iz
    pA, pB = geom.pA[:, s], geom.pB[:, s]
    return np.stack([pA[i] + tw * (pB[i] - pA[i]) for i in range(3)])


def dom_count(dom: Dom, x):
    """n_s (float64 [N]) at float32 world points x [3, N]."""
    g, K, R = dom.grid, dom.K, dom.grid["R"]
    u, v, z = _proj(x, g["e1"]), _proj(x, g["e2"]), _proj(x, g["d"])
    izp = g["z_ref"] - z
    Tx = (u - g["u0"]) / g["s"] - F32(0.5)
    Ty = (v - g["v0"]) / g["s"] - F32(0.5)
    i0, j0 = np.floor(Tx), np.floor(Ty)
    fx, fy = (Tx - i0).astype(np.float64), (Ty - j0).astype(np.float64)
    i0, j0 = i0.astype(np.int64), j0.astype(np.int64)
    out = np.zeros(x.shape[1])
    for di, dj, w in ((0, 0, (1 - fx) * (1 - fy)), (1, 0, fx * (1 - fy)), (0, 1, (1 - fx) * fy), (1, 1, fx * fy)):
        i, j = i0 + di, j0 + dj
        inside = (i >= 0) & (i < R) & (j >= 0) & (j < R)
        q = np.where(inside, j * R + i, 0)
        iz0 = dom.iz0[q]
        has = inside & (iz0 > 0)
        xl = ((iz0 - izp) / dom.delta).astype(np.float64) - 1.0
        jl = np.floor(xl)
        jj = np.clip(jl, 0, K - 1).astype(np.int64)
        Cj = dom.C[q, jj]
        Cp = np.where(jj > 0, dom.C[q, np.maximum(jj - 1, 0)], 0.0)
        n = np.where(xl >= K, dom.C[q, K - 1], Cp + (xl - jl) * (Cj - Cp))
        n = np.where(has & (xl >= 0), n, 0.0)
        out += w * n
    return out


def shadow_counts(geom: LevelGeom, ras, cam, lights, R: int, K: int, delta: float, dom_geom: LevelGeom = None):
    """Per light, n_s of every camera fragment (float64 tensor) or None (point lights); the
    DOM of each directional light is built from dom_geom (default: the same geometry; the
    camera raster's rows may be pieces of dom_geom's long segments)."""
    x = lookup_point(geom, ras, cam)
    out = []
    for light in lights:
        if light.kind != 0:
            out.append(None)
            continue
        dom = build_dom(geom if dom_geom is None else dom_geom, light.vec, R, K, delta)
        out.append(torch.as_tensor(dom_count(dom, x), dtype=DT))
    return out
