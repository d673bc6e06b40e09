"""Curved thick hairs: Catmull-Rom centre lines tessellated by screen length (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper represents each thick hair by a spline through its centre control points and lets
the tessellation stage subdivide it by distance to the camera (Sec. 5.2 shading pass; Sec. 6
uses 16 control points; the hierarchy build fits Catmull-Rom splines, Sec. 5.1).  Readings:

  * Centre line: the uniform Catmull-Rom spline through the level's centre vertices c_0..c_S
    (the polyline level's vertices), ends clamped (c_-1 = c_0, c_S+1 = c_S).  Segment k runs
    from c_k (u = 0) to c_k+1 (u = 1):
        P(u) = ((w0 c_k-1 + w1 c_k) + w2 c_k+1) + w3 c_k+2,
        w0 = 0.5 ((2 u2 - u3) - u), w1 = 0.5 ((3 u3 - 5 u2) + 2), w2 = 0.5 ((4 u2 - 3 u3) + u),
        w3 = 0.5 (u3 - u2),  u2 = u u, u3 = u2 u,
    float32, one rounding per operation in this order; u = 0 and u = 1 give c_k and c_k+1
    exactly (so consecutive segments share their joint).
  * Tessellation: segment k of the polyline level is split into m equal parameter steps,
    m = the smallest integer in [1, m_max] with (16 m L)^2 >= dX^2 + dY^2, where (dX, dY) is
    the segment's snapped screen extent (1/16 pixel) and L the target sub-segment length in
    pixels: an integer decision.  Segments with an endpoint outside the camera's guard band or
    behind the near plane are not split.
  * Sub-segment j of segment k joins P(j / m) and P((j + 1) / m) (u = float(j) / float(m));
    it keeps segment k's cross-section (a^, |a|, |b|), cluster, hair count, radius and
    absorption.  Rows are ordered by segment, then j; the row index is the segment id that
    breaks depth ties.
"""
from __future__ import annotations

import numpy as np

from . import raster as rs
from .render import LevelGeom

F32 = np.float32


def weights(u):
    """Catmull-Rom basis (w0, w1, w2, w3) at float32 u, fixed operation order."""
    u = np.asarray(u, dtype=F32)
    u2 = u * u
    u3 = u2 * u
    h = F32(0.5)
    w0 = h * ((F32(2.0) * u2 - u3) - u)
    w1 = h * ((F32(3.0) * u3 - F32(5.0) * u2) + F32(2.0))
    w2 = h * ((F32(4.0) * u2 - F32(3.0) * u3) + u)
    w3 = h * (u3 - u2)
    return w0, w1, w2, w3


def point(c, k, u):
    """P_k(u) for control points c [V, 3] float32 (one hair), segment index k, float32 u."""
    S = c.shape[0] - 1
    if u == F32(0.0):
        return c[k].copy()
    if u == F32(1.0):
        return c[k + 1].copy()
    i = [min(max(k + d, 0), S) for d in (-1, 0, 1, 2)]
    w0, w1, w2, w3 = weights(u)
    return ((w0 * c[i[0]] + w1 * c[i[1]]) + w2 * c[i[2]]) + w3 * c[i[3]]


def tess_counts(geom: LevelGeom, cam, max_px: int, max_sub: int):
    """Sub-segments per segment of a polyline thick-hair level (int64 [S_total])."""
    c = rs.cam_arrays(cam)
    XA, YA, _, _, okA = rs.project_points(geom.pA, c)
    XB, YB, _, _, okB = rs.project_points(geom.pB, c)
    d2 = (XB - XA) ** 2 + (YB - YA) ** 2
    T = 16 * int(max_px)
    m = np.ones(len(d2), dtype=np.int64)
    for j in range(1, max_sub):
        m += ((m == j) & ((j * T) ** 2 < d2)).astype(np.int64)
    return np.where(okA & okB, m, 1)


def curved_geometry(lod, cam, max_px: int, max_sub: int) -> LevelGeom:
    """The tessellated rows of a thick-hair level (lod dict as oracle.lod builds it)."""
    from .render import cluster_level
    poly = cluster_level(lod)
    m = tess_counts(poly, cam, max_px, max_sub)
    K, V, _ = lod["centers"].shape
    S = V - 1
    centers = lod["centers"].astype(F32)
    pA, pB, par = [], [], []
    for g in range(K * S):
        cl, k = divmod(g, S)
        for j in range(int(m[g])):
            u0 = F32(j) / F32(m[g])
            u1 = F32(j + 1) / F32(m[g])
            pA.append(point(centers[cl], k, u0))
            pB.append(point(centers[cl], k, u1))
            par.append(g)
    par = np.asarray(par, dtype=np.int64)
    return LevelGeom("cluster", np.asarray(pA, F32).T.copy(), np.asarray(pB, F32).T.copy(),
                     poly.sigma_a[par].copy(), ahat=poly.ahat[:, par].copy(), a_len=poly.a_len[par].copy(),
                     b_len=poly.b_len[par].copy(), n_total=poly.n_total[par].copy(), r=poly.r[par].copy(),
                     cluster=poly.cluster[par].copy(), seg_in_cluster=poly.seg_in_cluster[par].copy())
