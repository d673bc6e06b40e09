"""Projection, tile binning and coverage of hair segments (oracle, numpy).

The paper rasterises every (thick) hair segment as a camera-facing strip whose screen width
is computed per frame (Sec. 5.2, hair width calculation and shading pass).  This module
restates that as an exact integer predicate on a 1/16-pixel grid so the result is unique:

  * projection: v = R (p - c) with each row summed left to right, x = cx + fx (vx / -vz),
    y = cy - fy (vy / -vz), snapped X = rint(16 x), Y = rint(16 y) (half to even), inverse
    depth iz = 1 / -vz.  Float32, one rounding per operation, no fused multiply-add: these
    values decide integers, so they are taken in the kernel's precision.
  * cull: an endpoint nearer than z_near, a snapped coordinate outside the guard band
    [-2^14, 16 W + 2^14] (and likewise for H), or hw_fx > 32768 (2048 px).  A segment longer
    than 2^14 sub-pixels (1024 px) on an axis is drawn as pieces (render.split_long), each
    within that extent; the two limits keep every coverage product below 2^31.
  * half-width hw (pixels): a strand uses (w / 2) fy / z_mid; a thick hair uses the
    ellipse's support half-width across the view, at the segment midpoint, times fy / z_mid.
    The coverage radius is hw_fx = ceil(16 hw) sub-pixels, plus 8 (half a pixel) for the
    box filter.
  * fragment (segment, pixel centre P = (16 i + 8, 16 j + 8)) exists iff, with d = B - A,
    e = P - A:  d.d > 0,  0 <= e.d < d.d  (half-open, so a shared vertex is counted once),
    and (e x d)^2 < (hw_fx + 8)^2 (d.d).
  * depth key: t = float(e.d) / float(d.d), iz = izA + t (izB - izA) (float32, two
    roundings), key = 0xFFFFFFFF - bits(iz): nearer fragments have smaller keys.  Fragments
    of a pixel are composited in ascending (key, segment id).
  * tile binning: a segment belongs to every tile its integer box [min - R, max + R]
    (R = hw_fx + 8) overlaps, clipped to the screen.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
GUARD = 16384          # 2^14 sub-pixels = 1024 px
MAX_AXIS = 16384       # longest segment (or piece) extent per axis (sub-pixels)
MAX_HW_FX = 32768      # largest allowed coverage half-width (sub-pixels)
SPLIT_LEN = 16000      # a longer segment is cut into pieces of at most this extent (sub-pixels)
MAX_PIECES = 64


def cam_arrays(cam):
    """Camera fields as float32 scalars."""
    return dict(pos=np.asarray(cam.pos, dtype=F32), rot=np.asarray(cam.rot, dtype=F32).reshape(3, 3),
                fx=F32(cam.fx), fy=F32(cam.fy), cx=F32(cam.cx), cy=F32(cam.cy),
                z_near=F32(cam.z_near), W=int(cam.width), H=int(cam.height))


def view_transform(p, c):
    """v = R (p - c) in float32, rows summed left to right.  p: [3, N] float32."""
    R = c["rot"]
    d0 = p[0] - c["pos"][0]
    d1 = p[1] - c["pos"][1]
    d2 = p[2] - c["pos"][2]
    v = []
    for r in range(3):
        v.append((R[r, 0] * d0 + R[r, 1] * d1) + R[r, 2] * d2)
    return v


def project_points(p, c):
    """(X, Y) int64 sub-pixel coordinates, z = -vz, iz = 1/z, and an in-guard-band mask."""
    vx, vy, vz = view_transform(p, c)
    z = -vz
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        xs = c["cx"] + c["fx"] * (vx / z)
        ys = c["cy"] - c["fy"] * (vy / z)
        iz = F32(1.0) / z
        X16 = F32(16.0) * xs
        Y16 = F32(16.0) * ys
    ok = (z >= c["z_near"])
    ok &= (X16 >= F32(-GUARD)) & (X16 <= F32(16 * c["W"] + GUARD))
    ok &= (Y16 >= F32(-GUARD)) & (Y16 <= F32(16 * c["H"] + GUARD))
    X = np.where(ok, np.rint(np.where(ok, X16, 0)), 0).astype(np.int64)
    Y = np.where(ok, np.rint(np.where(ok, Y16, 0)), 0).astype(np.int64)
    return X, Y, z.astype(F32), iz.astype(F32), ok


def strand_halfwidth(zA, zB, width, c):
    """hw (pixels, float32) of a strand of diameter `width`: ((0.5 w) fy) / ((zA + zB) 0.5)."""
    zm = (zA + zB) * F32(0.5)
    with np.errstate(divide="ignore", invalid="ignore"):
        return ((F32(0.5) * width) * c["fy"]) / zm


def _norm3(x, y, z):
    return np.sqrt((x * x + y * y) + z * z)


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def cluster_halfwidth(pA, pB, zA, zB, ahat, a_len, b_len, c):
    """hw (pixels, float32) of a thick hair: support of its ellipse across the view.

    u = (B - A)/|B - A|; w = (c - m)/|c - m| with m the midpoint; x^ = normalize(w - (w.u) u),
    y^ = u x x^, b^ = u x a^; W = sqrt((|a| a^.y^)^2 + (|b| b^.y^)^2), or max(|a|, |b|) when
    |w - (w.u) u| <= 1e-7; hw = (W fy) / z_mid.  Float32, fixed operation order.
    """
    t = [pB[i] - pA[i] for i in range(3)]
    tl = _norm3(*t)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = [t[i] / tl for i in range(3)]
        m = [(pA[i] + pB[i]) * F32(0.5) for i in range(3)]
        w = [c["pos"][i] - m[i] for i in range(3)]
        wl = _norm3(*w)
        w = [w[i] / wl for i in range(3)]
        dwu = _dot(w, u)
        wp = [w[i] - dwu * u[i] for i in range(3)]
        wpl = _norm3(*wp)
        xh = [wp[i] / wpl for i in range(3)]
        yh = _cross(u, xh)
        bh = _cross(u, ahat)
        pa = a_len * _dot(ahat, yh)
        pb = b_len * _dot(bh, yh)
        W = np.sqrt(pa * pa + pb * pb)
        W = np.where(wpl > F32(1e-7), W, np.maximum(a_len, b_len))
        zm = (zA + zB) * F32(0.5)
        return (W * c["fy"]) / zm


def finalize_segments(XA, YA, XB, YB, okA, okB, hw):
    """Coverage radius and the final visibility mask (guard band, length and width limits)."""
    with np.errstate(invalid="ignore", over="ignore"):
        hw16 = np.ceil(F32(16.0) * hw)
    vis = okA & okB & np.isfinite(hw16) & (hw16 >= 0)
    hw_fx = np.where(vis, hw16, 0).astype(np.int64)
    vis &= (np.abs(XB - XA) <= MAX_AXIS) & (np.abs(YB - YA) <= MAX_AXIS) & (hw_fx <= MAX_HW_FX)
    return hw_fx, vis


def h_sign(pA, pB, c, XA, YA, XB, YB):
    """Sign that makes the cross-section offset h positive toward y^ = u x x^ (float64).

    Computed at the segment midpoint from the screen-space image of y^ (the Jacobian of
    the projection applied to y^) against the screen normal (dY, -dX) on which e x d > 0.
    """
    A = pA.astype(np.float64)
    B = pB.astype(np.float64)
    cam = c["pos"].astype(np.float64)
    R = c["rot"].astype(np.float64)
    t = B - A
    u = t / np.linalg.norm(t, axis=0)
    m = 0.5 * (A + B)
    w = cam[:, None] - m
    w = w / np.linalg.norm(w, axis=0)
    wp = w - (w * u).sum(0) * u
    nrm = np.linalg.norm(wp, axis=0)
    xh = wp / np.where(nrm > 0, nrm, 1.0)
    yh = np.cross(u.T, xh.T).T
    yv = R @ yh
    mv = R @ (m - cam[:, None])
    Z = -mv[2]
    sx = float(c["fx"]) * (yv[0] + (mv[0] / Z) * yv[2])
    sy = -float(c["fy"]) * (yv[1] + (mv[1] / Z) * yv[2])
    dX = (XB - XA).astype(np.float64)
    dY = (YB - YA).astype(np.float64)
    return np.where(sx * dY - sy * dX >= 0.0, 1.0, -1.0)


def tile_ranges(XA, YA, XB, YB, hw_fx, vis, W, H, tile):
    """Inclusive tile index ranges [tx0, tx1] x [ty0, ty1] per segment (empty -> tx0 > tx1)."""
    R = hw_fx + 8
    T = 16 * tile
    lox = np.minimum(XA, XB) - R
    hix = np.maximum(XA, XB) + R
    loy = np.minimum(YA, YB) - R
    hiy = np.maximum(YA, YB) + R
    ntx = (W + tile - 1) // tile
    nty = (H + tile - 1) // tile
    tx0 = np.clip(np.floor_divide(lox, T), 0, None)
    tx1 = np.clip(np.floor_divide(hix, T), None, ntx - 1)
    ty0 = np.clip(np.floor_divide(loy, T), 0, None)
    ty1 = np.clip(np.floor_divide(hiy, T), None, nty - 1)
    empty = ~vis | (tx0 > tx1) | (ty0 > ty1)
    tx1 = np.where(empty, tx0 - 1, tx1)
    return tx0, tx1, ty0, ty1


def tile_meets_footprint(XA, YA, XB, YB, hw_fx, seg, tx, ty, tile):
    """Whether the rectangle of tile (tx, ty)'s pixel centres meets segment seg's footprint
    (slab 0 <= t_num <= t_den, strip |cross| <= R sqrt(t_den)), by projecting its four corner
    centres on the segment's direction and normal (exact integers).  Applied to wide segments
    (R above 32 sub-pixels, 2 px); thin and zero-length segments keep every tile of their box."""
    xa, ya = XA[seg].astype(np.int64), YA[seg].astype(np.int64)
    dx, dy = XB[seg].astype(np.int64) - xa, YB[seg].astype(np.int64) - ya
    tden = dx * dx + dy * dy
    R = hw_fx[seg].astype(np.int64) + 8
    RR = R * R * tden
    ex0 = 16 * tile * tx.astype(np.int64) + 8 - xa
    ey0 = 16 * tile * ty.astype(np.int64) + 8 - ya
    span = 16 * (tile - 1)
    tn = [ex * dx + ey * dy for ex in (ex0, ex0 + span) for ey in (ey0, ey0 + span)]
    cr = [ex * dy - ey * dx for ex in (ex0, ex0 + span) for ey in (ey0, ey0 + span)]
    tmin, tmax = np.minimum.reduce(tn), np.maximum.reduce(tn)
    cmin, cmax = np.minimum.reduce(cr), np.maximum.reduce(cr)
    apart = (tmax < 0) | (tmin > tden) | ((cmin > 0) & (cmin * cmin >= RR)) | ((cmax < 0) & (cmax * cmax >= RR))
    return (tden <= 0) | (R <= 32) | ~apart


def bins(XA, YA, XB, YB, hw_fx, vis, W, H, tile):
    """(tile_id, seg_id) pairs, sorted by tile then segment id: the tiles of each segment's box
    widened by its radius whose pixel centres can meet its footprint."""
    tx0, tx1, ty0, ty1 = tile_ranges(XA, YA, XB, YB, hw_fx, vis, W, H, tile)
    ntx = (W + tile - 1) // tile
    nx = np.maximum(tx1 - tx0 + 1, 0)
    ny = np.maximum(ty1 - ty0 + 1, 0)
    cnt = nx * ny
    seg = np.repeat(np.arange(XA.size, dtype=np.int64), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(seg.size, dtype=np.int64) - start
    nxs = nx[seg]
    tx = tx0[seg] + local % np.maximum(nxs, 1)
    ty = ty0[seg] + local // np.maximum(nxs, 1)
    keep = tile_meets_footprint(XA, YA, XB, YB, hw_fx, seg, tx, ty, tile)
    seg, tx, ty = seg[keep], tx[keep], ty[keep]
    cnt = np.bincount(seg, minlength=XA.size)
    tid = ty * ntx + tx
    order = np.lexsort((seg, tid))
    return tid[order], seg[order], cnt


def candidate_pixels(XA, YA, XB, YB, hw_fx, vis, W, H, seg_subset=None, pix_filter=None):
    """All (segment, pixel) pairs whose pixel centre lies in the segment's expanded box."""
    R = hw_fx + 8
    lox = np.minimum(XA, XB) - R
    hix = np.maximum(XA, XB) + R
    loy = np.minimum(YA, YB) - R
    hiy = np.maximum(YA, YB) + R
    # pixel i has centre 16 i + 8; need lo < 16 i + 8 < hi (strict: the predicate is strict)
    i0 = np.clip(np.floor_divide(lox - 8, 16) + 1, 0, None)
    i1 = np.clip(-np.floor_divide(-(hix - 8), 16) - 1, None, W - 1)
    j0 = np.clip(np.floor_divide(loy - 8, 16) + 1, 0, None)
    j1 = np.clip(-np.floor_divide(-(hiy - 8), 16) - 1, None, H - 1)
    idx = np.arange(XA.size) if seg_subset is None else np.asarray(seg_subset)
    idx = idx[vis[idx]]
    nx = np.maximum(i1[idx] - i0[idx] + 1, 0)
    ny = np.maximum(j1[idx] - j0[idx] + 1, 0)
    cnt = nx * ny
    seg = np.repeat(idx, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(seg.size, dtype=np.int64) - start
    nxs = np.maximum(nx, 1)[np.repeat(np.arange(idx.size), cnt)]
    pi = i0[seg] + local % nxs
    pj = j0[seg] + local // nxs
    if pix_filter is not None:
        keep = pix_filter(pi, pj)
        seg, pi, pj = seg[keep], pi[keep], pj[keep]
    return seg, pi, pj


def coverage(XA, YA, XB, YB, hw_fx, seg, pi, pj):
    """Exact integer predicate for each candidate; returns mask and (t_num, t_den, cross)."""
    Ax, Ay, Bx, By = XA[seg], YA[seg], XB[seg], YB[seg]
    dx = Bx - Ax
    dy = By - Ay
    ex = (16 * pi + 8) - Ax
    ey = (16 * pj + 8) - Ay
    t_num = ex * dx + ey * dy
    t_den = dx * dx + dy * dy
    cross = ex * dy - ey * dx
    R = hw_fx[seg] + 8
    ok = (t_den > 0) & (t_num >= 0) & (t_num < t_den) & (cross * cross < R * R * t_den)
    return ok, t_num, t_den, cross


def depth_key(t_num, t_den, izA, izB):
    """(key uint32, t float32, iz float32) with t and iz rounded as the kernel rounds them."""
    t = t_num.astype(F32) / t_den.astype(F32)
    iz = izA + t * (izB - izA)
    key = np.uint32(0xFFFFFFFF) - iz.view(np.uint32)
    return key, t, iz
