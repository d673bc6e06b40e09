"""Per-fragment radiance and depth-ordered compositing (oracle).

  * Radiance of a fragment: L = sum over lights of E * f(omega_i, omega_o, h) * cos(theta_i)
    (Sec. 3, the fibre rendering equation with a directional or point light: f cos^2 theta_i
    d theta_i d phi_i = f cos theta_i d omega_i).  A directional light has irradiance E; a
    point light E = I / |x_L - x|^2.  No shadowing between hairs.  f is the near-field
    R / TT / TRT model (fiber, aggregate) for a (eta, alpha, beta_m, beta_n) material and the
    R / TT / D model (rttd) for an rttd.RTTD material.
  * Shading frame: u = unit segment tangent, omega_o toward the camera from the fragment's
    world point (perspective-correct parameter t_w = t izB / iz), x^ = normalize(omega_o -
    (omega_o . u) u), y^ = u x x^, sin theta = omega . u, phi = phi_o - phi_i =
    -atan2(omega_i . y^, omega_i . x^) (phi = 0 when |omega_o - (omega_o . u) u| < 1e-7).
  * Cross-section offset of a fragment: h = clamp(sigma sgn(e x d) delta / (hw + 1/2), -1, 1),
    delta the pixel centre's distance to the segment line in pixels and sigma the
    per-segment sign making h > 0 toward y^: h runs over [-1, 1] across the fragment
    footprint (half-width hw + 1/2), as a strip coordinate does across a rasterised strip.
  * Coverage alpha = clamp(min(delta + hw, 1/2) - max(delta - hw, -1/2), 0, 1): a unit box
    filter across the strip.
  * Compositing: fragments of a pixel in ascending (key, segment id), front to back,
    C = sum_k T_k alpha_k L_k, T_0 = 1, T_{k+1} = T_k (1 - alpha_k); output (C, 1 - T_N),
    premultiplied over transparent black.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import raster as rs
from . import rttd
from .aggregate import ellipse_chord, ellipse_support, f_ours, hair_counts
from .fiber import angles, f_single

DT = torch.float64


@dataclass
class LevelGeom:
    """Segments of one LoD level, one row per segment (global segment id = row index)."""
    kind: str                  # "strand", "cluster" or "mixed" (per-row `thick` decides)
    pA: np.ndarray             # f32 [3, S]
    pB: np.ndarray             # f32 [3, S]
    sigma_a: np.ndarray        # f32 [S, 3]
    width: np.ndarray = None   # f32 [S] strand diameter
    ahat: np.ndarray = None    # f32 [3, S]
    a_len: np.ndarray = None   # f32 [S]
    b_len: np.ndarray = None   # f32 [S]
    n_total: np.ndarray = None  # i32 [S]
    r: np.ndarray = None       # f32 [S]
    cluster: np.ndarray = None  # i64 [S] cluster of each segment
    seg_in_cluster: np.ndarray = None
    thick: np.ndarray = None   # bool [S]: mixed frames, rows that are thick hairs
    parent: np.ndarray = None  # i64 [rows]: after split_long, the segment each piece comes from


def strand_level(asset) -> LevelGeom:
    V, S, n = asset.verts_per_strand, asset.segs, asset.n_strands
    cols = (np.arange(n)[:, None] * V + np.arange(S)[None, :]).reshape(-1)
    strand = np.repeat(np.arange(n), S)
    return LevelGeom("strand", asset.xyz[:, cols].copy(), asset.xyz[:, cols + 1].copy(),
                     asset.sigma_a.T[strand].copy(), width=asset.width[strand].copy())


def cluster_level(lod) -> LevelGeom:
    K, V, _ = lod["centers"].shape
    S = V - 1
    c = lod["centers"]
    pA = c[:, :-1].reshape(K * S, 3).T.copy()
    pB = c[:, 1:].reshape(K * S, 3).T.copy()
    cl = np.repeat(np.arange(K), S)
    return LevelGeom("cluster", pA, pB, lod["sigma_a"].T[cl].copy(),
                     ahat=lod["ahat"].reshape(K * S, 3).T.copy(),
                     a_len=lod["axes"][:, :, 0].reshape(-1).copy(), b_len=lod["axes"][:, :, 1].reshape(-1).copy(),
                     n_total=lod["n_total"][cl].copy(), r=lod["r"][cl].copy(), cluster=cl,
                     seg_in_cluster=np.tile(np.arange(S), K))


@dataclass
class Raster:
    XA: np.ndarray
    YA: np.ndarray
    XB: np.ndarray
    YB: np.ndarray
    izA: np.ndarray
    izB: np.ndarray
    hw: np.ndarray          # f32 half-width (px)
    hw_fx: np.ndarray
    vis: np.ndarray
    sign: np.ndarray        # +-1 per segment
    # fragments, sorted by (pixel, key, seg)
    seg: np.ndarray
    pix: np.ndarray
    key: np.ndarray
    t_num: np.ndarray
    t_den: np.ndarray
    cross: np.ndarray
    W: int
    H: int


def segment_records(geom: LevelGeom, cam):
    c = rs.cam_arrays(cam)
    XA, YA, zA, izA, okA = rs.project_points(geom.pA, c)
    XB, YB, zB, izB, okB = rs.project_points(geom.pB, c)
    if geom.kind == "strand":
        hw = rs.strand_halfwidth(zA, zB, geom.width, c)
    elif geom.kind == "cluster":
        hw = rs.cluster_halfwidth(geom.pA, geom.pB, zA, zB, geom.ahat, geom.a_len, geom.b_len, c)
    else:   # mixed: each row by its own kind
        t = geom.thick
        hw = np.empty(zA.shape, dtype=np.float32)
        hw[~t] = rs.strand_halfwidth(zA[~t], zB[~t], geom.width[~t], c)
        hw[t] = rs.cluster_halfwidth(geom.pA[:, t], geom.pB[:, t], zA[t], zB[t], geom.ahat[:, t], geom.a_len[t],
                                     geom.b_len[t], c)
    hw_fx, vis = rs.finalize_segments(XA, YA, XB, YB, okA, okB, hw)
    return c, XA, YA, XB, YB, izA, izB, hw.astype(np.float32), hw_fx, vis


def split_long(geom: LevelGeom, cam) -> LevelGeom:
    """Segments longer than 1024 px on a screen axis, as pieces (projection step, Sec. 5.2).

    A segment whose snapped endpoints are both on the guard band and whose extent
    max(|dX|, |dY|) exceeds 2^14 sub-pixels is drawn as m = min(ceil(extent / 16000), 64)
    pieces of equal screen parameter: piece j runs between the world points of screen
    parameters j / m and (j + 1) / m, found with the perspective-correct parameter (inverse
    depth is affine on screen: t_w = s izB / (izA + s (izB - izA))), float32 with one rounding
    per operation: s = j / m, iz = izA + s (izB - izA), t_w = (s izB) / iz, P = A + t_w (B - A),
    and P = A, B exactly at s = 0, 1.  A piece keeps its segment's attributes; rows are in
    (segment, piece) order and `parent` maps each row to its segment.  Frames without such a
    segment are returned unchanged."""
    c = rs.cam_arrays(cam)
    XA, YA, _, izA, okA = rs.project_points(geom.pA, c)
    XB, YB, _, izB, okB = rs.project_points(geom.pB, c)
    ext = np.maximum(np.abs(XB - XA), np.abs(YB - YA))
    long = okA & okB & (ext > rs.MAX_AXIS)
    if not long.any():
        return geom
    m = np.where(long, np.minimum((ext + rs.SPLIT_LEN - 1) // rs.SPLIT_LEN, rs.MAX_PIECES), 1).astype(np.int64)
    parent = np.repeat(np.arange(m.size), m)
    j = np.arange(parent.size) - np.repeat(np.cumsum(m) - m, m)
    F = np.float32

    def point(jj):
        mm = m[parent].astype(F)
        sp = jj.astype(F) / mm
        a, b = izA[parent], izB[parent]
        iz = a + sp * (b - a)
        with np.errstate(divide="ignore", invalid="ignore"):
            tw = (sp * b) / iz
        A, B = geom.pA[:, parent], geom.pB[:, parent]
        P = np.stack([A[i] + tw * (B[i] - A[i]) for i in range(3)]).astype(F)
        P = np.where((jj == 0)[None, :], A, P)
        return np.where((jj == m[parent])[None, :], B, P)

    pick = lambda x: None if x is None else x[parent].copy()      # per-row attributes [S]
    out = LevelGeom(geom.kind, point(j), point(j + 1), geom.sigma_a[parent].copy(),
                    width=None if geom.width is None else geom.width[parent].copy(),
                    ahat=None if geom.ahat is None else geom.ahat[:, parent].copy(),
                    a_len=pick(geom.a_len), b_len=pick(geom.b_len), n_total=pick(geom.n_total), r=pick(geom.r),
                    cluster=pick(geom.cluster), seg_in_cluster=pick(geom.seg_in_cluster), thick=pick(geom.thick),
                    parent=parent if geom.parent is None else geom.parent[parent])
    return out


def rasterize(geom: LevelGeom, cam, pix_filter=None, rect=None) -> Raster:
    """All fragments, or (rect = (x0, y0, w, h)) only those of pixels inside the rectangle."""
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = segment_records(geom, cam)
    sign = rs.h_sign(geom.pA, geom.pB, c, XA, YA, XB, YB)
    subset = None
    if rect is not None:
        x0, y0, w, h = rect
        R = hw_fx + 8
        near = ((np.minimum(XA, XB) - R < 16 * (x0 + w)) & (np.maximum(XA, XB) + R > 16 * x0) &
                (np.minimum(YA, YB) - R < 16 * (y0 + h)) & (np.maximum(YA, YB) + R > 16 * y0))
        subset = np.nonzero(near & vis)[0]
        inner = pix_filter
        pix_filter = lambda i, j: ((i >= x0) & (i < x0 + w) & (j >= y0) & (j < y0 + h)
                                   & (inner(i, j) if inner else True))
    seg, pi, pj = rs.candidate_pixels(XA, YA, XB, YB, hw_fx, vis, c["W"], c["H"], seg_subset=subset,
                                      pix_filter=pix_filter)
    ok, t_num, t_den, cross = rs.coverage(XA, YA, XB, YB, hw_fx, seg, pi, pj)
    seg, pi, pj, t_num, t_den, cross = seg[ok], pi[ok], pj[ok], t_num[ok], t_den[ok], cross[ok]
    key, _, _ = rs.depth_key(t_num, t_den, izA[seg], izB[seg])
    pix = pj * c["W"] + pi
    order = np.lexsort((seg, key, pix))
    return Raster(XA, YA, XB, YB, izA, izB, hw, hw_fx, vis, sign,
                  seg[order], pix[order], key[order], t_num[order], t_den[order], cross[order],
                  c["W"], c["H"])


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=DT)


def _normalize(v):
    return v / torch.linalg.norm(v, dim=-1, keepdim=True)


def fragment_alpha_h(ras: Raster, hw):
    """alpha and h per fragment (float64).  hw: per-fragment half-width tensor (px)."""
    cross = _t(ras.cross)
    delta = torch.abs(cross) / torch.sqrt(_t(ras.t_den)) / 16.0
    alpha = torch.clamp(torch.minimum(delta + hw, torch.full_like(hw, 0.5))
                        - torch.maximum(delta - hw, torch.full_like(hw, -0.5)), 0.0, 1.0)
    sgn = torch.sign(cross) * _t(ras.sign[ras.seg])
    h = torch.clamp(sgn * delta / (hw + 0.5), -1.0, 1.0)
    return alpha, h


def perspective_t(t, izA, izB):
    """World parameter t_w of the point at screen parameter t on a segment whose endpoints
    have inverse depths izA, izB: inverse depth is affine in screen space, so with
    iz = izA + t (izB - izA) the world parameter is t_w = t izB / iz."""
    iz = izA + t * (izB - izA)
    return t * izB / iz


def azimuth(wi, xh, yh, degen):
    """phi = phi_o - phi_i with phi_o = 0 (Sec. 3.1): minus the angle of omega_i about u from
    x^ toward y^ = u x x^; 0 where the view runs along the fibre."""
    phi = -torch.atan2((wi * yh).sum(-1), (wi * xh).sum(-1))
    return torch.where(degen, torch.zeros_like(phi), phi)


def shading_inputs(geom: LevelGeom, ras: Raster, cam):
    """World point, tangent u and view direction per fragment (float64)."""
    s = ras.seg
    pA = _t(geom.pA[:, s].T)
    pB = _t(geom.pB[:, s].T)
    t = _t(ras.t_num) / _t(ras.t_den)
    tw = perspective_t(t, _t(ras.izA[s]), _t(ras.izB[s]))
    xw = pA + tw[:, None] * (pB - pA)
    u = _normalize(pB - pA)
    wo = _normalize(_t(np.asarray(cam.pos, dtype=np.float32))[None, :] - xw)
    return xw, u, wo


def frame(u, wo):
    """x^, y^ and the degenerate mask (|omega_o perp| < 1e-7)."""
    sin_to = (wo * u).sum(-1)
    wp = wo - sin_to[:, None] * u
    nrm = torch.linalg.norm(wp, dim=-1)
    degen = nrm < 1e-7
    # any vector orthogonal to u serves when the view runs along the fibre
    helper = torch.zeros_like(u)
    j = torch.argmin(torch.abs(u), dim=-1)
    helper[torch.arange(u.shape[0]), j] = 1.0
    hp = helper - (helper * u).sum(-1, keepdim=True) * u
    wp = torch.where(degen[:, None], hp, wp)
    xh = _normalize(wp)
    yh = torch.linalg.cross(u, xh, dim=-1)
    return xh, yh, degen, sin_to


def light_dirs(light, xw):
    vec = _t(np.asarray(light.vec, dtype=np.float32))
    rgb = _t(np.asarray(light.rgb, dtype=np.float32))
    if light.kind == 0:
        wi = vec.expand_as(xw)
        E = rgb.expand(xw.shape[0], 3)
    else:
        d = vec[None, :] - xw
        dist2 = (d * d).sum(-1)
        wi = d / torch.sqrt(dist2)[:, None]
        E = rgb[None, :] / dist2[:, None]
    return wi, E


def _mixed_radiance(geom: LevelGeom, ras: Raster, cam, lights, mat, shadow=None):
    """Mixed frames: strand fragments by f_single, thick-hair fragments by f_ours."""
    from dataclasses import replace
    thick_f = geom.thick[ras.seg]
    alpha = torch.zeros(len(ras.seg), dtype=DT)
    L = torch.zeros(len(ras.seg), 3, dtype=DT)
    for kind, m in (("strand", ~thick_f), ("cluster", thick_f)):
        if not m.any():
            continue
        sub = replace(ras, seg=ras.seg[m], pix=ras.pix[m], key=ras.key[m], t_num=ras.t_num[m], t_den=ras.t_den[m],
                      cross=ras.cross[m])
        sh = None if shadow is None else [None if n is None else n[torch.as_tensor(np.nonzero(m)[0])] for n in shadow]
        a, l = fragment_radiance(replace(geom, kind=kind), sub, cam, lights, mat, shadow=sh)
        idx = torch.as_tensor(np.nonzero(m)[0])
        alpha[idx] = a
        L[idx] = l
    return alpha, L


def material(m):
    """Oracle material from an object with the library's material fields, at the float32
    values the library receives: an (eta, alpha, beta_m, beta_n) tuple for model 0, an
    rttd.RTTD for model 1."""
    f = lambda v: float(np.float32(v))
    if getattr(m, "model", 0) == 1:
        return rttd.RTTD(f(m.beta_r), f(m.beta_tt), f(m.gamma_tt), tuple(f(v) for v in m.a_r),
                         tuple(f(v) for v in m.a_tt), tuple(f(v) for v in m.a_d))
    return (f(m.eta), f(m.alpha), f(m.beta_m), f(m.beta_n))


def fragment_radiance(geom: LevelGeom, ras: Raster, cam, lights, mat, params=None, shadow=None):
    """(alpha [F], L [F, 3]) in float64.

    params (cluster levels, for the gradient oracle): dict of torch tensors
    'a_len', 'b_len' [S], 'r' [S], 'sigma_a' [S, 3], and 'hw' [S] (the half-width recomputed
    from them); default: the level's stored values and the float32 half-width.
    shadow: per light, the number of hairs n_s in front of each fragment toward the light
    (oracle.shadow) or None: a strand with n_s > 0 is shaded by f_ours with n_total = 1 and
    n_F = 1 + n_s, a thick hair's n_F grows by n_s.
    """
    if geom.kind == "mixed":
        return _mixed_radiance(geom, ras, cam, lights, mat, shadow)
    s = ras.seg
    xw, u, wo = shading_inputs(geom, ras, cam)
    xh, yh, degen, sin_to = frame(u, wo)
    if params is None:
        hw = _t(ras.hw[s])
        sig = _t(geom.sigma_a[s])
    else:
        hw = params["hw"][s]
        sig = params["sigma_a"][s]
    alpha, h = fragment_alpha_h(ras, hw)
    if geom.kind == "cluster":
        ahat = _t(geom.ahat[:, s].T)
        bhat = torch.linalg.cross(u, ahat, dim=-1)
        if params is None:
            a_len, b_len, r = _t(geom.a_len[s]), _t(geom.b_len[s]), _t(geom.r[s])
        else:
            a_len, b_len, r = params["a_len"][s], params["b_len"][s], params["r"][s]
        n_total = _t(geom.n_total[s])
        W = ellipse_support(a_len, b_len, ahat, bhat, yh)
    L = torch.zeros(len(s), 3, dtype=DT)
    for li, light in enumerate(lights):
        ns = None if shadow is None else shadow[li]
        wi, E = light_dirs(light, xw)
        sin_ti = (wi * u).sum(-1)
        phi = azimuth(wi, xh, yh, degen)
        _, _, th, xd = angles(sin_ti, sin_to)
        sc = torch.clamp(sin_ti, -1.0, 1.0)
        cos_ti = torch.sqrt((1.0 - sc) * (1.0 + sc))
        if geom.kind == "strand":
            f = rttd.f_single(th, phi, mat) if isinstance(mat, rttd.RTTD) else f_single(th, xd, phi, h, sig, mat)
            if ns is not None:
                one = torch.ones_like(th)
                if isinstance(mat, rttd.RTTD):
                    fo = rttd.f_ours(th, phi, mat, one, one, 1.0 + ns, one)
                else:
                    fo = f_ours(th, xd, phi, h, sig, mat, one, one, 1.0 + ns, one)
                f = torch.where((ns > 0)[:, None], fo, f)
        else:
            Dp = wi - sin_ti[:, None] * u
            dn = torch.linalg.norm(Dp, dim=-1)
            D = Dp / torch.where(dn > 1e-7, dn, torch.ones_like(dn))[:, None]
            s_star = ellipse_chord(h, W, xh, yh, ahat, bhat, a_len, b_len, D)
            s_star = torch.where(dn > 1e-7, s_star, torch.zeros_like(s_star))
            rho, n_F, n_B = hair_counts(phi, s_star, n_total, r, a_len, b_len)
            if ns is not None:
                n_F = n_F + ns
            if isinstance(mat, rttd.RTTD):
                f = rttd.f_ours(th, phi, mat, n_total, rho, n_F, n_B)
            else:
                f = f_ours(th, xd, phi, h, sig, mat, n_total, rho, n_F, n_B)
        L = L + E * f * cos_ti[:, None]
    return alpha, L


def composite(ras: Raster, alpha, L):
    """Front-to-back over per pixel; returns (rgba [H, W, 4] float64 tensor)."""
    npx = ras.W * ras.H
    pix = torch.as_tensor(ras.pix, dtype=torch.int64)
    C = torch.zeros(npx, 3, dtype=DT)
    T = torch.ones(npx, dtype=DT)
    if len(ras.pix):
        first = np.ones(len(ras.pix), dtype=bool)
        first[1:] = ras.pix[1:] != ras.pix[:-1]
        start = np.maximum.accumulate(np.where(first, np.arange(len(ras.pix)), 0))
        rank = np.arange(len(ras.pix)) - start
        for k in range(int(rank.max()) + 1):
            sel = torch.as_tensor(np.nonzero(rank == k)[0])
            p = pix[sel]
            a = alpha[sel]
            C = C.index_add(0, p, T[p][:, None] * a[:, None] * L[sel])
            T = T.index_copy(0, p, T[p] * (1.0 - a))
    rgba = torch.cat([C, (1.0 - T)[:, None]], dim=1)
    return rgba.reshape(ras.H, ras.W, 4)


def render(geom: LevelGeom, cam, lights, mat, pix_filter=None, rect=None, shadow=None):
    """Oracle frame: returns (rgba float64 [H, W, 4] numpy, Raster).  shadow = (R, K, Delta):
    shade with deep opacity maps of that resolution, layer count and layer depth (the maps
    rasterise the segments themselves; the camera raster draws long segments as pieces).
    The Raster's segment ids index split_long(geom, cam)."""
    cgeom = split_long(geom, cam)
    ras = rasterize(cgeom, cam, pix_filter=pix_filter, rect=rect)
    ns = None
    if shadow is not None:
        from . import shadow as sh
        ns = sh.shadow_counts(cgeom, ras, cam, lights, *shadow, dom_geom=geom)
    alpha, L = fragment_radiance(cgeom, ras, cam, lights, mat, shadow=ns)
    return composite(ras, alpha, L).numpy(), ras


def select_level(geoms, cam, eps_w: float = 2.0):
    """Per-request LoD: the coarsest level whose widest visible thick hair (2 hw) is at most
    eps_w pixels (Sec. 5.1 step 5 with the threshold of Sec. 6, eps_w = 2 px); level 0 (the
    strands) when none is.  geoms: list ordered finer -> coarser."""
    for lvl in range(len(geoms) - 1, 0, -1):
        _, _, _, _, _, _, _, hw, _, vis = segment_records(geoms[lvl], cam)
        w = 2.0 * hw[vis].astype(np.float64)
        if w.size == 0 or float(w.max()) <= eps_w:
            return lvl
    return 0
