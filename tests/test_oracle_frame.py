"""Pins of the oracle's shading frame against an independent float64 ray trace (CPU).

The oracle turns a fragment into shading inputs with three conventions of its own: the side
of the strand on which the cross-section offset h is positive (raster.h_sign), the world
point of a fragment (the perspective-correct parameter render.perspective_t) and the
azimuth phi (render.azimuth, with x^ toward the camera and y^ = u x x^).  Here a wide strand
(and a one-hair and an elliptical thick hair) is rendered, and for every covered pixel
centre the camera ray is traced by brute force against the hair's cylinder:

  * h: its sign equals the sign of the ray's closest approach to the axis along y^ (the
    offset at which the view ray enters the fibre's cross-section, which the disc trace of
    the single-fibre tests takes as h), and its size that offset over the radius;
  * phi: the direction into which the surface at the ray's hit point mirrors the camera
    ray is where the R lobe of a fibre must peak: there phi equals the exit azimuth
    Phi(0, h) = -2 asin(h) of Sec. 3.1 at the traced offset, and theta_h = 0;
  * world point: the oracle's point on the centre line projects onto the foot of the pixel
    centre on the projected segment (perspective projection in float64);
  * point lights: E = I / d^2 is checked by its limits: moving a light twice as far along
    the same ray with four times the intensity leaves every fragment's radiance unchanged,
    and a distant point light approaches the directional light of the same direction.

Planted mistakes (a flipped h_sign, the affine screen parameter as world parameter, a
mirrored azimuth, a 1/d falloff) make these pins fail; each is planted in the oracle here,
on the CPU.
"""
import math

import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import raster as rs
from oracle import render as R
from oracle.fiber import angles, exit_azimuth

F32 = np.float32
W, H = 320, 240


def _camera():
    return hs.Camera(np.array([0.02, -0.01, 1.0], F32), np.eye(3, dtype=F32), 400.0, 400.0, 160.0, 120.0, W, H, 0.01)


def _polyline(a, b, n):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    pts = np.stack([a + (b - a) * k / n for k in range(n + 1)]).astype(F32)
    return pts[:-1].T.copy(), pts[1:].T.copy()


# straight thick strands, each a polyline of 3 segments, running in different screen
# directions and deep in z (strong perspective): radius 0.024 m, ~9 px at ~1 m
STRANDS = [((-0.28, -0.10, 0.25), (0.25, 0.12, -0.35)),
           ((0.22, 0.20, -0.30), (-0.20, -0.18, 0.20)),
           ((0.05, -0.25, 0.10), (-0.02, 0.26, -0.20))]
RADIUS = 0.024


def _strand_geom():
    pA, pB = zip(*[_polyline(a, b, 3) for a, b in STRANDS])
    pA, pB = np.concatenate(pA, 1), np.concatenate(pB, 1)
    S = pA.shape[1]
    return R.LevelGeom("strand", pA, pB, np.full((S, 3), 0.5, F32), width=np.full(S, 2 * RADIUS, F32))


def _thick_geom(a_len, b_len):
    """The strands as thick hairs of one ellipse each (a^ a fixed direction across u)."""
    g = _strand_geom()
    S = g.pA.shape[1]
    u = (g.pB - g.pA).astype(np.float64)
    u /= np.linalg.norm(u, axis=0)
    helper = np.array([0.0, 0.0, 1.0])[:, None]
    ahat = helper - (helper * u).sum(0) * u
    ahat /= np.linalg.norm(ahat, axis=0)
    n = 1 if a_len == b_len else 6
    return R.LevelGeom("cluster", g.pA, g.pB, g.sigma_a, ahat=ahat.astype(F32),
                       a_len=np.full(S, a_len, F32), b_len=np.full(S, b_len, F32),
                       n_total=np.full(S, n, np.int32), r=np.full(S, RADIUS if n == 1 else 0.004, F32),
                       cluster=np.arange(S), seg_in_cluster=np.zeros(S, np.int64))


def _rays(ras, cam):
    """Float64 camera rays through the fragments' pixel centres: origin o [3], unit d [F, 3]."""
    i = (ras.pix % ras.W).astype(np.float64) + 0.5
    j = (ras.pix // ras.W).astype(np.float64) + 0.5
    dv = np.stack([(i - cam.cx) / cam.fx, -(j - cam.cy) / cam.fy, -np.ones_like(i)], 1)
    d = dv @ np.asarray(cam.rot, np.float64)          # R^T dv, rows
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.asarray(cam.pos, np.float64), d


def _trace(geom, ras, cam):
    """Per fragment: closest approach of the ray to the segment's axis (offset b along the true
    y^ and axis parameter), the first hit on the (elliptical) cylinder and its normal."""
    o, d = _rays(ras, cam)
    pA = geom.pA[:, ras.seg].T.astype(np.float64)
    pB = geom.pB[:, ras.seg].T.astype(np.float64)
    L = np.linalg.norm(pB - pA, axis=1)
    u = (pB - pA) / L[:, None]
    w0 = o[None, :] - pA
    b = (d * u).sum(1)
    dd = (d * w0).sum(1)
    e = (u * w0).sum(1)
    den = 1.0 - b * b
    s_ray = (b * e - dd) / den
    tau = (e - b * dd) / den
    n_c = (o[None, :] + s_ray[:, None] * d) - (pA + tau[:, None] * u)
    x_true = -d - (-(d * u).sum(1))[:, None] * u
    x_true /= np.linalg.norm(x_true, axis=1, keepdims=True)
    y_true = np.cross(u, x_true)
    off = (n_c * y_true).sum(1)
    # elliptical cross-section: |q . a^| / |a| and |q . b^| / |b| on the unit circle
    if geom.kind == "cluster":
        ah = geom.ahat[:, ras.seg].T.astype(np.float64)
        bh = np.cross(u, ah)
        al = geom.a_len[ras.seg].astype(np.float64)
        bl = geom.b_len[ras.seg].astype(np.float64)
    else:
        ah = np.cross(u, np.eye(3)[np.argmin(np.abs(u), 1)])
        ah /= np.linalg.norm(ah, axis=1, keepdims=True)
        bh = np.cross(u, ah)
        al = bl = np.full(len(ras.seg), RADIUS)
    # ray in the cross-section coordinates scaled to the unit circle: q(s) = q0 + s qd
    q0 = w0 - (w0 * u).sum(1)[:, None] * u
    qd = d - (d * u).sum(1)[:, None] * u
    q0s = np.stack([(q0 * ah).sum(1) / al, (q0 * bh).sum(1) / bl], 1)
    qds = np.stack([(qd * ah).sum(1) / al, (qd * bh).sum(1) / bl], 1)
    A2 = (qds * qds).sum(1)
    B2 = (q0s * qds).sum(1)
    C2 = (q0s * q0s).sum(1) - 1.0
    disc = B2 * B2 - A2 * C2
    hit = disc > 0
    s_hit = (-B2 - np.sqrt(np.maximum(disc, 0.0))) / A2
    X = o[None, :] + s_hit[:, None] * d
    q = X - pA - ((X - pA) * u).sum(1)[:, None] * u
    # outward normal of the ellipse (gradient of (q.a^/|a|)^2 + (q.b^/|b|)^2)
    nrm = ((q * ah).sum(1) / al ** 2)[:, None] * ah + ((q * bh).sum(1) / bl ** 2)[:, None] * bh
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    W_sup = np.sqrt((al * (ah * y_true).sum(1)) ** 2 + (bl * (bh * y_true).sum(1)) ** 2)
    return dict(o=o, d=d, u=u, L=L, tau=tau, off=off, W=W_sup, hit=hit, X=X, n=nrm, pA=pA, pB=pB)


def _oracle_frame(geom, cam):
    ras = R.rasterize(geom, cam)
    xw, u, wo = R.shading_inputs(geom, ras, cam)
    xh, yh, degen, sin_to = R.frame(u, wo)
    hw = R._t(ras.hw[ras.seg])
    _, h = R.fragment_alpha_h(ras, hw)
    return ras, xw, u, wo, xh, yh, degen, sin_to, hw, h


def _inside(tr, margin=0.02):
    """Fragments whose ray meets the hair inside the segment (not at its ends)."""
    return tr["hit"] & (tr["tau"] > margin * tr["L"]) & (tr["tau"] < (1 - margin) * tr["L"])


GEOMS = {"strand": _strand_geom, "one-hair thick hair": lambda: _thick_geom(RADIUS, RADIUS),
         "elliptical thick hair": lambda: _thick_geom(0.03, 0.012)}


def check_h(geom, cam):
    ras, xw, u, wo, xh, yh, degen, sin_to, hw, h = _oracle_frame(geom, cam)
    tr = _trace(geom, ras, cam)
    h_true = tr["off"] / tr["W"]
    sel = _inside(tr) & (np.abs(h_true) > 0.1) & (np.abs(h_true) < 0.9)
    assert sel.sum() > 300
    h = h.numpy()
    assert np.all(np.sign(h[sel]) == np.sign(h_true[sel]))
    # size: the strip coordinate h (hw + 1/2) is the pixel distance to the centre line; over
    # the hair's projected half-width at the fragment's own depth (hw holds the segment
    # midpoint's) it is the traced offset over the half-width, up to perspective
    z = -((tr["pA"] + tr["tau"][:, None] * tr["u"] - np.asarray(cam.pos, np.float64)) @ np.asarray(cam.rot, np.float64).T)[:, 2]
    hw_local = tr["W"] * cam.fy / z
    scaled = h * (hw.numpy() + 0.5) / hw_local
    assert np.max(np.abs(scaled[sel] - h_true[sel])) < 0.04, np.max(np.abs(scaled[sel] - h_true[sel]))
    return ras, tr, h_true, sel, (xw, u, wo, xh, yh, degen, sin_to, hw, h)


@pytest.mark.parametrize("kind", list(GEOMS))
def test_h_sign_and_size_match_the_traced_offset(kind):
    check_h(GEOMS[kind](), _camera())


def check_phi(geom, cam):
    """The mirror direction of the camera ray at its hit point: phi = Phi(0, h_traced), theta_h = 0."""
    ras, tr, h_true, sel, (xw, u, wo, xh, yh, degen, sin_to, hw, h) = check_h(geom, cam)
    d, nrm = tr["d"], tr["n"]
    r = d - 2.0 * (d * nrm).sum(1)[:, None] * nrm            # toward the light whose R reaches the camera
    wi = torch.as_tensor(r)
    phi = R.azimuth(wi, xh, yh, degen).numpy()
    if geom.kind == "cluster" and not np.allclose(geom.a_len, geom.b_len):
        # an ellipse's normal at the hit is not radial: compare with the mirror about the
        # traced normal's own azimuth, gamma = angle of the normal from x^ toward y^
        g = np.arctan2((nrm * yh.numpy()).sum(1), (nrm * xh.numpy()).sum(1))
        want = -2.0 * g
    else:
        want = exit_azimuth(0, torch.as_tensor(np.arcsin(np.clip(h_true, -1, 1))), torch.zeros(1)).numpy()
    diff = (phi - want + math.pi) % (2 * math.pi) - math.pi
    assert np.max(np.abs(diff[sel])) < 0.03, np.max(np.abs(diff[sel]))
    sin_ti = (wi * u).sum(-1)
    _, _, th, _ = angles(sin_ti, sin_to)
    assert np.max(np.abs(th.numpy()[sel])) < 0.03


@pytest.mark.parametrize("kind", list(GEOMS))
def test_azimuth_of_the_mirror_direction_is_the_r_exit_azimuth(kind):
    check_phi(GEOMS[kind](), _camera())


def check_world_point(geom, cam):
    """The oracle's world point projects onto the pixel centre's foot on the projected segment."""
    ras = R.rasterize(geom, cam)
    xw, _, _ = R.shading_inputs(geom, ras, cam)
    X = xw.numpy()
    Rm = np.asarray(cam.rot, np.float64)
    pos = np.asarray(cam.pos, np.float64)

    def proj(P):
        v = (P - pos) @ Rm.T
        return np.stack([cam.cx + cam.fx * v[:, 0] / -v[:, 2], cam.cy - cam.fy * v[:, 1] / -v[:, 2]], 1)

    pA = geom.pA[:, ras.seg].T.astype(np.float64)
    pB = geom.pB[:, ras.seg].T.astype(np.float64)
    a, b = proj(pA), proj(pB)
    c = np.stack([(ras.pix % ras.W) + 0.5, (ras.pix // ras.W) + 0.5], 1)
    ab = b - a
    foot = a + (((c - a) * ab).sum(1) / (ab * ab).sum(1))[:, None] * ab
    err = np.linalg.norm(proj(X) - foot, axis=1)
    # the oracle's screen parameter comes from endpoints snapped to 1/16 px
    assert err.max() < 0.07, err.max()
    return err


def test_world_point_projects_to_the_pixel_foot():
    check_world_point(_strand_geom(), _camera())


def _radiance(geom, cam, lights):
    ras = R.rasterize(geom, cam)
    mat = (1.55, -0.05236, 0.3, 0.3)
    _, L = R.fragment_radiance(geom, ras, cam, lights, mat)
    return L.numpy()


def check_point_light(geom, cam):
    base = np.array([0.1, 0.3, 0.2], np.float64)
    dirn = np.array([0.4, 0.5, 0.7])
    dirn /= np.linalg.norm(dirn)
    one = hs.Light(1, base.astype(F32), np.full(3, 0.5, F32))
    # twice as far from every fragment is not one position; scale about a single fragment's
    # point instead: the light at x + 2 (p - x) with 4 I seen from x itself
    ras = R.rasterize(geom, cam)
    xw, _, _ = R.shading_inputs(geom, ras, cam)
    k = len(ras.seg) // 2
    x = xw[k].numpy()
    far = hs.Light(1, (x + 2.0 * (base - x)).astype(F32), np.full(3, 2.0, F32))
    mat = (1.55, -0.05236, 0.3, 0.3)
    _, L1 = R.fragment_radiance(geom, ras, cam, [one], mat)
    _, L2 = R.fragment_radiance(geom, ras, cam, [far], mat)
    assert abs(L2[k, 0].item() / L1[k, 0].item() - 1.0) < 1e-5
    # a distant point light approaches the directional light of the same direction
    D = 1.0e4
    dist = hs.Light(1, (D * dirn).astype(F32), np.full(3, D * D, F32))
    dl = hs.Light(0, dirn.astype(F32), np.ones(3, F32))
    Lp = _radiance(geom, cam, [dist])
    Ld = _radiance(geom, cam, [dl])
    rel = np.abs(Lp - Ld) / np.maximum(np.abs(Ld), 1e-12)
    assert np.median(rel) < 2e-4 and rel.max() < 5e-3, (np.median(rel), rel.max())


def test_point_light_falloff_and_direction():
    check_point_light(_strand_geom(), _camera())


# ---- planted mistakes: each pin above fails on a plausible error in the oracle --------------

def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_planted_flipped_h_sign_is_caught(monkeypatch):
    orig = rs.h_sign
    monkeypatch.setattr(rs, "h_sign", lambda *a: -orig(*a))
    assert _fails(check_h, _strand_geom(), _camera())
    assert _fails(check_h, _thick_geom(0.03, 0.012), _camera())


def test_planted_affine_world_parameter_is_caught(monkeypatch):
    monkeypatch.setattr(R, "perspective_t", lambda t, izA, izB: t)
    assert _fails(check_world_point, _strand_geom(), _camera())


def test_planted_mirrored_azimuth_is_caught(monkeypatch):
    orig = R.azimuth
    monkeypatch.setattr(R, "azimuth", lambda wi, xh, yh, degen: -orig(wi, xh, yh, degen))
    assert _fails(check_phi, _strand_geom(), _camera())


def test_planted_y_axis_flip_is_caught(monkeypatch):
    orig = R.frame

    def flipped(u, wo):
        xh, yh, degen, s = orig(u, wo)
        return xh, -yh, degen, s
    monkeypatch.setattr(R, "frame", flipped)
    assert _fails(check_phi, _strand_geom(), _camera())


def test_planted_linear_falloff_is_caught(monkeypatch):
    orig = R.light_dirs

    def linear(light, xw):
        wi, E = orig(light, xw)
        if light.kind == 1:
            d2 = ((R._t(np.asarray(light.vec, F32))[None, :] - xw) ** 2).sum(-1)
            E = E * torch.sqrt(d2)[:, None]
        return wi, E
    monkeypatch.setattr(R, "light_dirs", linear)
    assert _fails(check_point_light, _strand_geom(), _camera())
