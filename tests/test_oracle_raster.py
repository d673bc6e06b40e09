"""Pins for projection, coverage, binning, depth order and compositing (oracle/raster.py,
oracle/render.py): brute force with Python integers, the pinhole model in float64, and
closed forms of front-to-back compositing."""
import math

import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import raster as rs
from oracle import render as R


def _cam(W=64, H=48):
    rot = np.eye(3, dtype=np.float32)
    return hs.Camera(np.array([0.0, 0.0, 1.0], np.float32), rot, 60.0, 60.0, W / 2, H / 2, W, H, 0.01)


def test_projection_matches_pinhole_model():
    rng = np.random.default_rng(0)
    cam = _cam(640, 480)
    c = rs.cam_arrays(cam)
    p = np.stack([rng.uniform(-0.3, 0.3, 500), rng.uniform(-0.3, 0.3, 500), rng.uniform(-0.5, 0.5, 500)]).astype(np.float32)
    X, Y, z, iz, ok = rs.project_points(p, c)
    p64 = p.astype(np.float64)
    zz = 1.0 - p64[2]
    x = cam.cx + cam.fx * p64[0] / zz
    y = cam.cy - cam.fy * p64[1] / zz
    assert ok.all()
    assert np.all(np.abs(X - 16 * x) <= 0.5 + 1e-3)
    assert np.all(np.abs(Y - 16 * y) <= 0.5 + 1e-3)
    assert np.allclose(iz, 1.0 / zz, rtol=1e-6)
    # the optical axis lands on the principal point
    X0, Y0, _, _, _ = rs.project_points(np.array([[0.0], [0.0], [0.2]], np.float32), c)
    assert X0[0] == 16 * cam.cx and Y0[0] == 16 * cam.cy
    # behind the near plane and outside the guard band are culled
    _, _, _, _, ok2 = rs.project_points(np.array([[0.0, 100.0], [0.0, 0.0], [0.995, 0.0]], np.float32), c)
    assert not ok2[0] and not ok2[1]


def _brute_fragments(XA, YA, XB, YB, hw_fx, vis, W, H):
    out = set()
    for s in range(len(XA)):
        if not vis[s]:
            continue
        ax, ay, bx, by = int(XA[s]), int(YA[s]), int(XB[s]), int(YB[s])
        dx, dy = bx - ax, by - ay
        den = dx * dx + dy * dy
        Rr = int(hw_fx[s]) + 8
        for j in range(H):
            for i in range(W):
                ex, ey = 16 * i + 8 - ax, 16 * j + 8 - ay
                num = ex * dx + ey * dy
                cr = ex * dy - ey * dx
                if den > 0 and 0 <= num < den and cr * cr < Rr * Rr * den:
                    out.add((s, j * W + i))
    return out


def _random_segments(rng, n, W, H, crafted=True):
    XA = rng.integers(-40, 16 * W + 40, n)
    YA = rng.integers(-40, 16 * H + 40, n)
    L = rng.integers(0, 16 * 12, n)
    ang = rng.uniform(0, 2 * math.pi, n)
    XB = XA + np.round(L * np.cos(ang)).astype(np.int64)
    YB = YA + np.round(L * np.sin(ang)).astype(np.int64)
    hw_fx = rng.integers(0, 40, n)
    if crafted:
        # endpoints exactly on pixel centres (t_num = 0 and t_num = t_den cases), axis-aligned
        # segments through centres (cross = 0), zero-length segments, and shared vertices
        XA[:6] = [8, 24, 40, 56, 56, 200]
        YA[:6] = [8, 8, 24, 24, 40, 100]
        XB[:6] = [40, 24, 40 + 48, 56, 56, 200]
        YB[:6] = [8, 56, 24 + 48, 24, 88, 100]
        XA[6], YA[6] = XB[0], YB[0]
        XB[6], YB[6] = XB[0] + 32, YB[0]
        hw_fx[:7] = [0, 8, 3, 5, 0, 7, 0]
    return XA, YA, XB, YB, hw_fx, np.ones(n, dtype=bool)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_coverage_equals_python_integer_brute_force(seed):
    rng = np.random.default_rng(seed)
    W, H = 24, 20
    XA, YA, XB, YB, hw_fx, vis = _random_segments(rng, 60, W, H)
    seg, pi, pj = rs.candidate_pixels(XA, YA, XB, YB, hw_fx, vis, W, H)
    ok, *_ = rs.coverage(XA, YA, XB, YB, hw_fx, seg, pi, pj)
    ours = set(zip(seg[ok].tolist(), (pj[ok] * W + pi[ok]).tolist()))
    assert ours == _brute_fragments(XA, YA, XB, YB, hw_fx, vis, W, H)


def test_shared_vertex_counted_once():
    # two collinear segments meeting at a pixel centre: that pixel belongs to the second only
    XA = np.array([8, 40]); YA = np.array([8, 8]); XB = np.array([40, 72]); YB = np.array([8, 8])
    hw = np.array([0, 0]); vis = np.ones(2, bool)
    seg, pi, pj = rs.candidate_pixels(XA, YA, XB, YB, hw, vis, 8, 2)
    ok, *_ = rs.coverage(XA, YA, XB, YB, hw, seg, pi, pj)
    got = sorted(zip(seg[ok].tolist(), pi[ok].tolist(), pj[ok].tolist()))
    assert got == [(0, 0, 0), (0, 1, 0), (1, 2, 0), (1, 3, 0)]


def _brute_tiles(XA, YA, XB, YB, hw_fx, vis, W, H, tile):
    """Tile sets by enumerating every tile's pixel centres (Python integers).

    kept: the box tiles (box = the segment's bounding box widened by R = hw_fx + 8) except
    those whose pixel centres, every one of them (the tile's whole grid, on the image or
    not), lie beyond the same one of the four lines that bound the footprint's region:
    t_num < 0, t_num > t_den, or cross^2 >= R^2 t_den on one side (cross > 0, or cross < 0).
    Thin (R <= 2 px) and zero-length segments keep the whole box.
    real: the tiles holding a pixel centre of the closed real footprint
    0 <= t_num <= t_den, cross^2 <= R^2 t_den."""
    ntx, nty = -(-W // tile), -(-H // tile)
    kept, real = [], set()
    for s in range(len(XA)):
        if not vis[s]:
            continue
        Rr = int(hw_fx[s]) + 8
        xa, ya = int(XA[s]), int(YA[s])
        lox, hix = min(xa, int(XB[s])) - Rr, max(xa, int(XB[s])) + Rr
        loy, hiy = min(ya, int(YB[s])) - Rr, max(ya, int(YB[s])) + Rr
        dx, dy = int(XB[s]) - xa, int(YB[s]) - ya
        tden = dx * dx + dy * dy
        for ty in range(nty):
            for tx in range(ntx):
                x0, x1 = 16 * tile * tx, 16 * tile * (tx + 1) - 1
                y0, y1 = 16 * tile * ty, 16 * tile * (ty + 1) - 1
                if not (lox <= x1 and hix >= x0 and loy <= y1 and hiy >= y0):
                    continue
                beyond = [True, True, True, True]
                for j in range(tile):
                    for i in range(tile):
                        ex = 16 * (tile * tx + i) + 8 - xa
                        ey = 16 * (tile * ty + j) + 8 - ya
                        tn, cr = ex * dx + ey * dy, ex * dy - ey * dx
                        out = cr * cr >= Rr * Rr * tden
                        side = [tn < 0, tn > tden, cr > 0 and out, cr < 0 and out]
                        beyond = [b and c for b, c in zip(beyond, side)]
                        if tden > 0 and 0 <= tn <= tden and cr * cr <= Rr * Rr * tden:
                            real.add((ty * ntx + tx, s))
                if tden == 0 or Rr <= 32 or not any(beyond):
                    kept.append((ty * ntx + tx, s))
    return sorted(kept), real


def _wide_segments(rng, W, H):
    """Random segments, half of them wide (radius 2.5 to 25 px) and longer, so that the
    footprint rule drops tiles of their boxes."""
    XA, YA, XB, YB, hw_fx, vis = _random_segments(rng, 80, W, H)
    ang = rng.uniform(0, 2 * math.pi, 40)
    L = rng.integers(16 * 4, 16 * 40, 40)
    XB[40:] = XA[40:] + np.round(L * np.cos(ang)).astype(np.int64)
    YB[40:] = YA[40:] + np.round(L * np.sin(ang)).astype(np.int64)
    hw_fx[40:] = rng.integers(40, 400, 40)
    return XA, YA, XB, YB, hw_fx, vis


@pytest.mark.parametrize("tile", [8, 16])
def test_binning_equals_brute_force_over_pixel_centres(tile):
    """The tile rule (corner projections) against the enumeration of every tile's pixel
    centres; the kept set holds every tile with a pixel centre in the real footprint, and
    every fragment's tile holds its segment."""
    rng = np.random.default_rng(4)
    W, H = 70, 45
    XA, YA, XB, YB, hw_fx, vis = _wide_segments(rng, W, H)
    vis[3] = False
    tid, seg, _ = rs.bins(XA, YA, XB, YB, hw_fx, vis, W, H, tile)
    kept, real = _brute_tiles(XA, YA, XB, YB, hw_fx, vis, W, H, tile)
    got = list(zip(tid.tolist(), seg.tolist()))
    assert got == kept
    pairs = set(got)
    assert real <= pairs
    wide = [(t, s) for t, s in got if int(hw_fx[s]) + 8 > 32]
    assert len(wide) > 50 and len(real) < len(pairs)     # the rule is exercised and conservative
    # every fragment's tile holds its segment
    ntx = -(-W // tile)
    sg, pi, pj = rs.candidate_pixels(XA, YA, XB, YB, hw_fx, vis, W, H)
    ok, *_ = rs.coverage(XA, YA, XB, YB, hw_fx, sg, pi, pj)
    for s, i, j in zip(sg[ok], pi[ok], pj[ok]):
        assert ((j // tile) * ntx + i // tile, s) in pairs


def test_planted_binning_mistakes_are_caught(monkeypatch):
    """Plausible mistakes in the tile rule (tile origin, the strip test left out, the
    half-pixel offset of pixel centres) differ from the enumeration."""
    rng = np.random.default_rng(4)
    W, H, tile = 70, 45, 16
    XA, YA, XB, YB, hw_fx, vis = _wide_segments(rng, W, H)
    kept, _ = _brute_tiles(XA, YA, XB, YB, hw_fx, vis, W, H, tile)
    orig = rs.tile_meets_footprint
    for plant in (lambda XA, YA, XB, YB, hw_fx, seg, tx, ty, tile:          # tile origin off by one tile
                  orig(XA, YA, XB, YB, hw_fx, seg, tx + 1, ty, tile),
                  lambda XA, YA, XB, YB, hw_fx, seg, tx, ty, tile:          # the slab alone
                  orig(XA, YA, XB, YB, hw_fx * 1000 + 1000, seg, tx, ty, tile),
                  lambda XA, YA, XB, YB, hw_fx, seg, tx, ty, tile:          # the pixel-centre offset dropped
                  orig(XA + 8, YA + 8, XB + 8, YB + 8, hw_fx, seg, tx, ty, tile)):
        monkeypatch.setattr(rs, "tile_meets_footprint", plant)
        tid, seg, _ = rs.bins(XA, YA, XB, YB, hw_fx, vis, W, H, tile)
        assert list(zip(tid.tolist(), seg.tolist())) != kept


def test_depth_key_orders_nearer_first():
    rng = np.random.default_rng(2)
    izA = rng.uniform(0.5, 2.0, 200).astype(np.float32)
    izB = rng.uniform(0.5, 2.0, 200).astype(np.float32)
    t_num = rng.integers(0, 1000, 200)
    t_den = np.full(200, 1000)
    key, t, iz = rs.depth_key(t_num, t_den, izA, izB)
    z64 = 1.0 / (izA.astype(np.float64) + (t_num / 1000.0) * (izB.astype(np.float64) - izA))
    order_key = np.lexsort((np.arange(200), key))
    # nearer (smaller z) first, up to float32 rounding of iz
    zs = z64[order_key]
    assert np.all(np.diff(zs) >= -1e-6 * zs[1:])


def test_fragment_order_is_python_sort_of_key_then_segment():
    asset = hs.make_asset(40, 6, 60.0, seed=9)
    cam = hs.camera_for(asset, 48, 40)
    ras = R.rasterize(R.strand_level(asset), cam)
    recs = sorted(zip(ras.pix.tolist(), ras.key.tolist(), ras.seg.tolist()))
    assert recs == list(zip(ras.pix.tolist(), ras.key.tolist(), ras.seg.tolist()))


def test_box_filter_alpha_is_overlap_length():
    rng = np.random.default_rng(8)
    for _ in range(50):
        d = rng.uniform(0, 2)
        hw = rng.uniform(0, 1.5)
        xs = np.linspace(-0.5, 0.5, 200001)
        brute = np.mean(np.abs(xs - d) <= hw)          # unit pixel box, strip of half-width hw at offset d
        alpha = min(d + hw, 0.5) - max(d - hw, -0.5)
        assert abs(max(0.0, min(1.0, alpha)) - brute) < 1e-4


def _ras_one_pixel(n):
    return R.Raster(*([np.zeros(1)] * 10), seg=np.arange(n), pix=np.zeros(n, dtype=np.int64),
                    key=np.arange(n), t_num=np.zeros(n), t_den=np.ones(n), cross=np.zeros(n), W=1, H=1)


def test_compositing_closed_forms():
    ras = _ras_one_pixel(1)
    out = R.composite(ras, torch.tensor([0.3], dtype=torch.float64), torch.tensor([[1.0, 2.0, 3.0]], dtype=torch.float64))
    assert np.allclose(out.numpy()[0, 0], [0.3, 0.6, 0.9, 0.3])
    ras2 = _ras_one_pixel(2)
    a = torch.tensor([0.3, 0.5], dtype=torch.float64)
    L = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]], dtype=torch.float64)
    out = R.composite(ras2, a, L).numpy()[0, 0]
    # front-to-back over: C = a1 L1 + (1 - a1) a2 L2, alpha = 1 - (1 - a1)(1 - a2)
    assert np.allclose(out, [0.3, 0.7 * 0.5, 0.0, 1 - 0.7 * 0.5])
    swapped = R.composite(ras2, a.flip(0), L.flip(0)).numpy()[0, 0]
    assert not np.allclose(swapped[:3], out[:3])        # the order matters
    assert np.isclose(swapped[3], out[3])               # coverage does not depend on it


def test_binning_drops_the_box_tiles_beyond_a_wide_segments_ends():
    """A short, wide segment (a thick hair's step): its footprint is a 2R-wide band of the
    segment's length, so the box widened by R holds many tiles the footprint never reaches;
    the bins keep every tile a fragment lands in and far fewer than the box."""
    XA, YA, XB, YB = np.array([800]), np.array([800]), np.array([960]), np.array([800])
    hw_fx = np.array([600]); vis = np.ones(1, bool)
    W, H = 128, 128
    tid, seg, _ = rs.bins(XA, YA, XB, YB, hw_fx, vis, W, H, 16)
    tx0, tx1, ty0, ty1 = rs.tile_ranges(XA, YA, XB, YB, hw_fx, vis, W, H, 16)
    box = int((tx1[0] - tx0[0] + 1) * (ty1[0] - ty0[0] + 1))
    assert len(tid) < box
    sg, pi, pj = rs.candidate_pixels(XA, YA, XB, YB, hw_fx, vis, W, H)
    ok, *_ = rs.coverage(XA, YA, XB, YB, hw_fx, sg, pi, pj)
    kept = set(tid.tolist())
    hit = {(j // 16) * (-(-W // 16)) + i // 16 for i, j in zip(pi[ok], pj[ok])}
    assert hit and hit <= kept
