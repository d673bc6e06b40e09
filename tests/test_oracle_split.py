"""Pins of the long-segment pieces (oracle, CPU): a segment longer than 1024 px on a screen
axis is drawn as pieces of equal screen parameter (render.split_long).  The pieces join end
to end exactly, stay within the coverage predicate's extent limit, their endpoints project to
the screen parameters j / m of the whole segment, and each piece's fragments are the whole
segment's strip over the piece's parameter range at the piece's own width (checked with
unbounded Python integers) except within two sub-pixels of the border or two pixels of a
joint; frames without long segments are left as they are, and a thick hair wider than 256 px
and longer than 1024 px is drawn, piece by piece, exactly as the integer predicate says."""
import math

import numpy as np

import hairsynth as hs
from oracle import raster as rs
from oracle import render as R

F32 = np.float32
W, H = 3840, 2160


def _camera():
    return hs.Camera(np.zeros(3, F32), np.eye(3, dtype=F32), 1800.0, 1800.0, W / 2.0, H / 2.0, W, H, 0.01)


def _long_strands():
    # two strands of one segment each, crossing most of the image obliquely and in depth
    pA = np.array([[-0.95, -0.5, -1.0], [0.9, -0.45, -1.4]], F32).T.copy()
    pB = np.array([[0.9, 0.48, -1.6], [-0.8, 0.5, -0.9]], F32).T.copy()
    n = pA.shape[1]
    return R.LevelGeom("strand", pA, pB, np.full((n, 3), 0.5, F32), width=np.full(n, 3e-3, F32))


def _coverage_pixels(XA, YA, XB, YB, hw_fx, s):
    """Pixels of the integer predicate for segment s over its whole bounding box (int64, with
    the products' range checked first)."""
    xa, ya, xb, yb = int(XA[s]), int(YA[s]), int(XB[s]), int(YB[s])
    Rr = int(hw_fx[s]) + 8
    dx, dy = xb - xa, yb - ya
    tden = dx * dx + dy * dy
    i0, i1 = max(0, (min(xa, xb) - Rr) // 16 - 1), min(W - 1, (max(xa, xb) + Rr) // 16 + 1)
    j0, j1 = max(0, (min(ya, yb) - Rr) // 16 - 1), min(H - 1, (max(ya, yb) + Rr) // 16 + 1)
    ext = 16 * max(W, H) + Rr
    assert (ext * (abs(dx) + abs(dy))) ** 2 < 2 ** 62 and Rr * Rr * tden < 2 ** 62
    jj, ii = np.meshgrid(np.arange(j0, j1 + 1, dtype=np.int64), np.arange(i0, i1 + 1, dtype=np.int64), indexing="ij")
    ex, ey = 16 * ii + 8 - xa, 16 * jj + 8 - ya
    tn, cr = ex * dx + ey * dy, ex * dy - ey * dx
    m = (tden > 0) & (tn >= 0) & (tn < tden) & (cr * cr < Rr * Rr * tden)
    return set((jj[m] * W + ii[m]).tolist())


def test_pieces_join_and_project_to_equal_screen_parameters():
    g = _long_strands()
    cam = _camera()
    c = rs.cam_arrays(cam)
    XA, YA, _, izA, okA = rs.project_points(g.pA, c)
    XB, YB, _, izB, okB = rs.project_points(g.pB, c)
    ext = np.maximum(np.abs(XB - XA), np.abs(YB - YA))
    assert okA.all() and okB.all() and (ext > rs.MAX_AXIS).all()
    sp = R.split_long(g, cam)
    m = np.bincount(sp.parent)
    assert np.array_equal(m, (ext + rs.SPLIT_LEN - 1) // rs.SPLIT_LEN)
    pXA, pYA, _, _, _ = rs.project_points(sp.pA, c)
    pXB, pYB, _, _, _ = rs.project_points(sp.pB, c)
    assert (np.maximum(np.abs(pXB - pXA), np.abs(pYB - pYA)) <= rs.MAX_AXIS).all()
    o = 0
    for s, ms in enumerate(m):
        rows = np.arange(o, o + ms)
        o += ms
        assert np.array_equal(sp.pA[:, rows[0]], g.pA[:, s]) and np.array_equal(sp.pB[:, rows[-1]], g.pB[:, s])
        assert np.array_equal(sp.pB[:, rows[:-1]], sp.pA[:, rows[1:]])       # joints shared exactly
        # each joint projects to screen parameter j / m of the whole segment (float64 pinhole)
        P = np.asarray(g.pA[:, s], np.float64), np.asarray(g.pB[:, s], np.float64)
        proj = lambda p: np.array([cam.cx + cam.fx * p[0] / -p[2], cam.cy - cam.fy * p[1] / -p[2]])
        a, b = proj(P[0]), proj(P[1])
        for j in range(1, ms):
            q = proj(sp.pA[:, rows[j]].astype(np.float64))
            want = a + (j / ms) * (b - a)
            assert np.linalg.norm(q - want) < 1e-3, (s, j, q, want)


def test_pieces_cover_what_the_whole_segment_covers():
    """Piece j of m draws the whole segment's strip over screen parameters [j/m, (j+1)/m), at
    its own half-width (taken at the piece's mid depth): checked pixel by pixel with unbounded
    Python integers on the whole segment's snapped line.  The pieces' snapped endpoints lie on
    that line up to rounding, so a pixel may differ only where its centre lies within two
    sub-pixels of the strip's border or within two pixels of a joint."""
    g = _long_strands()
    cam = _camera()
    sp = R.split_long(g, cam)
    c, XA, YA, XB, YB, _, _, _, hw_fx, vis = R.segment_records(g, cam)
    assert not vis.any()                                  # too long for one predicate
    _, pXA, pYA, pXB, pYB, _, _, _, phw_fx, pvis = R.segment_records(sp, cam)
    assert pvis.all()
    ras = R.rasterize(sp, cam)
    m = np.bincount(sp.parent)
    first = np.cumsum(m) - m
    total, bad = 0, []
    for r in range(sp.pA.shape[1]):
        s_ = int(sp.parent[r])
        j, ms = r - int(first[s_]), int(m[s_])
        xa, ya = int(XA[s_]), int(YA[s_])
        dx, dy = int(XB[s_]) - xa, int(YB[s_]) - ya
        tden = dx * dx + dy * dy
        Rr = int(phw_fx[r]) + 8
        got = set(ras.pix[ras.seg == r].tolist())
        # pixels near the piece's part of the line
        lo = min(int(pXA[r]), int(pXB[r])) - Rr - 32, max(int(pXA[r]), int(pXB[r])) + Rr + 32
        lo_y = min(int(pYA[r]), int(pYB[r])) - Rr - 32, max(int(pYA[r]), int(pYB[r])) + Rr + 32
        want = set()
        near = []
        for jy in range(max(0, lo_y[0] // 16), min(H - 1, lo_y[1] // 16) + 1):
            for ix in range(max(0, lo[0] // 16), min(W - 1, lo[1] // 16) + 1):
                ex, ey = 16 * ix + 8 - xa, 16 * jy + 8 - ya
                tn, cr = ex * dx + ey * dy, ex * dy - ey * dx
                if j * tden <= ms * tn < (j + 1) * tden and cr * cr < Rr * Rr * tden:
                    want.add(jy * W + ix)
        total += len(want)
        for p in want ^ got:
            x, y = p % W, p // W
            ex, ey = 16 * x + 8 - xa, 16 * y + 8 - ya
            dist = abs(ex * dy - ey * dx) / math.sqrt(tden)
            t = (ex * dx + ey * dy) / tden
            joint = min(abs(t - j / ms), abs(t - (j + 1) / ms)) * math.sqrt(tden) / 16.0
            if not (abs(dist - Rr) < 2.0 or joint < 2.0):
                bad.append((r, x, y, dist, Rr, joint))
    assert total > 2000
    assert not bad, bad[:5]


def test_frames_without_long_segments_are_unchanged():
    asset, cam, _ = hs.config(1, scale=0.2)
    geom = R.strand_level(asset)
    assert R.split_long(geom, cam) is geom


def test_thick_hairs_up_to_2048_px_wide_are_drawn():
    cam = _camera()
    pA = np.array([[-0.2, 0.0, -0.5]], F32).T.copy()
    pB = np.array([[0.2, 0.05, -0.6]], F32).T.copy()
    geom = R.LevelGeom("cluster", pA, pB, np.full((1, 3), 0.5, F32), ahat=np.array([[0.0], [1.0], [0.0]], F32),
                       a_len=np.array([0.09], F32), b_len=np.array([0.05], F32), n_total=np.array([40], np.int32),
                       r=np.array([4e-5], F32), cluster=np.zeros(1, np.int64), seg_in_cluster=np.zeros(1, np.int64))
    _, _, _, _, _, _, _, hw, hw_fx, vis = R.segment_records(geom, cam)
    assert hw[0] > 256.0 and not vis[0]                     # wider than 1024 px on screen
    sp = R.split_long(geom, cam)
    _, XA, YA, XB, YB, _, _, phw, phw_fx, pvis = R.segment_records(sp, cam)
    assert sp.pA.shape[1] >= 2 and pvis.all() and (phw > 256.0).all() and (phw_fx <= rs.MAX_HW_FX).all()
    ras = R.rasterize(sp, cam)
    for r in range(sp.pA.shape[1]):
        assert set(ras.pix[ras.seg == r].tolist()) == _coverage_pixels(XA, YA, XB, YB, phw_fx, r)
    assert len(ras.seg) > 500000
