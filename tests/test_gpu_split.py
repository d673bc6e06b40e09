"""Long segments on the GPU: a segment longer than 1024 px on a screen axis is drawn as pieces
of equal screen parameter (projection step, Sec. 5.2) instead of being culled.  At 3840x2160,
strands up to ~2700 px long and thick hairs longer than 1024 px and wider than 256 px in
half-width: the piece records are bit-exact against the oracle's split geometry, the fragment
count is the oracle's, the radiance matches it within 1e-4, no segment is culled for its
size, and the backward pass of the wide thick hairs matches the oracle's autograd gradient;
mixed-level frames (plain and shadowed) whose every row is drawn in pieces match the oracle."""
import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import grad as OG
from oracle import lod as OL
from oracle import mixed as M
from oracle import render as R

pytestmark = pytest.mark.gpu

F32 = np.float32
W, H = 3840, 2160
RTOL, ATOL = 1e-4, 1e-7


@pytest.fixture(scope="module")
def ctx(hip):
    c = hip.Context(0)
    yield c
    c.close()


def _camera():
    return hs.Camera(np.zeros(3, F32), np.eye(3, dtype=F32), 1800.0, 1800.0, W / 2.0, H / 2.0, W, H, 0.01)


def _strand_asset(seed=61):
    """Two single-segment strands crossing most of the image obliquely and in depth (drawn as
    3 and 2 pieces) and 200 short ones in front of the camera."""
    rng = np.random.default_rng(seed)
    long_a = np.array([[-0.95, -0.5, -1.0], [0.9, 0.48, -1.6]], F32)
    long_b = np.array([[0.9, -0.45, -1.4], [-0.8, 0.5, -0.9]], F32)
    n_short = 200
    c = rng.uniform([-0.8, -0.45, -1.6], [0.8, 0.45, -0.9], size=(n_short, 3))
    d = rng.normal(size=(n_short, 3))
    d *= rng.uniform(0.002, 0.05, size=(n_short, 1)) / np.linalg.norm(d, axis=1, keepdims=True)
    pts = np.concatenate([long_a[None], long_b[None], np.stack([c, c + d], 1).astype(F32)], 0)   # [n, 2, 3]
    n = pts.shape[0]
    xyz = np.ascontiguousarray(pts.reshape(2 * n, 3).T)
    sig = np.ascontiguousarray(rng.uniform(0.2, 1.5, size=(3, n)).astype(F32))
    width = np.full(n, 3e-3, F32)
    width[2:] = rng.uniform(40e-6, 2e-3, size=n - 2)
    return hs.Asset(n, 1, xyz, width, sig)


def _thick_lod():
    """Two thick hairs of two segments each, every segment longer than 1024 px and over 300 px
    in half-width; the cross-section's long axis a^ is the screen's y direction made normal to
    the segment's tangent."""
    centers = np.array([[[-0.5, -0.1, -0.7], [0.0, 0.0, -0.8], [0.45, 0.12, -0.75]],
                        [[-0.6, 0.35, -0.9], [0.1, -0.05, -0.85], [0.7, -0.35, -0.8]]], F32)
    K, V, _ = centers.shape
    S = V - 1
    t = centers[:, 1:] - centers[:, :-1]
    u = t / np.linalg.norm(t, axis=-1, keepdims=True)
    y = np.array([0.0, 1.0, 0.0])
    a = y - (u @ y)[..., None] * u
    ahat = (a / np.linalg.norm(a, axis=-1, keepdims=True)).astype(F32)
    axes = np.array([[[0.15, 0.06], [0.14, 0.05]], [[0.16, 0.07], [0.15, 0.06]]], F32)
    return dict(centers=centers, ahat=ahat, axes=axes, n_total=np.array([300, 450], np.int32),
                sigma_a=np.array([[0.3, 0.5], [0.6, 0.9], [1.1, 1.6]], F32), r=np.array([4e-5, 5e-5], F32)), K, S


def _lights_for(asset):
    return hs.default_lights(asset, with_point=True)


def _check_rows(ctx, ws, geom, cam, stats, what):
    """Piece records on the GPU against the oracle's split geometry, bit for bit; returns the
    pieces and the widest visible half-width (px)."""
    sp = R.split_long(geom, cam)
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = R.segment_records(sp, cam)
    rows = sp.pA.shape[1]
    assert sp is not geom and rows > geom.pA.shape[1]
    assert stats["segments"] == rows, what
    ri, rf = ctx.debug_segments(ws, rows)
    v = (ri[:, 5] & 1).astype(bool)
    assert np.array_equal(v, vis), what
    for col, ref in enumerate((XA, YA, XB, YB, hw_fx)):
        assert np.array_equal(ri[v, col], ref[vis]), (what, col)
    for col, ref in enumerate((izA, izB, hw)):
        assert np.array_equal(rf[v, col].view(np.uint32), ref[vis].view(np.uint32)), (what, col)
    assert stats["segments_visible"] == int(vis.sum()), what
    return sp, float(hw[vis].max())


def _radiance(got, ref, what, hw_max):
    """Within 1e-4 relative, and an absolute term for coverage at a strip's border: alpha there
    is the difference of a pixel's distance to the axis and the half-width, both of magnitude
    up to 2 hw + 1 px and each a few float32 roundings in the kernel, so a fragment's alpha
    carries up to about 8 ulp(1) (2 hw_max + 1) of absolute error, scaled by the radiance."""
    got = np.asarray(got, np.float64)
    hw_max = np.asarray(hw_max, np.float64)
    if hw_max.ndim == 2:                     # per pixel: the widest fragment there
        hw_max = hw_max[..., None]
    atol = ATOL + 8 * 2.0 ** -24 * (2 * hw_max + 1) * max(1.0, float(np.abs(ref).max()))
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + atol)
    bad = int((err > 0).sum())
    print(f"[{what}] violations {bad} of {ref.size}", flush=True)
    for i in np.argsort(err, axis=None)[::-1][:min(bad, 5)]:
        idx = np.unravel_index(i, ref.shape)
        print(f"  at {idx}: got {got[idx]!r} oracle {ref[idx]!r}", flush=True)
    assert bad == 0, what


def test_long_strands_drawn_as_pieces(hip, ctx):
    print("case: long strands at 3840x2160", flush=True)
    asset = _strand_asset()
    cam = _camera()
    lights = _lights_for(asset)
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    img, stats, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    torch.cuda.synchronize()
    geom = R.strand_level(asset)
    _, hw_max = _check_rows(ctx, ws, geom, cam, stats, "long strands")
    assert stats["segments_culled_long"] == 0
    ref, ras = R.render(geom, cam, lights, tuple(float(v) for v in asset.material.as_array()))
    print(f"long strands: {stats['fragments']} fragments, oracle {len(ras.seg)}", flush=True)
    assert stats["fragments"] == len(ras.seg)
    _radiance(img.cpu().numpy(), ref, "long strands at 3840x2160", hw_max)
    # the same frame again on the warm workspace (capacities of the pieces' pass)
    img2, stats2, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(img.view(torch.int32), img2.view(torch.int32))
    assert stats2["fragments"] == stats["fragments"]
    ws.close()
    ctx.release(aid)


def _rects(img, sp, cam, n=4, size=32):
    """Rectangles at the pieces' joints (screen midpoints of the interior piece ends) and at
    the deepest pixel."""
    c = R.rs.cam_arrays(cam)
    XB, YB = R.rs.project_points(sp.pB, c)[:2]
    out = []
    joints = [r for r in range(sp.pA.shape[1] - 1) if sp.parent[r] == sp.parent[r + 1]]
    for r in joints[:n]:
        x, y = int(XB[r]) // 16, int(YB[r]) // 16
        out.append((min(max(x - size // 2, 0), W - size), min(max(y - size // 2, 0), H - size), size, size))
    alpha = img[..., 3]
    y, x = np.unravel_index(np.argmax(alpha), alpha.shape)
    out.append((int(min(max(x - size // 2, 0), W - size)), int(min(max(y - size // 2, 0), H - size)), size, size))
    return out


def test_long_wide_thick_hairs(hip, ctx):
    print("case: thick hairs longer than 1024 px and wider than 256 px at 3840x2160", flush=True)
    lod, K, S = _thick_lod()
    asset = hs.make_asset(40, S, 90.0, seed=62, sigma_spread=True)
    cam = _camera()
    lights = _lights_for(asset)
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    ws = ctx.workspace()
    img, stats, _ = ctx.render(aid, 1, cam, lights, ws=ws)
    torch.cuda.synchronize()
    geom = R.cluster_level(lod)
    hw = R.segment_records(geom, cam)[7]
    assert (hw > 256.0).all()
    sp, hw_max = _check_rows(ctx, ws, geom, cam, stats, "long wide thick hairs")
    assert stats["segments_culled_long"] == 0
    ras = R.rasterize(sp, cam)
    print(f"long wide thick hairs: {stats['fragments']} fragments, oracle {len(ras.seg)}", flush=True)
    assert stats["fragments"] == len(ras.seg)
    got = img.cpu().numpy()
    mat = tuple(float(v) for v in asset.material.as_array())
    # rectangles at the joints, at the deepest pixel and on the footprints' borders
    alpha = got[..., 3]
    ys, xs = np.nonzero((alpha > 0) & (alpha < 0.5))
    rng = np.random.default_rng(64)
    border = [(int(min(max(xs[i] - 16, 0), W - 32)), int(min(max(ys[i] - 16, 0), H - 32)), 32, 32)
              for i in rng.choice(ys.size, size=3, replace=False)]
    for rect in _rects(got, sp, cam) + border:
        x0, y0, w, h = rect
        ref, _ = R.render(geom, cam, lights, mat, rect=rect)
        _radiance(got[y0:y0 + h, x0:x0 + w], ref[y0:y0 + h, x0:x0 + w], f"thick pieces rect {rect}", hw_max)
    ws.close()
    ctx.release(aid)


def _close(got, ref, what, rel=2e-3, floor=2e-3):
    scale = float(np.abs(ref).max())
    err = np.abs(got - ref)
    bad = int((err > floor * scale + rel * np.abs(ref)).sum())
    print(f"[{what}] max |err| {float(err.max()):.3e} (scale {scale:.3e}), violations {bad}/{ref.size}", flush=True)
    assert bad == 0, what


def test_long_wide_thick_hairs_backward(hip, ctx):
    """The gradient of a loss that weights rectangles across the four joints between pieces:
    every piece's contribution lands on its segment's parameters."""
    print("case: backward of long wide thick hairs at 3840x2160", flush=True)
    lod, K, S = _thick_lod()
    asset = hs.make_asset(40, S, 90.0, seed=62, sigma_spread=True)
    cam = _camera()
    lights = _lights_for(asset)
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    geom = R.cluster_level(lod)
    sp = R.split_long(geom, cam)
    img, _, _ = ctx.render(aid, 1, cam, lights)
    torch.cuda.synchronize()
    rng = np.random.default_rng(63)
    d_rgba = np.zeros((H, W, 4))
    keep = np.zeros((H, W), bool)
    for x0, y0, w, h in _rects(img.cpu().numpy(), sp, cam, n=4, size=48)[:4]:   # the four joints
        d_rgba[y0:y0 + h, x0:x0 + w] = rng.normal(size=(h, w, 4))
        keep[y0:y0 + h, x0:x0 + w] = True
    ras = R.rasterize(sp, cam, pix_filter=lambda i, j: keep[j, i])
    assert len(np.unique(sp.parent[ras.seg])) == 4 and len(np.unique(ras.seg)) == 8
    mat = tuple(float(v) for v in asset.material.as_array())
    g_axes, g_r, g_sig, _ = OG.cluster_vjp(geom, cam, lights, mat, d_rgba, K, S, ras=ras)
    dev = "cuda:0"
    d = torch.tensor(d_rgba, dtype=torch.float32, device=dev).contiguous()
    da = torch.empty((K, S, 2), dtype=torch.float32, device=dev)
    dr = torch.empty(K, dtype=torch.float32, device=dev)
    ds = torch.empty((3, K), dtype=torch.float32, device=dev)
    ctx.render_backward(aid, 1, cam, lights, d, da, dr, ds)
    torch.cuda.synchronize()
    _close(da.cpu().numpy(), g_axes, "d_axes")
    _close(dr.cpu().numpy(), g_r, "d_r")
    _close(ds.cpu().numpy(), g_sig, "d_sigma_a")
    ctx.release(aid)


def _curtain(n=240, seed=81):
    """Straight two-segment strands spanning the image left to right, every segment 1000-1600
    px long at 3840x2160, receding in depth; widths 60 um to 1 mm."""
    rng = np.random.default_rng(seed)
    y = rng.uniform(-0.4, 0.4, n)
    z = rng.uniform(-0.05, 0.05, n)
    v0 = np.stack([rng.uniform(-0.85, -0.75, n), y, -1.0 + z], 1)
    v1 = np.stack([rng.uniform(-0.02, 0.02, n), y + 0.03 * np.sin(7 * y), -1.1 + z], 1)
    v2 = np.stack([rng.uniform(0.75, 0.85, n), y - 0.02, -1.25 + z], 1)
    pts = np.stack([v0, v1, v2], 1).astype(F32)
    xyz = np.ascontiguousarray(pts.reshape(3 * n, 3).T)
    sig = np.ascontiguousarray(rng.uniform(0.2, 1.5, size=(3, n)).astype(F32))
    return hs.Asset(n, 2, xyz, rng.uniform(60e-6, 1e-3, n).astype(F32), sig)


@pytest.fixture(scope="module")
def curtain(hip, ctx):
    asset = _curtain()
    assigns = hs.kmeans_hierarchy(asset, (40, 10, 3), seed=81)
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, assigns)
    lods = [OL.build_level(asset, a) for a in assigns]
    for l, lod in enumerate(lods, 1):
        ctx.set_lod(aid, l, lod)
    geoms = M.level_geoms(asset, lods)
    yield asset, aid, geoms, M.groups(assigns)
    ctx.release(aid)


def _hw_per_pixel(ras):
    out = np.zeros(W * H)
    np.maximum.at(out, ras.pix, ras.hw[ras.seg].astype(np.float64))
    return out.reshape(H, W)


@pytest.mark.parametrize("shadow", [None, (128, 4, 0.02)])
def test_mixed_frame_drawn_as_pieces(hip, ctx, curtain, shadow):
    print(f"case: mixed frame of long rows at 3840x2160, shadow {shadow}", flush=True)
    asset, aid, geoms, grps = curtain
    cam = _camera()
    lights = _lights_for(asset)
    G, S = ctx.lod_groups(aid), asset.segs
    levels = np.random.default_rng(82).integers(0, 4, size=(G, S)).astype(np.int32)
    lev = torch.tensor(levels, device="cuda:0")
    ws = ctx.workspace()
    if shadow is None:
        img, stats, _ = ctx.render_mixed(aid, cam, lights, lev, ws=ws)
    else:
        img, stats, _ = ctx.render_mixed_shadowed(aid, cam, lights, lev, shadow=shadow, ws=ws)
    torch.cuda.synchronize()
    mixed = M.mixed_geometry(geoms, grps, levels)
    assert len(np.unique(levels)) >= 3 and mixed.thick.any() and not mixed.thick.all()
    sp, _ = _check_rows(ctx, ws, mixed, cam, stats, "mixed rows")
    ri, _ = ctx.debug_segments(ws, sp.pA.shape[1])
    assert np.array_equal((ri[:, 5] & 8) != 0, sp.thick)
    assert stats["segments_culled_long"] == 0
    ref, ras = R.render(mixed, cam, lights, tuple(float(v) for v in asset.material.as_array()), shadow=shadow)
    print(f"mixed pieces: {stats['fragments']} fragments, oracle {len(ras.seg)}", flush=True)
    assert stats["fragments"] == len(ras.seg)
    _radiance(img.cpu().numpy(), ref, f"mixed frame in pieces, shadow {shadow}", _hw_per_pixel(ras))
    ws.close()
