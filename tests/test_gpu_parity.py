"""GPU parity of the HIP path against the CPU oracle, through the C-ABI.

Bar: projected segments, tile bins and per-pixel fragment order bit-exact; radiance within
1e-4 relative per pixel (float32 kernel vs float64 oracle; absolute floor 1e-7 for
near-black values).
"""
import math
import os

import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import lod as OL
from oracle import render as R

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-4, 1e-7


def mat_of(asset):
    return tuple(float(v) for v in asset.material.as_array())


def assert_radiance(got, ref, mask=None, what=""):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    if mask is not None:
        err = err[mask]
    bad = int((err > 0).sum())
    worst = float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-7)).max()) if got.size else 0.0
    print(f"[{what}] max rel err {worst:.3e}, violations {bad}", flush=True)
    assert bad == 0, f"{what}: {bad} values beyond 1e-4 rel"


@pytest.fixture(scope="module")
def ctx(hip):
    c = hip.Context(0)
    yield c
    c.close()


def _render(hip, ctx, asset, cam, lights, level=0, aid=None, lod=None):
    if aid is None:
        aid = ctx.upload_asset(asset)
    if lod is not None:
        ctx.set_lod(aid, 1, lod)
    ws = ctx.workspace()
    img, stats, rc = ctx.render(aid, level, cam, lights, ws=ws)
    torch.cuda.synchronize()
    return aid, ws, img.cpu().numpy(), stats


def test_segments_bins_bit_exact_config1(hip, ctx):
    print("case: 1k strands at 256x256, segments/bins", flush=True)
    asset, cam, lights = hs.config(1)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights)
    geom = R.strand_level(asset)
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = R.segment_records(geom, cam)
    ri, rf = ctx.debug_segments(ws, asset.n_segments)
    v = (ri[:, 5] & 1).astype(bool)
    assert np.array_equal(v, vis)
    for col, ref in enumerate((XA, YA, XB, YB, hw_fx)):
        assert np.array_equal(ri[v, col], ref[vis]), col
    assert np.array_equal(rf[:, 0].view(np.uint32), izA.view(np.uint32))
    assert np.array_equal(rf[:, 1].view(np.uint32), izB.view(np.uint32))
    assert np.array_equal(rf[:, 2].view(np.uint32), hw.view(np.uint32))
    sign = R.rs.h_sign(geom.pA, geom.pB, c, XA, YA, XB, YB)
    assert np.array_equal(((ri[v, 5] & 2) != 0), sign[vis] < 0)
    # bins: same tile sets (list order inside a tile is free)
    ntx, nty = -(-cam.width // 16), -(-cam.height // 16)
    tid, sid, _ = R.rs.bins(XA, YA, XB, YB, hw_fx, vis, cam.width, cam.height, 16)
    assert stats["pairs"] == len(tid)
    ts, segs = ctx.debug_bins(ws, ntx * nty, int(stats["pairs"]))
    ref_start = np.searchsorted(tid, np.arange(ntx * nty + 1))
    assert np.array_equal(ts.astype(np.int64), ref_start)
    for t in range(ntx * nty):
        assert np.array_equal(np.sort(segs[ts[t]:ts[t + 1]]), sid[ref_start[t]:ref_start[t + 1]]), t
    ws.close()


def test_radiance_and_count_config1(hip, ctx):
    print("case: 1k strands at 256x256, radiance", flush=True)
    asset, cam, lights = hs.config(1)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights)
    ref, ras = R.render(R.strand_level(asset), cam, lights, mat_of(asset))
    assert stats["fragments"] == len(ras.seg)
    assert stats["overflow_pixels"] == 0
    assert_radiance(img, ref, what="1k strands at 256x256")
    ws.close()


def _oracle_lists(ras, x0, y0, w, h, W):
    px = ras.pix % W
    py = ras.pix // W
    sel = (px >= x0) & (px < x0 + w) & (py >= y0) & (py < y0 + h)
    local = (py[sel] - y0) * w + (px[sel] - x0)
    order = np.lexsort((ras.seg[sel], ras.key[sel], local))
    counts = np.bincount(local, minlength=w * h)
    return counts.reshape(h, w), ras.key[sel][order], ras.seg[sel][order], np.nonzero(sel)[0][order]


def test_fragment_order_bit_exact(hip, ctx):
    print("case: fragment lists, 1k strands at 256x256, rect", flush=True)
    asset, cam, lights = hs.config(1)
    aid = ctx.upload_asset(asset)
    geom = R.strand_level(asset)
    ras = R.rasterize(geom, cam)
    cnt = np.bincount(ras.pix, minlength=cam.width * cam.height).reshape(cam.height, cam.width)
    j, i = np.unravel_index(np.argmax(cnt), cnt.shape)
    x0, y0 = max(0, i - 20), max(0, j - 20)
    w, h = min(40, cam.width - x0), min(40, cam.height - y0)
    counts, keys, segs, alpha, hoff = ctx.debug_fragments(aid, 0, cam, lights, x0, y0, w, h, cap=400000)
    rc, rk, rsg, idx = _oracle_lists(ras, x0, y0, w, h, cam.width)
    assert np.array_equal(counts, rc)
    assert np.array_equal(keys, rk)
    assert np.array_equal(segs, rsg)
    a_ref, h_ref = R.fragment_alpha_h(ras, R._t(ras.hw[ras.seg]))
    assert np.allclose(alpha, a_ref.numpy()[idx], rtol=1e-5, atol=1e-7)
    assert np.allclose(hoff, h_ref.numpy()[idx], rtol=1e-5, atol=2e-6)
    assert counts.max() > 10


def test_strand_alpha_at_float_rounding(hip, ctx):
    """Every fragment of the config-1 frame: the strand coverage alpha (the 1-D box overlap of
    the pixel with the strand's width at the pixel centre's distance from the centre line)
    within two float32 roundings of the oracle's float64 value, relative, also at edge pixels
    of low coverage, where alpha is a small difference of numbers near 1/2."""
    print("case: strand alpha precision, 1k strands at 256x256, whole frame", flush=True)
    asset, cam, lights = hs.config(1)
    aid = ctx.upload_asset(asset)
    ras = R.rasterize(R.strand_level(asset), cam)
    W, H = cam.width, cam.height
    counts, keys, segs, alpha, hoff = ctx.debug_fragments(aid, 0, cam, lights, 0, 0, W, H, cap=len(ras.seg) + 16)
    rc, rk, rsg, idx = _oracle_lists(ras, 0, 0, W, H, W)
    assert np.array_equal(counts, rc) and np.array_equal(keys, rk) and np.array_equal(segs, rsg)
    hw = ras.hw[ras.seg].astype(np.float64)[idx]
    a_ref = R.fragment_alpha_h(ras, R._t(ras.hw[ras.seg]))[0].numpy()[idx]
    delta = (np.abs(ras.cross.astype(np.float64)) / np.sqrt(ras.t_den.astype(np.float64)) / 16.0)[idx]
    err = np.abs(alpha.astype(np.float64) - a_ref)
    rel = err / np.maximum(a_ref, 1e-30)
    edge = (delta + hw > 0.5) & (a_ref > 0)   # alpha = 1/2 - (delta - hw): the cancelling form
    print(f"alpha: {len(a_ref)} fragments, {int(edge.sum())} at the strands' edges, max rel err "
          f"{float(rel[a_ref > 0].max()):.3e} (edges {float(rel[edge].max()):.3e})", flush=True)
    assert int(edge.sum()) > 1000
    assert np.all(err <= 2.0 ** -23 * a_ref + 1e-30)


@pytest.mark.parametrize("W,H", [(17, 9), (1, 1), (33, 47)])
def test_ragged_and_tiny_images(hip, ctx, W, H):
    print(f"case: ragged {W}x{H}", flush=True)
    asset = hs.make_asset(300, 8, 60.0, seed=5)
    cam = hs.camera_for(asset, W, H)
    lights = hs.default_lights(asset, with_point=True)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights)
    ref, ras = R.render(R.strand_level(asset), cam, lights, mat_of(asset))
    assert stats["fragments"] == len(ras.seg)
    assert_radiance(img, ref, what=f"{W}x{H}")
    ws.close()


def test_empty_frame_and_culling(hip, ctx):
    print("case: empty frame", flush=True)
    asset = hs.make_asset(50, 6, 60.0, seed=2)
    cam = hs.camera_for(asset, 64, 48)
    # turn the camera around: everything is behind it
    cam.rot = (np.diag([-1.0, 1.0, -1.0]) @ cam.rot.astype(np.float64)).astype(np.float32)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, hs.default_lights(asset, False))
    assert stats["fragments"] == 0 and stats["segments_visible"] == 0
    assert np.all(img == 0.0)
    ws.close()


def test_single_strand_and_point_light(hip, ctx):
    print("case: single strand", flush=True)
    asset = hs.make_asset(1, 40, 60.0, seed=8)
    cam = hs.camera_for(asset, 96, 96)
    lights = hs.default_lights(asset, with_point=True)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights)
    ref, ras = R.render(R.strand_level(asset), cam, lights, mat_of(asset))
    assert stats["fragments"] == len(ras.seg) > 0
    assert_radiance(img, ref, what="single strand")
    ws.close()


def test_determinism_bitwise(hip, ctx):
    print("case: determinism", flush=True)
    asset, cam, lights = hs.config(2, scale=0.05)
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    a, s1, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    a = a.clone()
    b, s2, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    torch.cuda.synchronize()
    assert s1["fragments"] == s2["fragments"]
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    ws.close()


# ---- thick-hair levels ---------------------------------------------------------------------

def _cluster_case(n=2000, segs=12, k=40, W=160, H=128, seed=21):
    asset = hs.make_asset(n, segs, 90.0, seed=seed, sigma_spread=True)
    cam = hs.camera_for(asset, W, H)
    lights = hs.default_lights(asset, with_point=True)
    assign = hs.kmeans_assign(asset, k, seed=seed)
    return asset, cam, lights, assign


def test_build_lod_matches_oracle(hip, ctx):
    print("case: build_lod", flush=True)
    asset, cam, lights, assign = _cluster_case()
    assign2 = hs.kmeans_assign(asset, 7, seed=3)
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, [assign, assign2])
    nl, counts, S = ctx.lod_info(aid)
    assert nl == 2 and counts[1] == assign.max() + 1 and counts[2] == assign2.max() + 1 and S == asset.segs
    for lvl, asg in ((1, assign), (2, assign2)):
        got = ctx.get_lod(aid, lvl)
        ref = OL.build_level(asset, asg)
        assert np.array_equal(got.centers, ref["centers"])                # same float64 order
        assert np.array_equal(got.n_total, ref["n_total"])
        assert np.array_equal(got.r, ref["r"])
        assert np.array_equal(got.sigma_a, ref["sigma_a"])
        assert np.allclose(got.axes, ref["axes"], rtol=2e-6, atol=0)
        dots = np.abs((got.ahat.astype(np.float64) * ref["ahat"]).sum(-1))
        elong = ref["axes"][..., 0] > ref["axes"][..., 1] * (1 + 1e-3)
        assert np.all(dots[elong] > 1 - 1e-5)


def test_cluster_level_radiance(hip, ctx):
    print("case: cluster level radiance", flush=True)
    asset, cam, lights, assign = _cluster_case()
    lod = OL.build_level(asset, assign)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights, level=1, lod=lod)
    geom = R.cluster_level(lod)
    ref, ras = R.render(geom, cam, lights, mat_of(asset))
    assert stats["fragments"] == len(ras.seg)
    assert_radiance(img, ref, what="cluster level")
    ws.close()


def test_one_strand_clusters_match_strands_on_gpu(hip, ctx):
    print("case: one-strand clusters", flush=True)
    asset, cam, lights = hs.config(1, scale=0.2)
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, [np.arange(asset.n_strands, dtype=np.int32)])
    ws = ctx.workspace()
    a, sa, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    a = a.cpu().numpy()
    b, sb, _ = ctx.render(aid, 1, cam, lights, ws=ws)
    b = b.cpu().numpy()
    assert sa["fragments"] == sb["fragments"]
    assert_radiance(b, a.astype(np.float64), what="one-strand LoD (GPU strands vs GPU clusters)")
    ws.close()


def test_select_level_matches_oracle(hip, ctx):
    print("case: select level", flush=True)
    asset, cam, lights, assign = _cluster_case(k=200)
    assigns = [assign, hs.kmeans_assign(asset, 30, seed=1), hs.kmeans_assign(asset, 4, seed=1)]
    aid = ctx.upload_asset(asset)
    lods = [OL.build_level(asset, a) for a in assigns]
    for l, lod in enumerate(lods, 1):
        ctx.set_lod(aid, l, lod)
    geoms = [R.strand_level(asset)] + [R.cluster_level(lod) for lod in lods]
    for eps in (0.5, 2.0, 6.0, 1e6):
        assert ctx.select_level(aid, cam, eps) == R.select_level(geoms, cam, eps), eps


# ---- full-size configuration (the benchmark's launch) ----------------------------------------

def golden(name):
    """Stored oracle values of a full-size frame (written by tests/golden/make_golden.py)."""
    import json
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}.json")) as f:
        return json.load(f)


def check_census(hip, ctx, aid, level, cam, lights, stats, gold, what):
    """The frame's fragment count, the counts of its densest, a middle and a sparse row and of
    its deepest pixels, against the oracle's stored census."""
    assert stats["fragments"] == gold["fragments"], (what, stats["fragments"], gold["fragments"])
    rows = np.asarray(gold["rows"])
    nz = np.nonzero(rows)[0]
    for y in (int(np.argmax(rows)), int(nz[len(nz) // 2]), int(nz[len(nz) // 20])):
        cnt, *_ = ctx.debug_fragments(aid, level, cam, lights, 0, y, cam.width, 1, int(rows[y]) + 64)
        assert int(cnt.sum()) == int(rows[y]), (what, y)
    for d in gold["deepest"][:2]:
        cnt, *_ = ctx.debug_fragments(aid, level, cam, lights, d["x"], d["y"], 1, 1, max(d["count"], 1536))
        assert int(cnt[0, 0]) == d["count"], (what, d)
    print(f"[{what}] {gold['fragments']} fragments; rows and deepest pixels ({gold['deepest'][0]['count']}) "
          "equal the oracle's census", flush=True)


def test_config2_full_size_sampled(hip, ctx):
    """100k strands x 32 segments at 1920x1080 (the benchmark's launch): the fragment count,
    row counts and deepest-pixel counts against the oracle's stored census, the frame against
    the oracle on pixel rectangles (densest pixel, dense, medium, sparse), and determinism."""
    print("case: 100k strands at 1920x1080", flush=True)
    asset, cam, lights = hs.config(2)
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    img, stats, rc = ctx.render(aid, 0, cam, lights, ws=ws)
    img2, stats2, _ = ctx.render(aid, 0, cam, lights, ws=ws.__class__(ctx))
    torch.cuda.synchronize()
    assert torch.equal(img.view(torch.int32), img2.view(torch.int32))
    got = img.cpu().numpy()
    print(f"100k strands at 1080p: {stats['fragments']} fragments, {stats['ms_total']:.3f} ms", flush=True)
    gold = golden("strands_100k_1080p")
    check_census(hip, ctx, aid, 0, cam, lights, stats, gold, "100k strands 1080p")
    alpha = got[..., 3]
    ys, xs = np.nonzero(alpha > 0)
    order = np.argsort(alpha[ys, xs])
    picks = [(gold["deepest"][0]["x"], gold["deepest"][0]["y"])]
    picks += [(int(xs[k]), int(ys[k])) for k in (order[-1], order[len(order) // 2], order[len(order) // 20])]
    geom = R.strand_level(asset)
    mat = mat_of(asset)
    for x, y in picks:
        x0 = int(min(max(x - 8, 0), cam.width - 24))
        y0 = int(min(max(y - 8, 0), cam.height - 24))
        ref, ras = R.render(geom, cam, lights, mat, rect=(x0, y0, 24, 24))
        assert_radiance(got[y0:y0 + 24, x0:x0 + 24], ref[y0:y0 + 24, x0:x0 + 24], what=f"100k-strand 1080p rect {x0},{y0}")
    ws.close()


def test_wide_thick_hairs_full_size_sampled(hip, ctx):
    """Thick hairs tens of pixels wide at 1920x1080 (20k strands x 16 segments in 60
    clusters): tile binning keeps only the tiles a wide segment's footprint can reach, and the
    oracle enumerates pixels without any binning, so rectangles on the footprints' borders and
    at the deepest pixel show a tile dropped by mistake as missing coverage."""
    print("case: wide thick hairs at 1920x1080", flush=True)
    asset, cam, lights, assign = _cluster_case(n=20000, segs=16, k=60, W=1920, H=1080, seed=33)
    lod = OL.build_level(asset, assign)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights, level=1, lod=lod)
    alpha = img[..., 3]
    inside = alpha > 0
    edge = inside & ~(np.roll(inside, 1, 0) & np.roll(inside, -1, 0) & np.roll(inside, 1, 1) & np.roll(inside, -1, 1))
    ys, xs = np.nonzero(edge)
    assert ys.size > 0
    rng = np.random.default_rng(33)
    picks = [(int(ys[i]), int(xs[i])) for i in rng.choice(ys.size, size=3, replace=False)]
    picks.append(tuple(int(v) for v in np.unravel_index(np.argmax(alpha * (alpha < 1.0)), alpha.shape)))
    geom = R.cluster_level(lod)
    mat = mat_of(asset)
    print(f"wide thick hairs: {stats['fragments']} fragments", flush=True)
    for y, x in picks:
        x0 = int(min(max(x - 12, 0), cam.width - 24))
        y0 = int(min(max(y - 12, 0), cam.height - 24))
        ref, ras = R.render(geom, cam, lights, mat, rect=(x0, y0, 24, 24))
        assert_radiance(img[y0:y0 + 24, x0:x0 + 24], ref[y0:y0 + 24, x0:x0 + 24],
                        what=f"wide thick hairs 1080p rect {x0},{y0}")
    ws.close()
    ctx.release(aid)

def test_pixels_deeper_than_one_batch(hip, ctx):
    """A dense asset seen small: pixels hold more fragments than one LDS batch (1536) and are
    rendered in exact depth-key slices; radiance and count still match the oracle."""
    print("case: deep pixels", flush=True)
    asset = hs.make_asset(12000, 16, 60.0, seed=31)
    cam = hs.camera_for(asset, 40, 40, fill=0.5)
    lights = hs.default_lights(asset, with_point=True)
    ref, ras = R.render(R.strand_level(asset), cam, lights, mat_of(asset))
    depth = np.bincount(ras.pix, minlength=cam.width * cam.height)
    cap = hip.HAIR_PIXEL_CAPACITY
    assert depth.max() > cap, depth.max()           # at least two key slices
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights)
    assert stats["fragments"] == len(ras.seg)
    assert stats["deep_pixels"] == int((depth > cap).sum()) and stats["overflow_pixels"] == 0
    assert_radiance(img, ref, what="deep pixels")
    ws.close()


@pytest.mark.parametrize("W,H", [(3840, 2160), (4112, 2320), (4200, 4100)])
def test_large_images_binning(hip, ctx, W, H):
    """Tile binning at 4K (per-block tile counters above 64 KiB of LDS), on an image with more
    tiles than one binning pass holds (37,265 > 36,864: two passes), and on one with more than
    2^16 tiles (67,591: the multi-block scans and the separate capacity checks instead of the
    single-block ones).  The hair is framed low so that it crosses the pass boundary; bins,
    fragment count and a rectangle of radiance across the boundary match the oracle, and a
    second (warm) frame on the same workspace equals the first bit for bit."""
    import dataclasses
    print(f"case: large image {W}x{H}", flush=True)
    asset = hs.make_asset(3000, 16, 90.0, seed=41)
    cam = hs.camera_for(asset, W, H)
    cam = dataclasses.replace(cam, cy=cam.cy + 0.35 * H)
    lights = hs.default_lights(asset, with_point=True)
    geom = R.strand_level(asset)
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = R.segment_records(geom, cam)
    tid, sid, _ = R.rs.bins(XA, YA, XB, YB, hw_fx, vis, W, H, 16)
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights)
    T = -(-W // 16) * -(-H // 16)
    assert stats["pairs"] == len(tid)
    ts, segs = ctx.debug_bins(ws, T, int(stats["pairs"]))
    ref_start = np.searchsorted(tid, np.arange(T + 1))
    assert np.array_equal(ts.astype(np.int64), ref_start)
    got_sorted = np.concatenate([np.sort(segs[ts[t]:ts[t + 1]]) for t in range(T)]) if len(tid) else segs
    assert np.array_equal(got_sorted, sid)
    assert stats["fragments"] == len(R.rasterize(geom, cam).seg)
    x0, y0 = 1800, 2270 if H > 2300 else 1800
    y0 = min(y0, H - 24)
    ref, ras = R.render(geom, cam, lights, mat_of(asset), rect=(x0, y0, 24, 24))
    assert_radiance(img[y0:y0 + 24, x0:x0 + 24], ref[y0:y0 + 24, x0:x0 + 24], what=f"{W}x{H} rect")
    img2, st2, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    torch.cuda.synchronize()
    assert st2["fragments"] == stats["fragments"]
    assert np.array_equal(img2.cpu().numpy().view(np.uint32), np.asarray(img, dtype=np.float32).view(np.uint32))
    ws.close()


def _layered_asset(depths, width_px=40, half_extent=0.2):
    """One horizontal single-segment strand per depth, all crossing pixel row 20 of a 40 x 40
    camera at the origin looking down -z (fy = fx = 74.6): every covered pixel holds one
    fragment per strand, with the depth key of that strand's 1 / z."""
    fy = float(np.float32(74.6))
    d = np.asarray(depths, dtype=np.float64)
    n = len(d)
    y = -0.5 * d / fy                                   # pixel row centre 20.5
    xyz = np.empty((3, 2 * n), dtype=np.float32)
    xyz[0, 0::2], xyz[0, 1::2] = -half_extent * d, half_extent * d
    xyz[1, 0::2] = xyz[1, 1::2] = y
    xyz[2, 0::2] = xyz[2, 1::2] = -d
    sig = np.repeat(np.array([0.3, 0.6, 1.2], dtype=np.float32)[:, None], n, axis=1)
    asset = hs.Asset(n, 1, xyz, np.full(n, 80e-6, dtype=np.float32), np.ascontiguousarray(sig))
    cam = hs.Camera(np.zeros(3, np.float32), np.eye(3, dtype=np.float32), fy, fy, 20.0, 20.0, width_px, 40, 0.01)
    return asset, cam


def _key_runs(ras, n_pix):
    """Per pixel: fragment count, and the largest number of fragments sharing one depth key."""
    depth = np.bincount(ras.pix, minlength=n_pix)
    same = np.zeros(n_pix, dtype=np.int64)
    if len(ras.pix):
        run_start = np.r_[True, (np.diff(ras.pix) != 0) | (np.diff(ras.key.astype(np.int64)) != 0)]
        ids = np.cumsum(run_start) - 1
        run_len = np.bincount(ids)
        np.maximum.at(same, ras.pix[run_start], run_len)
    return depth, same


def test_deep_pixels_with_clustered_keys(hip, ctx):
    """Pixels of about 5,000 fragments whose keys crowd into a tiny part of their key range:
    the first histogram over the pixel's range puts more than one batch into one bin, so the
    slicing refines inside it; several slices chain front to back.  Count and radiance match
    the oracle."""
    print("case: deep pixels, clustered keys", flush=True)
    cap = hip.HAIR_PIXEL_CAPACITY
    cluster = 1.0 + 3e-7 * np.arange(5000)
    depths = np.concatenate([np.linspace(0.5, 0.9, 17), cluster, np.linspace(3.0, 10.0, 41)])
    asset, cam = _layered_asset(depths)
    lights = hs.default_lights(asset, with_point=False)
    ref, ras = R.render(R.strand_level(asset), cam, lights, mat_of(asset))
    depth, same = _key_runs(ras, cam.width * cam.height)
    deep = np.nonzero(depth > cap)[0]
    assert len(deep) >= 20 and depth.max() >= 3 * cap and same.max() <= cap
    # the refinement is exercised: some bin of the first histogram holds more than a batch
    st = np.r_[0, np.cumsum(depth)]
    p = deep[0]
    k = ras.key[st[p]:st[p + 1]].astype(np.int64)
    width = -(-(int(k.max()) - int(k.min()) + 1) // cap)
    assert np.bincount((k - k.min()) // width).max() > cap
    aid, ws, img, stats = _render(hip, ctx, asset, cam, lights)
    assert stats["fragments"] == len(ras.seg)
    assert stats["deep_pixels"] == len(deep) and stats["overflow_pixels"] == 0
    assert_radiance(img, ref, what="deep clustered")
    # the whole order of the deep row, slice after slice, is the oracle's
    counts, keys, segs, alpha, hoff = ctx.debug_fragments(aid, 0, cam, lights, 0, 20, 40, 1, cap=40 * 5200)
    rc, rk, rsg, idx = _oracle_lists(ras, 0, 20, 40, 1, cam.width)
    assert np.array_equal(counts, rc) and counts.max() == depth.max()
    assert np.array_equal(keys, rk)
    assert np.array_equal(segs, rsg)
    ws.close()


def test_pixels_with_one_key_beyond_a_batch(hip, ctx):
    """More fragments than one LDS batch at a single depth key (two such runs in a pixel, one
    of more than two batches): the pixel is sliced by segment id inside the key, so its order
    is the exact (key, segment id) order; the frame reports no overflow, every pixel matches
    the oracle and a deep pixel's whole fragment list equals the oracle's."""
    print("case: equal keys beyond a batch", flush=True)
    cap = hip.HAIR_PIXEL_CAPACITY
    depths = np.concatenate([np.full(2 * cap + 100, 1.0), np.full(cap + 10, 1.5), np.linspace(2.0, 3.0, 5)])
    asset, cam = _layered_asset(depths, half_extent=0.1)
    # a second layer of strands on another row that stays within one batch
    extra, _ = _layered_asset(np.linspace(1.5, 2.5, 300), half_extent=0.2)
    extra.xyz[1] += (6.0 * np.linspace(1.5, 2.5, 300) / 74.6).repeat(2).astype(np.float32)
    n = asset.n_strands + extra.n_strands
    asset = hs.Asset(n, 1, np.concatenate([asset.xyz, extra.xyz], axis=1),
                     np.concatenate([asset.width, extra.width]), np.concatenate([asset.sigma_a, extra.sigma_a], axis=1))
    lights = hs.default_lights(asset, with_point=False)
    ref, ras = R.render(R.strand_level(asset), cam, lights, mat_of(asset))
    depth, same = _key_runs(ras, cam.width * cam.height)
    over = same > cap
    assert over.sum() >= 10 and ((depth > 0) & ~over).sum() >= 10 and same.max() > 2 * cap
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    out, stats, rc = ctx.render(aid, 0, cam, lights, ws=ws, raise_on_error=False)
    torch.cuda.synchronize()
    assert rc == hip.HAIR_OK, (rc, hip.last_error())
    assert stats["fragments"] == len(ras.seg)
    assert stats["overflow_pixels"] == 0 and stats["deep_pixels"] == int((depth > cap).sum())
    assert_radiance(out.cpu().numpy(), ref, what="equal keys beyond a batch")
    # the whole order of one such pixel
    p = int(np.nonzero(over)[0][len(np.nonzero(over)[0]) // 2])
    x, y = p % cam.width, p // cam.width
    cnt, keys, segs, alpha, hoff = ctx.debug_fragments(aid, 0, cam, lights, x, y, 1, 1, int(depth[p]) + 16, ws=ws)
    sel = ras.pix == p
    assert int(cnt[0, 0]) == int(depth[p])
    assert np.array_equal(keys, ras.key[sel]) and np.array_equal(segs, ras.seg[sel].astype(np.uint32))
    ws.close()
