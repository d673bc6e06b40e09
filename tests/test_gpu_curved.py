"""Curved thick hairs on the GPU against the oracle (C-ABI): the tessellated rows' records
bit-exact (snapped endpoints, inverse depths, half-widths, flags), fragment counts exact,
radiance within 1e-4 relative per pixel, both materials, and the reduction to the plain
thick-hair frame when no segment is split."""
import dataclasses

import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import curve as CV
from oracle import lod as OL
from oracle import render as R

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-4, 1e-7


def _check(got, ref, what):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    worst = float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-7)).max()) if got.size else 0.0
    print(f"[{what}] max rel err {worst:.3e}, violations {int((err > 0).sum())}", flush=True)
    assert int((err > 0).sum()) == 0, what


@pytest.fixture(scope="module")
def ctx(hip):
    c = hip.Context(0)
    yield c
    c.close()


def _scene(material=None, seed=31):
    asset = hs.make_asset(1500, 10, 90.0, seed=seed, sigma_spread=True)
    if material is not None:
        asset = dataclasses.replace(asset, material=material)
    cam = hs.camera_for(asset, 320, 272)
    lights = hs.default_lights(asset, with_point=True)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 30, seed=seed))
    return asset, cam, lights, lod


@pytest.mark.parametrize("material,max_px,max_sub", [(None, 2, 16), (None, 1, 5), ("rttd", 1, 8)])
def test_curved_rows_and_radiance(hip, ctx, material, max_px, max_sub):
    print(f"case: curved thick hairs ({material}, max_px {max_px}, max_sub {max_sub})", flush=True)
    asset, cam, lights, lod = _scene(hs.Material.rttd() if material == "rttd" else None)
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    ws = ctx.workspace()
    img, st, _ = ctx.render_curved(aid, 1, cam, lights, max_px, max_sub, ws=ws)
    geom = CV.curved_geometry(lod, cam, max_px, max_sub)
    n = geom.pA.shape[1]
    assert st["segments"] == n and n > lod["n_total"].size * asset.segs
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = R.segment_records(geom, cam)
    ri, rf = ctx.debug_segments(ws, n)
    v = (ri[:, 5] & 1).astype(bool)
    assert np.array_equal(v, vis)
    for col, ref in enumerate((XA, YA, XB, YB, hw_fx)):
        assert np.array_equal(ri[v, col], ref[vis]), col
    for col, ref in enumerate((izA, izB, hw)):
        assert np.array_equal(rf[:, col].view(np.uint32), ref.view(np.uint32)), col
    ref, ras = R.render(geom, cam, lights, R.material(asset.material))
    assert st["fragments"] == len(ras.seg)
    _check(img.cpu().numpy(), ref, f"curved {material} {max_px}/{max_sub}")
    ws.close()
    ctx.release(aid)


def test_unsplit_curve_is_the_plain_level(hip, ctx):
    print("case: curved with one step per segment", flush=True)
    asset, cam, lights, lod = _scene(seed=32)
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    ws = ctx.workspace()
    a, sa, _ = ctx.render(aid, 1, cam, lights, ws=ws)
    b, sb, _ = ctx.render_curved(aid, 1, cam, lights, 4096, 1, ws=ws)
    assert sa["fragments"] == sb["fragments"] and sa["segments"] == sb["segments"]
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    ws.close()
    ctx.release(aid)


def test_curved_wide_hairs_full_size_sampled(hip, ctx):
    """Curved thick hairs up to ~150 px in radius at 1920x1080 (20k strands x 16 segments in 60
    clusters, at most 2 px per step): every tessellated record bit-exact, and the radiance on
    rectangles at the footprints' borders and at the deepest pixel against the oracle, which
    enumerates pixels without tile binning."""
    print("case: curved wide thick hairs at 1920x1080", flush=True)
    asset = hs.make_asset(20000, 16, 90.0, seed=34, sigma_spread=True)
    cam = hs.camera_for(asset, 1920, 1080)
    lights = hs.default_lights(asset, with_point=True)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 60, seed=34))
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    ws = ctx.workspace()
    img, st, _ = ctx.render_curved(aid, 1, cam, lights, 2, 16, ws=ws)
    geom = CV.curved_geometry(lod, cam, 2, 16)
    n = geom.pA.shape[1]
    assert st["segments"] == n
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = R.segment_records(geom, cam)
    ri, rf = ctx.debug_segments(ws, n)
    v = (ri[:, 5] & 1).astype(bool)
    assert np.array_equal(v, vis)
    for col, ref in enumerate((XA, YA, XB, YB, hw_fx)):
        assert np.array_equal(ri[v, col], ref[vis]), col
    got = img.cpu().numpy()
    alpha = got[..., 3]
    inside = alpha > 0
    edge = inside & ~(np.roll(inside, 1, 0) & np.roll(inside, -1, 0) & np.roll(inside, 1, 1) & np.roll(inside, -1, 1))
    ys, xs = np.nonzero(edge)
    assert ys.size > 0
    rng = np.random.default_rng(34)
    picks = [(int(ys[i]), int(xs[i])) for i in rng.choice(ys.size, size=3, replace=False)]
    picks.append(tuple(int(q) for q in np.unravel_index(np.argmax(alpha * (alpha < 1.0)), alpha.shape)))
    mat = R.material(asset.material)
    print(f"curved wide thick hairs: {n} segments, {st['fragments']} fragments", flush=True)
    for y, x in picks:
        x0 = int(min(max(x - 12, 0), cam.width - 24))
        y0 = int(min(max(y - 12, 0), cam.height - 24))
        ref, _ = R.render(geom, cam, lights, mat, rect=(x0, y0, 24, 24))
        _check(got[y0:y0 + 24, x0:x0 + 24], ref[y0:y0 + 24, x0:x0 + 24], f"curved wide 1080p rect {x0},{y0}")
    ws.close()
    ctx.release(aid)
