"""Deep opacity map shadows on the GPU against the oracle (C-ABI): the light grid bit-exact,
every texel's first hit bit-exact and its layer counts within float32 summation error, and
the shadowed frame within 1e-4 relative per pixel, at the strand level, at a thick-hair level,
with the R / TT / D material, on a ragged map size; plus the reductions (no directional light:
the plain frame, bit for bit) and the effect (the frame darkens, coverage is unchanged)."""
import dataclasses

import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import lod as OL
from oracle import render as R
from oracle import shadow as SH

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


def _dom_parity(ctx, ws, geom, light, li, R, K, delta, what):
    tex, grid = ctx.debug_dom(ws, li, R)
    dom = SH.build_dom(geom, light.vec, R, K, delta)
    g = dom.grid
    want = np.concatenate([g["e1"], g["e2"], g["d"], g["omega"], [g["u0"], g["v0"], g["s"], g["z_ref"]]]).astype(np.float32)
    assert np.array_equal(grid.view(np.uint32), want.view(np.uint32)), (grid, want)
    assert np.array_equal(tex[:, 0].view(np.uint32), dom.iz0.view(np.uint32))
    C = tex[:, 1:1 + K].astype(np.float64)
    err = np.abs(C - dom.C) - (1e-5 * np.abs(dom.C) + 1e-6)
    print(f"[{what} DOM] texels with hair {(dom.iz0 > 0).sum()}, max count {dom.C[:, -1].max():.3f}, "
          f"max abs err {float(np.abs(C - dom.C).max()):.3e}", flush=True)
    assert int((err > 0).sum()) == 0
    # layers past K repeat the total
    assert np.array_equal(tex[:, K:8], np.repeat(tex[:, K:K + 1], 8 - K, axis=1))


@pytest.mark.parametrize("material", ["rttrt", "rttd"])
def test_shadowed_strands(hip, ctx, material):
    print(f"case: shadowed strands ({material})", flush=True)
    asset, cam, lights = hs.config(1)
    if material == "rttd":
        asset = dataclasses.replace(asset, material=hs.Material.rttd())
    lights = hs.default_lights(asset, with_point=True)
    R_, K, delta = 200, 4, 0.02
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    img, st, _ = ctx.render_shadowed(aid, 0, cam, lights, (R_, K, delta), ws=ws)
    geom = R.strand_level(asset)
    _dom_parity(ctx, ws, geom, lights[0], 0, R_, K, delta, f"strands {material}")
    with pytest.raises(hip.HairError):
        ctx.debug_dom(ws, 1, R_)                         # the point light has no map
    ref, ras = R.render(geom, cam, lights, R.material(asset.material), shadow=(R_, K, delta))
    assert st["fragments"] == len(ras.seg)
    got = img.cpu().numpy()
    _check(got, ref, f"shadowed strands {material}")
    plain, _, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    p = plain.cpu().numpy()
    assert float(got[..., :3].sum()) < float(p[..., :3].sum())         # shadows darken the frame
    assert np.array_equal(got[..., 3], p[..., 3])                      # coverage unchanged
    ws.close()
    ctx.release(aid)


@pytest.mark.parametrize("r_scale", [1.0, 25.0])
def test_shadowed_thick_hairs(hip, ctx, r_scale):
    """r_scale 25: hair radii scaled up so that the clusters are denser (rho up to 0.13) and
    the counts in the map reach about three hairs."""
    print(f"case: shadowed thick hairs (r x {r_scale})", flush=True)
    asset = hs.make_asset(2000, 12, 90.0, seed=21, sigma_spread=True)
    cam = hs.camera_for(asset, 160, 128)
    lights = hs.default_lights(asset, with_point=False)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 60, seed=21))
    lod["r"] = (lod["r"] * np.float32(r_scale)).astype(np.float32)
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    ws = ctx.workspace()
    R_, K, delta = 96, 3, 0.03
    img, st, _ = ctx.render_shadowed(aid, 1, cam, lights, (R_, K, delta), ws=ws)
    geom = R.cluster_level(lod)
    _dom_parity(ctx, ws, geom, lights[0], 0, R_, K, delta, f"thick hairs r x {r_scale}")
    ref, ras = R.render(geom, cam, lights, R.material(asset.material), shadow=(R_, K, delta))
    assert st["fragments"] == len(ras.seg)
    _check(img.cpu().numpy(), ref, f"shadowed thick hairs r x {r_scale}")
    ws.close()
    ctx.release(aid)


def test_without_directional_lights_the_plain_frame(hip, ctx):
    print("case: shadowed render with point lights only", flush=True)
    asset, cam, _ = hs.config(1, scale=0.5)
    lights = [hs.default_lights(asset, with_point=True)[1]]
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    a, _, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    b, _, _ = ctx.render_shadowed(aid, 0, cam, lights, (64, 2, 0.02), ws=ws)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    ws.close()
    ctx.release(aid)
