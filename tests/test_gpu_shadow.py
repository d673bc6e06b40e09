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


@pytest.mark.parametrize("material", ["rttrt", "rttd"])
def test_shadowed_mixed_frame(hip, ctx, material):
    """A mixed-level frame (a random level per group and segment) with deep opacity maps: the
    map of the frame's own rows (grid and first hits bit-exact, counts within float32 summation
    error) and the frame within 1e-4 of the oracle; with one level everywhere it is that
    level's shadowed frame."""
    print(f"case: shadowed mixed frame ({material})", flush=True)
    from oracle import mixed as M
    asset = hs.make_asset(2500, 10, 90.0, seed=23, sigma_spread=True)
    if material == "rttd":
        asset = dataclasses.replace(asset, material=hs.Material.rttd())
    assigns = hs.kmeans_hierarchy(asset, (400, 80, 12), seed=23)
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, assigns)
    lods = [OL.build_level(asset, a) for a in assigns]
    for l, lod in enumerate(lods, 1):
        ctx.set_lod(aid, l, lod)
    geoms = M.level_geoms(asset, lods)
    grps = M.groups(assigns)
    cam = hs.camera_for(asset, 120, 104)
    lights = hs.default_lights(asset, with_point=True)
    G, S = ctx.lod_groups(aid), asset.segs
    levels = np.random.default_rng(41).integers(0, 4, size=(G, S)).astype(np.int32)
    R_, K, delta = 96, 4, 0.02
    ws = ctx.workspace()
    lev = torch.tensor(levels, device="cuda:0")
    img, st, _ = ctx.render_mixed_shadowed(aid, cam, lights, lev, (R_, K, delta), ws=ws)
    torch.cuda.synchronize()
    mixed = M.mixed_geometry(geoms, grps, levels)
    assert st["segments"] == mixed.pA.shape[1]
    _dom_parity(ctx, ws, mixed, lights[0], 0, R_, K, delta, "mixed frame")
    ref, ras = R.render(mixed, cam, lights, R.material(asset.material), shadow=(R_, K, delta))
    assert st["fragments"] == len(ras.seg)
    _check(img.cpu().numpy(), ref, f"shadowed mixed frame ({material})")
    plain, _, _ = ctx.render_mixed(aid, cam, lights, lev, ws=ws)
    torch.cuda.synchronize()
    assert not torch.equal(plain, img)
    # one level everywhere: the level's own shadowed frame (rows in another order)
    for l in (0, 2):
        uni = torch.full((G, S), l, dtype=torch.int32, device="cuda:0")
        a, _, _ = ctx.render_mixed_shadowed(aid, cam, lights, uni, (R_, K, delta), ws=ws)
        b, _, _ = ctx.render_shadowed(aid, l, cam, lights, (R_, K, delta), ws=ws)
        torch.cuda.synchronize()
        x, y = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(x - y) <= 2e-4 * np.abs(y) + 1e-7), l
    ws.close()
    ctx.release(aid)
