"""R / TT / D material model on the GPU against the oracle, through the C-ABI: strand level,
thick-hair level, a mixed-level frame, the full-size strand frame on a sampled rectangle, and
the backward pass.  Bar as for the R / TT / TRT model: fragment counts exact, radiance within
1e-4 relative per pixel (absolute floor 1e-7), gradients within the backward test's bound."""
import dataclasses

import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import grad as OG
from oracle import lod as OL
from oracle import mixed as M
from oracle import render as R

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-4, 1e-7
RTTD = hs.Material.rttd()


def _check(got, ref, what):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    worst = float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-7)).max()) if got.size else 0.0
    print(f"[{what}] max rel err {worst:.3e}, violations {int((err > 0).sum())}", flush=True)
    assert int((err > 0).sum()) == 0, what


def _rttd(asset):
    return dataclasses.replace(asset, material=RTTD)


@pytest.fixture(scope="module")
def ctx(hip):
    c = hip.Context(0)
    yield c
    c.close()


def test_rttd_strand_level(hip, ctx):
    print("case: R/TT/D strands, 1k strands at 256x256", flush=True)
    asset, cam, lights = hs.config(1)
    asset = _rttd(asset)
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    img, st, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    ref, ras = R.render(R.strand_level(asset), cam, lights, R.material(asset.material))
    assert st["fragments"] == len(ras.seg)
    _check(img.cpu().numpy(), ref, "rttd strands")
    # the model changes the image: the same asset under R / TT / TRT differs
    aid2 = ctx.upload_asset(dataclasses.replace(asset, material=hs.Material()))
    img2, _, _ = ctx.render(aid2, 0, cam, lights, ws=ws)
    assert not torch.equal(img, img2)
    ws.close()
    ctx.release(aid)
    ctx.release(aid2)


def test_rttd_thick_hair_level(hip, ctx):
    print("case: R/TT/D thick hairs", flush=True)
    asset = _rttd(hs.make_asset(2000, 12, 90.0, seed=21, sigma_spread=True))
    cam = hs.camera_for(asset, 160, 128)
    lights = hs.default_lights(asset, with_point=True)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 40, seed=21))
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    ws = ctx.workspace()
    img, st, _ = ctx.render(aid, 1, cam, lights, ws=ws)
    ref, ras = R.render(R.cluster_level(lod), cam, lights, R.material(asset.material))
    assert st["fragments"] == len(ras.seg)
    _check(img.cpu().numpy(), ref, "rttd thick hairs")
    ws.close()
    ctx.release(aid)


def test_rttd_mixed_frame(hip, ctx):
    print("case: R/TT/D mixed frame", flush=True)
    asset = _rttd(hs.make_asset(1500, 10, 90.0, seed=24, sigma_spread=True))
    assigns = hs.kmeans_hierarchy(asset, (300, 60, 10), seed=24)
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, assigns)            # memberships; the level data below is the oracle's
    lods = [OL.build_level(asset, a) for a in assigns]
    for l, lod in enumerate(lods, 1):
        ctx.set_lod(aid, l, lod)
    geoms = M.level_geoms(asset, lods)
    grps = M.groups(assigns)
    cam = hs.camera_for(asset, 112, 96)
    lights = hs.default_lights(asset, with_point=True)
    G, S = ctx.lod_groups(aid), asset.segs
    levels = np.random.default_rng(9).integers(0, 4, size=(G, S)).astype(np.int32)
    lev = torch.tensor(levels, device="cuda:0")
    ws = ctx.workspace()
    img, st, _ = ctx.render_mixed(aid, cam, lights, lev, eps_w=2.0, ws=ws)
    mixed = M.mixed_geometry(geoms, grps, levels)
    ref, ras = R.render(mixed, cam, lights, R.material(asset.material))
    assert st["fragments"] == len(ras.seg)
    _check(img.cpu().numpy(), ref, "rttd mixed")
    ws.close()
    ctx.release(aid)


def test_rttd_config2_full_size_sampled(hip, ctx):
    """100k strands x 32 segments at 1920x1080 (the benchmark's frame) with the R / TT / D
    material: the densest 24x24 rectangle against the oracle."""
    print("case: R/TT/D 100k strands at 1920x1080", flush=True)
    asset, cam, lights = hs.config(2)
    asset = _rttd(asset)
    aid = ctx.upload_asset(asset)
    ws = ctx.workspace()
    img, st, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    got = img.cpu().numpy()
    a = got[..., 3]
    y, x = np.unravel_index(np.argmax(a * (a < 1.0) + (a >= 1.0) * 0.5), a.shape)
    x0, y0 = int(min(max(x - 12, 0), cam.width - 24)), int(min(max(y - 12, 0), cam.height - 24))
    ref, ras = R.render(R.strand_level(asset), cam, lights, R.material(asset.material), rect=(x0, y0, 24, 24))
    _check(got[y0:y0 + 24, x0:x0 + 24], ref[y0:y0 + 24, x0:x0 + 24], f"rttd 100k-strand 1080p rect {x0},{y0}")
    ws.close()
    ctx.release(aid)


def _close(got, ref, what):
    scale = float(np.abs(ref).max())
    err = np.abs(got - ref)
    tol = 2e-3 * scale + 2e-3 * np.abs(ref)
    print(f"[{what}] max |err| {float(err.max()):.3e} (scale {scale:.3e}), violations {int((err > tol).sum())}",
          flush=True)
    assert int((err > tol).sum()) == 0, what


def test_rttd_backward_matches_oracle_gradient(hip, ctx):
    print("case: R/TT/D backward vs oracle", flush=True)
    asset = _rttd(hs.make_asset(400, 6, 90.0, seed=15, sigma_spread=True))
    cam = hs.camera_for(asset, 96, 80)
    lights = hs.default_lights(asset, with_point=True)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 8, seed=15))
    K, S = lod["n_total"].size, asset.segs
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    d_rgba = np.random.default_rng(15).normal(size=(cam.height, cam.width, 4))
    g_axes, g_r, g_sig, _ = OG.cluster_vjp(R.cluster_level(lod), cam, lights, R.material(asset.material), d_rgba, K, S)
    dev = "cuda:0"
    d = torch.tensor(d_rgba, dtype=torch.float32, device=dev).contiguous()
    da = torch.empty((K, S, 2), dtype=torch.float32, device=dev)
    dr = torch.empty(K, dtype=torch.float32, device=dev)
    ds = torch.empty((3, K), dtype=torch.float32, device=dev)
    ctx.render_backward(aid, 1, cam, lights, d, da, dr, ds)
    torch.cuda.synchronize()
    _close(da.cpu().numpy(), g_axes, "rttd d_axes")
    _close(dr.cpu().numpy(), g_r, "rttd d_r")
    assert not np.any(g_sig) and not torch.any(ds)      # the model does not read sigma_a
    ctx.release(aid)
