"""Frames enqueued with hair_render_async and finished with hair_ws_finish: each equals the
same frame of hair_render bit for bit (frames in flight on two workspaces, a cold workspace,
a frame that outgrows the workspace and is rendered again at finish), and a workspace that
holds a frame refuses other calls until it is finished."""
import numpy as np
import pytest
import torch

import hairsynth as hs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip):
    c = hip.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def scene(ctx):
    asset, cam, lights = hs.config(1)
    aid = ctx.upload_asset(asset)
    yield asset, aid, lights
    ctx.release(aid)


def _sync(ctx, aid, cam, lights):
    ws = ctx.workspace()
    img, st, _ = ctx.render(aid, 0, cam, lights, ws=ws)
    torch.cuda.synchronize()
    img = img.clone()
    ws.close()
    return img, st


def _same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_frames_in_flight_equal_sync_frames(hip, ctx, scene):
    print("case: async frames in flight on two workspaces", flush=True)
    asset, aid, lights = scene
    cams = [hs.camera_for(asset, 256, 192, azimuth=0.4 * k) for k in range(6)]
    wss = [ctx.workspace(), ctx.workspace()]
    for ws in wss:                                   # warm: capacities known
        ctx.render(aid, 0, cams[0], lights, ws=ws)
    outs = [torch.empty((192, 256, 4), dtype=torch.float32, device="cuda:0") for _ in cams]
    stats = [None] * len(cams)
    for k, cam in enumerate(cams):
        ctx.render_async(aid, 0, cam, lights, outs[k], wss[k % 2])
        if k >= 1:
            stats[k - 1], rc = wss[(k - 1) % 2].finish()
            assert rc == hip.HAIR_OK
    stats[-1], _ = wss[(len(cams) - 1) % 2].finish()
    torch.cuda.synchronize()
    for k, cam in enumerate(cams):
        ref, st = _sync(ctx, aid, cam, lights)
        assert _same(outs[k], ref), k
        for key in ("fragments", "pairs", "segments_visible", "batches", "deep_pixels"):
            assert stats[k][key] == st[key], (k, key)
        assert stats[k]["ms_total"] > 0.0 and stats[k]["ms_tile"] > 0.0
    for ws in wss:
        ws.close()


def test_cold_workspace_runs_synchronously(hip, ctx, scene):
    print("case: async frame on a cold workspace", flush=True)
    asset, aid, lights = scene
    cam = hs.camera_for(asset, 200, 150, azimuth=1.0)
    ws = ctx.workspace()
    out = torch.empty((150, 200, 4), dtype=torch.float32, device="cuda:0")
    ctx.render_async(aid, 0, cam, lights, out, ws)
    st, rc = ws.finish()
    torch.cuda.synchronize()
    ref, st_ref = _sync(ctx, aid, cam, lights)
    assert rc == hip.HAIR_OK and _same(out, ref) and st["fragments"] == st_ref["fragments"]
    st2, rc2 = ws.finish()                           # nothing held any more
    assert rc2 == hip.HAIR_OK and st2["fragments"] == 0
    ws.close()


def test_outgrown_frame_is_rendered_again_at_finish(hip, ctx, scene):
    print("case: async frame beyond the capacities", flush=True)
    asset, aid, lights = scene
    small = hs.camera_for(asset, 64, 48)
    large = hs.camera_for(asset, 640, 512)
    ws = ctx.workspace()
    ctx.render(aid, 0, small, lights, ws=ws)         # capacities of a small frame
    out = torch.empty((512, 640, 4), dtype=torch.float32, device="cuda:0")
    ctx.render_async(aid, 0, large, lights, out, ws)
    st, rc = ws.finish()
    torch.cuda.synchronize()
    ref, st_ref = _sync(ctx, aid, large, lights)
    assert rc == hip.HAIR_OK and _same(out, ref)
    assert st["fragments"] == st_ref["fragments"] and st["batches"] == st_ref["batches"]
    # the workspace now keeps the larger capacities: the same frame again stays deferred
    out2 = torch.empty_like(out)
    ctx.render_async(aid, 0, large, lights, out2, ws)
    st2, _ = ws.finish()
    torch.cuda.synchronize()
    assert _same(out2, ref) and st2["fragments"] == st_ref["fragments"]
    ws.close()


def test_held_workspace_refuses_other_calls(hip, ctx, scene):
    print("case: calls on a workspace that holds a frame", flush=True)
    asset, aid, lights = scene
    cam = hs.camera_for(asset, 128, 96)
    ws = ctx.workspace()
    ctx.render(aid, 0, cam, lights, ws=ws)
    out = torch.empty((96, 128, 4), dtype=torch.float32, device="cuda:0")
    ctx.render_async(aid, 0, cam, lights, out, ws)
    _, _, rc = ctx.render(aid, 0, cam, lights, ws=ws, raise_on_error=False)
    assert rc == hip.HAIR_EINVAL and "hair_ws_finish" in hip.last_error()
    with pytest.raises(hip.HairError):
        ctx.render_async(aid, 0, cam, lights, out, ws)
    st, rc = ws.finish()
    assert rc == hip.HAIR_OK and st["fragments"] > 0
    ctx.render_async(aid, 0, cam, lights, out, ws)   # a held frame at destruction is waited for
    ws.close()
    torch.cuda.synchronize()
    ref, _ = _sync(ctx, aid, cam, lights)
    assert _same(out, ref)


def test_asset_released_before_finish(hip, ctx, scene):
    print("case: asset released while its frame is held", flush=True)
    asset, aid, lights = scene
    cam = hs.camera_for(asset, 128, 96)
    tmp = ctx.upload_asset(asset)
    ws = ctx.workspace()
    ctx.render(tmp, 0, cam, lights, ws=ws)
    out = torch.empty((96, 128, 4), dtype=torch.float32, device="cuda:0")
    ctx.render_async(tmp, 0, cam, lights, out, ws)
    ctx.release(tmp)                                 # waits for the device before freeing
    _, rc = ws.finish(raise_on_error=False)
    assert rc == hip.HAIR_ENOENT
    img, st, rc2 = ctx.render(aid, 0, cam, lights, ws=ws)   # the workspace is free again
    torch.cuda.synchronize()
    ref, _ = _sync(ctx, aid, cam, lights)
    assert rc2 == hip.HAIR_OK and _same(img, ref)
    ws.close()


@pytest.mark.parametrize("material", ["rtt", "rttd"])
def test_thick_hair_levels_async(hip, ctx, material):
    """Thick-hair levels (and the R/TT/D material) through the deferred-check path: every level
    of a small hierarchy, frames in flight on two workspaces, equal to synchronous frames."""
    print(f"case: async thick-hair levels, {material}", flush=True)
    import dataclasses
    asset = hs.make_asset(1500, 10, 90.0, seed=27, sigma_spread=True)
    if material == "rttd":
        asset = dataclasses.replace(asset, material=hs.Material.rttd())
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, hs.kmeans_hierarchy(asset, (300, 60, 10), seed=27))
    cam = hs.camera_for(asset, 160, 120)
    lights = hs.default_lights(asset, with_point=True)
    wss = [ctx.workspace(), ctx.workspace()]
    for ws in wss:
        ctx.render(aid, 0, cam, lights, ws=ws)
    outs = [torch.empty((120, 160, 4), dtype=torch.float32, device="cuda:0") for _ in range(4)]
    for level in range(4):
        ctx.render_async(aid, level, cam, lights, outs[level], wss[level % 2])
        if level >= 1:
            wss[(level - 1) % 2].finish()
    wss[1].finish()
    torch.cuda.synchronize()
    for level in range(4):
        ws = ctx.workspace()
        ref, _, _ = ctx.render(aid, level, cam, lights, ws=ws)
        torch.cuda.synchronize()
        assert _same(outs[level], ref), level
        ws.close()
    for ws in wss:
        ws.close()
    ctx.release(aid)
