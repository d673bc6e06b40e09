"""hair_render_noalloc, the frame entry point that allocates nothing (its buffers are carved
from a static device scratch array): through the C-ABI its frames equal hair_render's bit for
bit, on consecutive calls whose second input is smaller (the scratch keeps the first call's
contents); a frame too large for the scratch fails with HAIR_ENOMEM and leaves the image as
it was."""
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


def _same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def _reference(ctx, aid, level, cam, lights):
    ws = ctx.workspace()
    img, st, _ = ctx.render(aid, level, cam, lights, ws=ws)
    torch.cuda.synchronize()
    img = img.clone()
    ws.close()
    return img, st


def test_noalloc_equals_render_on_consecutive_calls(hip, ctx):
    big, cam_big, lights_big = hs.config(1)                      # 1,000 x 16 strands, 256 x 256, 1 light
    small = hs.make_asset(300, 8, 60.0, seed=5)
    cam_small = hs.camera_for(small, 120, 90, azimuth=0.7)
    lights_small = hs.default_lights(small, True)
    a_big = ctx.upload_asset(big)
    a_small = ctx.upload_asset(small)
    assert hip.lib.hair_noalloc_scratch_bytes() == 64 << 20
    cases = [("1000x16 strands at 256x256", a_big, cam_big, lights_big),
             ("300x8 strands at 120x90 with a point light", a_small, cam_small, lights_small)]
    for name, aid, cam, lights in cases:
        print("case: noalloc", name, flush=True)
        out = torch.full((cam.height, cam.width, 4), float("nan"), dtype=torch.float32, device="cuda:0")
        out, st, rc = ctx.render_noalloc(aid, 0, cam, lights, out)
        torch.cuda.synchronize()
        ref, st_ref = _reference(ctx, aid, 0, cam, lights)
        assert rc == hip.HAIR_OK
        assert st["fragments"] > 0
        for key in ("fragments", "pairs", "segments", "segments_visible", "batches", "deep_pixels",
                    "overflow_pixels"):
            assert st[key] == st_ref[key], (name, key)
        assert _same(out, ref), name
    ctx.release(a_big)
    ctx.release(a_small)


def test_noalloc_rejects_frames_beyond_the_scratch(hip, ctx):
    print("case: noalloc frames too large for the scratch", flush=True)
    # 20k x 32 strands at 1920x1080: the strand level's segment records and binning matrix
    # alone exceed 64 MiB (rejected before any launch); its 2,000-thick-hair level has 64k
    # segments but tens of millions of fragments (rejected once the frame's sizes are read back)
    asset = hs.make_asset(20000, 32, 90.0, seed=33)
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, [hs.kmeans_assign(asset, 2000, seed=33)])
    cam = hs.camera_for(asset, 1920, 1080)
    lights = hs.default_lights(asset, True)
    for level in (0, 1):
        out = torch.full((1080, 1920, 4), 7.0, dtype=torch.float32, device="cuda:0")
        _, _, rc = ctx.render_noalloc(aid, level, cam, lights, out, raise_on_error=False)
        torch.cuda.synchronize()
        assert rc == hip.HAIR_ENOMEM, (level, rc, hip.last_error())
        assert "static scratch" in hip.last_error()
        assert bool((out == 7.0).all()), level
    # the scratch still serves a frame that fits, after the rejected ones
    small = hs.make_asset(200, 8, 60.0, seed=9)
    a2 = ctx.upload_asset(small)
    cam2 = hs.camera_for(small, 64, 48)
    out = torch.empty((48, 64, 4), dtype=torch.float32, device="cuda:0")
    out, st, rc = ctx.render_noalloc(a2, 0, cam2, lights[:1], out)
    ref, st_ref = _reference(ctx, a2, 0, cam2, lights[:1])
    assert rc == hip.HAIR_OK and st["fragments"] == st_ref["fragments"] and _same(out, ref)
    ctx.release(a2)
    ctx.release(aid)
