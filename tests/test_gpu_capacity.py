"""Warm frames on a workspace's kept capacities: a frame that outgrows them is rendered again
with its sizes read back, and every frame equals the same frame on a fresh workspace, bit for
bit (small -> large -> small on one workspace; also the shadow pass and the backward pass,
which share the workspace's buffers)."""
import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import lod as OL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip):
    c = hip.Context(0)
    yield c
    c.close()


def _fresh(ctx, fn):
    ws = ctx.workspace()
    out = fn(ws)
    torch.cuda.synchronize()
    out = out.clone()
    ws.close()
    return out


def test_outgrown_capacities_rerender_exactly(hip, ctx):
    print("case: capacities small -> large -> small", flush=True)
    small, cam_s, lights = hs.config(1, scale=0.1)
    large, cam_l, _ = hs.config(1)
    cam_l = hs.camera_for(large, 640, 512)
    a_s = ctx.upload_asset(small)
    a_l = ctx.upload_asset(large)
    ws = ctx.workspace()
    seq = [(a_s, cam_s), (a_l, cam_l), (a_s, cam_s), (a_l, cam_l)]
    for aid, cam in seq:
        img, st, _ = ctx.render(aid, 0, cam, lights, ws=ws)
        torch.cuda.synchronize()
        ref = _fresh(ctx, lambda w: ctx.render(aid, 0, cam, lights, ws=w)[0])
        print(f"  {cam.width}x{cam.height}: {st['fragments']} fragments", flush=True)
        assert torch.equal(img.view(torch.int32), ref.view(torch.int32))
    # the shadow pass on the same workspace (a light view of another size)
    img, _, _ = ctx.render_shadowed(a_l, 0, cam_l, lights, (320, 3, 0.02), ws=ws)
    torch.cuda.synchronize()
    ref = _fresh(ctx, lambda w: ctx.render_shadowed(a_l, 0, cam_l, lights, (320, 3, 0.02), ws=w)[0])
    assert torch.equal(img.view(torch.int32), ref.view(torch.int32))
    ws.close()
    ctx.release(a_s)
    ctx.release(a_l)


def test_backward_after_larger_frames(hip, ctx):
    print("case: backward on a warm workspace", flush=True)
    asset = hs.make_asset(400, 6, 90.0, seed=11, sigma_spread=True)
    cam = hs.camera_for(asset, 96, 80)
    lights = hs.default_lights(asset, with_point=True)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 8, seed=11))
    K, S = lod["n_total"].size, asset.segs
    aid = ctx.upload_asset(asset)
    ctx.set_lod(aid, 1, lod)
    d = torch.tensor(np.random.default_rng(1).normal(size=(cam.height, cam.width, 4)), dtype=torch.float32,
                     device="cuda:0")

    def grads(ws):
        da = torch.empty((K, S, 2), dtype=torch.float32, device="cuda:0")
        dr = torch.empty(K, dtype=torch.float32, device="cuda:0")
        ds = torch.empty((3, K), dtype=torch.float32, device="cuda:0")
        ctx.render_backward(aid, 1, cam, lights, d, da, dr, ds, ws=ws)
        torch.cuda.synchronize()
        return torch.cat([da.reshape(-1), dr, ds.reshape(-1)])

    ws = ctx.workspace()
    big = hs.camera_for(asset, 512, 400)
    ctx.render(aid, 0, big, lights, ws=ws)      # capacities of a larger strand frame
    g1 = grads(ws)
    g2 = grads(ws)
    ws2 = ctx.workspace()
    g0 = grads(ws2)
    ws2.close()
    # the backward sums gradients with float atomics: equal up to summation order
    assert torch.allclose(g1, g0, rtol=1e-5, atol=1e-6) and torch.allclose(g2, g0, rtol=1e-5, atol=1e-6)
    ws.close()
    ctx.release(aid)
