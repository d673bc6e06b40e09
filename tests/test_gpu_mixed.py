"""Per-group LoD selection and mixed-level frames on the GPU against the oracle (C-ABI)."""
import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import lod as OL
from oracle import mixed as M
from oracle import render as R

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-4, 1e-7


def oracle_levels(ctx, aid, asset, assigns):
    """The hierarchy's memberships from hair_build_lod, every level's data from the oracle's
    construction (uploaded with hair_set_lod, which keeps the memberships): both sides then
    render the same level data, none of it computed by the HIP path."""
    ctx.build_lod(aid, assigns)
    lods = [OL.build_level(asset, a) for a in assigns]
    for l, lod in enumerate(lods, 1):
        ctx.set_lod(aid, l, lod)
    return lods


@pytest.fixture(scope="module")
def scene(hip):
    ctx = hip.Context(0)
    asset = hs.make_asset(2500, 10, 90.0, seed=23, sigma_spread=True)
    assigns = hs.kmeans_hierarchy(asset, (400, 80, 12), seed=23)
    aid = ctx.upload_asset(asset)
    lods = oracle_levels(ctx, aid, asset, assigns)
    geoms = M.level_geoms(asset, lods)
    grps = M.groups(assigns)
    cam = hs.camera_for(asset, 120, 104)
    lights = hs.default_lights(asset, with_point=True)
    G, S = int(assigns[-1].max()) + 1, asset.segs
    widths = M.level_widths(geoms[1], grps[1], G, S, cam)
    eps = float(np.median(widths[widths > 0]))
    yield ctx, asset, aid, assigns, geoms, grps, cam, lights, eps
    ctx.close()


def test_groups_and_initial_levels(hip, scene):
    print("case: mixed LoD init", flush=True)
    ctx, asset, aid, assigns, geoms, grps, cam, lights, eps = scene
    G = ctx.lod_groups(aid)
    assert G == int(assigns[-1].max()) + 1
    lev = torch.empty((G, asset.segs), dtype=torch.int32, device="cuda:0")
    ctx.lod_init(aid, cam, eps, lev)
    ref = M.init_levels(geoms, grps, cam, eps)
    got = lev.cpu().numpy()
    assert len(np.unique(ref)) >= 3
    assert np.array_equal(got, ref)


def test_mixed_frame_matches_oracle_and_updates_levels(hip, scene):
    print("case: mixed frame", flush=True)
    ctx, asset, aid, assigns, geoms, grps, cam, lights, eps = scene
    G, S = ctx.lod_groups(aid), asset.segs
    rng = np.random.default_rng(7)
    levels = rng.integers(0, 4, size=(G, S)).astype(np.int32)
    lev = torch.tensor(levels, device="cuda:0")
    ws = ctx.workspace()
    img, st, _ = ctx.render_mixed(aid, cam, lights, lev, eps_w=eps, ws=ws)
    torch.cuda.synchronize()
    mixed = M.mixed_geometry(geoms, grps, levels)
    assert st["segments"] == mixed.pA.shape[1]
    # projected rows bit-exact, with the thick-hair flag
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = R.segment_records(mixed, cam)
    ri, rf = ctx.debug_segments(ws, mixed.pA.shape[1])
    assert np.array_equal((ri[:, 5] & 1).astype(bool), vis)
    for col, ref in enumerate((XA, YA, XB, YB, hw_fx)):
        assert np.array_equal(ri[vis, col], ref[vis]), col
    assert np.array_equal(rf[:, 2].view(np.uint32), hw.view(np.uint32))
    assert np.array_equal((ri[:, 5] & 8) != 0, mixed.thick)
    ref, ras = R.render(mixed, cam, lights, tuple(float(v) for v in asset.material.as_array()))
    assert st["fragments"] == len(ras.seg)
    got = img.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    print(f"mixed frame: {len(ras.seg)} fragments, max rel err "
          f"{float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-7)).max()):.3e}", flush=True)
    assert int((err > 0).sum()) == 0
    # the deferred update that followed the frame
    assert np.array_equal(lev.cpu().numpy(), M.update_levels(geoms, grps, cam, eps, levels))
    ws.close()


def test_mixed_frame_with_few_thick_cells_matches_oracle(hip, scene):
    """A frame of strands with a few coarse cells: few batches hold thick-hair fragments, so the
    strand-only kernel takes most batches and the mixed one takes the listed rest."""
    print("case: mixed frame, few thick cells", flush=True)
    ctx, asset, aid, assigns, geoms, grps, cam, lights, eps = scene
    G, S = ctx.lod_groups(aid), asset.segs
    rng = np.random.default_rng(11)
    levels = np.zeros((G, S), dtype=np.int32)
    pick = rng.choice(G * S, size=max(1, G * S // 150), replace=False)
    levels.reshape(-1)[pick] = rng.integers(1, 4, size=pick.size)
    lev = torch.tensor(levels, device="cuda:0")
    img, st, _ = ctx.render_mixed(aid, cam, lights, lev)
    torch.cuda.synchronize()
    mixed = M.mixed_geometry(geoms, grps, levels)
    assert mixed.thick.any() and mixed.thick.mean() < 0.05
    ref, ras = R.render(mixed, cam, lights, tuple(float(v) for v in asset.material.as_array()))
    assert st["fragments"] == len(ras.seg)
    got = img.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    assert int((err > 0).sum()) == 0


def test_uniform_mixed_equals_level_render(hip, scene):
    print("case: uniform mixed", flush=True)
    ctx, asset, aid, assigns, geoms, grps, cam, lights, eps = scene
    G, S = ctx.lod_groups(aid), asset.segs
    for l in (0, 3):
        lev = torch.full((G, S), l, dtype=torch.int32, device="cuda:0")
        a, _, _ = ctx.render_mixed(aid, cam, lights, lev)
        b, _, _ = ctx.render(aid, l, cam, lights)
        torch.cuda.synchronize()
        assert torch.equal(lev, torch.full_like(lev, l))          # eps_w = 0: levels unchanged
        x, y = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(x - y) <= 2e-4 * np.abs(y) + 1e-7), l


def test_mixed_errors(hip, scene):
    print("case: mixed errors", flush=True)
    ctx, asset, aid, assigns, geoms, grps, cam, lights, eps = scene
    G, S = ctx.lod_groups(aid), asset.segs
    bad = torch.full((G, S), 0, dtype=torch.int32, device="cuda:0")
    bad[0, 0] = 9
    with pytest.raises(hip.HairError) as e:
        ctx.render_mixed(aid, cam, lights, bad)
    assert e.value.code == hip.HAIR_EINVAL
    aid2 = ctx.upload_asset(asset)
    ctx.build_lod(aid2, [hs.kmeans_assign(asset, 40, seed=1), hs.kmeans_assign(asset, 9, seed=2)])
    with pytest.raises(hip.HairError):
        ctx.lod_groups(aid2)
    ctx.release(aid2)


def test_mixed_frame_full_size_sampled(hip):
    """A mixed-level frame at 1920x1080 (20k strands x 16 segments; 2000 / 300 / 40 thick
    hairs; a random level per group and segment): every projected row bit-exact, the deferred
    level update equal, the fragment count equal to the oracle's stored census, and the
    radiance on rectangles at coverage borders and at the deepest pixel (most fragments, from
    the census) against the oracle."""
    print("case: mixed frame at 1920x1080", flush=True)
    ctx = hip.Context(0)
    asset = hs.make_asset(20000, 16, 90.0, seed=35, sigma_spread=True)
    assigns = hs.kmeans_hierarchy(asset, (2000, 300, 40), seed=35)
    aid = ctx.upload_asset(asset)
    lods = oracle_levels(ctx, aid, asset, assigns)
    geoms = M.level_geoms(asset, lods)
    grps = M.groups(assigns)
    cam = hs.camera_for(asset, 1920, 1080)
    lights = hs.default_lights(asset, with_point=True)
    G, S = ctx.lod_groups(aid), asset.segs
    levels = np.random.default_rng(35).integers(0, 4, size=(G, S)).astype(np.int32)
    lev = torch.tensor(levels, device="cuda:0")
    ws = ctx.workspace()
    img, st, _ = ctx.render_mixed(aid, cam, lights, lev, eps_w=2.0, ws=ws)
    torch.cuda.synchronize()
    mixed = M.mixed_geometry(geoms, grps, levels)
    n = mixed.pA.shape[1]
    assert st["segments"] == n
    c, XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = R.segment_records(mixed, cam)
    ri, rf = ctx.debug_segments(ws, n)
    assert np.array_equal((ri[:, 5] & 1).astype(bool), vis)
    for col, ref in enumerate((XA, YA, XB, YB, hw_fx)):
        assert np.array_equal(ri[vis, col], ref[vis]), col
    assert np.array_equal(lev.cpu().numpy(), M.update_levels(geoms, grps, cam, 2.0, levels))
    got = img.cpu().numpy().astype(np.float64)
    # the fragment count and the deepest pixel (most fragments) from the oracle's stored census
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mixed_20k_1080p.json")) as f:
        gold = json.load(f)
    assert st["fragments"] == gold["fragments"]
    deep = gold["deepest"][0]
    alpha = got[..., 3]
    inside = alpha > 0
    edge = inside & ~(np.roll(inside, 1, 0) & np.roll(inside, -1, 0) & np.roll(inside, 1, 1) & np.roll(inside, -1, 1))
    ys, xs = np.nonzero(edge)
    rng = np.random.default_rng(36)
    picks = [(int(ys[i]), int(xs[i])) for i in rng.choice(ys.size, size=2, replace=False)]
    picks.append((deep["y"], deep["x"]))
    mat = tuple(float(v) for v in asset.material.as_array())
    print(f"mixed 1080p: {n} segments, {st['fragments']} fragments, deepest pixel {deep['count']}", flush=True)
    for y, x in picks:
        x0 = int(min(max(x - 12, 0), cam.width - 24))
        y0 = int(min(max(y - 12, 0), cam.height - 24))
        ref, _ = R.render(mixed, cam, lights, mat, rect=(x0, y0, 24, 24))
        err = np.abs(got - ref)[y0:y0 + 24, x0:x0 + 24] - (RTOL * np.abs(ref) + ATOL)[y0:y0 + 24, x0:x0 + 24]
        print(f"[mixed 1080p rect {x0},{y0}] violations {int((err > 0).sum())}", flush=True)
        assert int((err > 0).sum()) == 0
    ws.close()
    ctx.release(aid)
    ctx.close()


def test_far_view_lod_frame_matches_oracle(hip):
    """The regime the LoD is for: a groom of locks (20k strands x 32 segments in locks of 16, a
    smooth flow; 1250 / 312 / 78 thick hairs by k-means on the strands' paths) at the paper's
    far view (its bounding sphere covering 0.3% of 1920x1080).  The initial per-(group,
    segment) levels at eps_w = 2 px equal the oracle's and go mostly coarse, and the whole
    frame (fragment count and every pixel) matches the oracle."""
    print("case: far-view LoD frame", flush=True)
    ctx = hip.Context(0)
    n = 20000
    asset = hs.make_asset(n, 32, 90.0, seed=41, sigma_spread=True, clumps=n // 16, flow=0.99)
    assigns = hs.kmeans_hierarchy(asset, (n // 16, n // 64, n // 256), seed=41, iters=20, features="path")
    aid = ctx.upload_asset(asset)
    lods = oracle_levels(ctx, aid, asset, assigns)
    geoms = M.level_geoms(asset, lods)
    grps = M.groups(assigns)
    cam = hs.camera_occupancy(asset, 1920, 1080, 0.003)
    lights = hs.default_lights(asset, with_point=True)
    G, S = ctx.lod_groups(aid), asset.segs
    lev = torch.empty((G, S), dtype=torch.int32, device="cuda:0")
    ctx.lod_init(aid, cam, 2.0, lev)
    levels = M.init_levels(geoms, grps, cam, 2.0)
    assert np.array_equal(lev.cpu().numpy(), levels)
    assert (levels > 0).mean() > 0.5
    img, st, _ = ctx.render_mixed(aid, cam, lights, lev)
    torch.cuda.synchronize()
    mixed = M.mixed_geometry(geoms, grps, levels)
    ref, ras = R.render(mixed, cam, lights, tuple(float(v) for v in asset.material.as_array()))
    assert st["fragments"] == len(ras.seg)
    got = img.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    print(f"far view: {(levels > 0).mean():.3f} of the cells coarse, {len(ras.seg)} fragments, max rel err "
          f"{float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-7)).max()):.3e}", flush=True)
    assert int((err > 0).sum()) == 0
    ctx.close()
