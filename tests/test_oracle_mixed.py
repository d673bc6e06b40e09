"""Oracle pins for per-group LoD selection and mixed-level frames."""
import numpy as np
import pytest

import hairsynth as hs
from oracle import lod as OL
from oracle import mixed as M
from oracle import render as R


@pytest.fixture(scope="module")
def scene():
    asset = hs.make_asset(600, 8, 90.0, seed=21, sigma_spread=True)
    assigns = hs.kmeans_hierarchy(asset, (120, 30, 6), seed=21)
    lods = [OL.build_level(asset, a) for a in assigns]
    cam = hs.camera_for(asset, 64, 56)
    lights = hs.default_lights(asset, with_point=True)
    geoms = M.level_geoms(asset, lods)
    grps = M.groups(assigns)
    return asset, assigns, lods, cam, lights, geoms, grps


def mat_of(asset):
    return tuple(float(v) for v in asset.material.as_array())


def test_hierarchy_is_nested_and_groups_cover(scene):
    asset, assigns, lods, cam, lights, geoms, grps = scene
    G = int(assigns[-1].max()) + 1
    for l, g in enumerate(grps):
        n_owner = asset.n_strands if l == 0 else int(assigns[l - 1].max()) + 1
        assert g.size == n_owner and g.min() >= 0 and g.max() < G
    # a strand's group equals its clusters' groups at every level
    for l, a in enumerate(assigns, start=1):
        assert np.array_equal(grps[l][a], grps[0])
    bad = [assigns[0].copy(), np.roll(assigns[-1], 1)]
    with pytest.raises(ValueError):
        M.groups(bad)


def test_uniform_levels_reproduce_single_level_frames(scene):
    asset, assigns, lods, cam, lights, geoms, grps = scene
    G, S = int(assigns[-1].max()) + 1, asset.segs
    mat = mat_of(asset)
    for l in (0, 2):
        mixed = M.mixed_geometry(geoms, grps, np.full((G, S), l, np.int32))
        a, _ = R.render(mixed, cam, lights, mat)
        b, _ = R.render(geoms[l], cam, lights, mat)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-15), l


def test_mixed_fragments_shade_as_their_own_level(scene):
    """In a genuinely mixed frame every fragment has the coverage, alpha and radiance it has in
    the frame of its own level; only the per-pixel merge differs."""
    asset, assigns, lods, cam, lights, geoms, grps = scene
    G, S = int(assigns[-1].max()) + 1, asset.segs
    rng = np.random.default_rng(5)
    levels = rng.integers(0, len(geoms), size=(G, S)).astype(np.int32)
    mixed = M.mixed_geometry(geoms, grps, levels)
    mat = mat_of(asset)
    ras = R.rasterize(mixed, cam)
    alpha, L = R.fragment_radiance(mixed, ras, cam, lights, mat)
    # map every mixed row back to (level, row of that level)
    lists = [M.owners_by_group(grps[l], G) for l in range(len(geoms))]
    src = []
    for g in range(G):
        for k in range(S):
            lv = int(levels[g, k])
            src += [(lv, int(o) * S + k) for o in lists[lv][g]]
    assert len(src) == mixed.pA.shape[1]
    checked = 0
    for l, gm in enumerate(geoms):
        rows = np.array([i for i, (lv, _) in enumerate(src) if lv == l], dtype=np.int64)
        if rows.size == 0:
            continue
        orig = np.array([src[i][1] for i in rows])
        r2 = R.rasterize(gm, cam)
        a2, L2 = R.fragment_radiance(gm, r2, cam, lights, mat)
        ref = {(int(s), int(p)): i for i, (s, p) in enumerate(zip(r2.seg, r2.pix))}
        m = np.isin(ras.seg, rows)
        to_orig = dict(zip(rows.tolist(), orig.tolist()))
        for i in np.nonzero(m)[0]:
            j = ref[(to_orig[int(ras.seg[i])], int(ras.pix[i]))]
            assert abs(float(alpha[i]) - float(a2[j])) <= 1e-12
            assert np.allclose(L[i].numpy(), L2[j].numpy(), rtol=1e-12, atol=1e-15)
            checked += 1
        # and no fragment of those rows is missing
        own = np.isin(r2.seg, orig)
        assert int(own.sum()) == int(m.sum())
    assert checked == len(ras.seg) and checked > 0


def test_selection_rules(scene):
    asset, assigns, lods, cam, lights, geoms, grps = scene
    G, S, n = int(assigns[-1].max()) + 1, asset.segs, len(geoms) - 1
    assert np.all(M.init_levels(geoms, grps, cam, np.inf) == n)
    assert np.all(M.init_levels(geoms, grps, cam, 0.0) == 0)
    widths = [M.level_widths(geoms[l], grps[l], G, S, cam) for l in range(n + 1)]
    eps = float(np.median(widths[1]))
    lev = M.init_levels(geoms, grps, cam, eps)
    assert len(np.unique(lev)) >= 2
    # the chosen level qualifies and the next coarser one does not
    for g in range(G):
        for k in range(S):
            L = int(lev[g, k])
            if L >= 1:
                assert widths[L][g, k] <= eps
            for l in range(L + 1, n + 1):
                assert widths[l][g, k] > eps
    # the initial levels are a fixed point of the deferred update (strand widths < eps here)
    assert float(widths[0].max()) <= eps
    assert np.array_equal(M.update_levels(geoms, grps, cam, eps, lev), lev)
    # a huge threshold coarsens by one level per frame, zero refines by one
    start = np.ones((G, S), np.int32)
    assert np.all(M.update_levels(geoms, grps, cam, np.inf, start) == 2)
    vis_w = widths[1] > 0
    up = M.update_levels(geoms, grps, cam, 0.0, start)
    assert np.all(up[vis_w] == 0) and np.all(up[~vis_w] == 2)


def test_uniform_levels_reproduce_single_level_shadowed_frames(scene):
    """A mixed frame's deep opacity map holds the frame's own rows: with one level everywhere
    the shadowed mixed frame is that level's shadowed frame (the rows in another order)."""
    asset, assigns, lods, cam, lights, geoms, grps = scene
    G, S = int(assigns[-1].max()) + 1, asset.segs
    mat = mat_of(asset)
    sh = (48, 3, 0.02)
    for l in (0, 2):
        mixed = M.mixed_geometry(geoms, grps, np.full((G, S), l, np.int32))
        a, _ = R.render(mixed, cam, lights, mat, shadow=sh)
        b, _ = R.render(geoms[l], cam, lights, mat, shadow=sh)
        assert np.allclose(a, b, rtol=1e-9, atol=1e-13), l
        plain, _ = R.render(geoms[l], cam, lights, mat)
        assert np.abs(a - plain).max() > 1e-6                # the map does shadow

