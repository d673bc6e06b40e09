"""Pins for thick-hair construction, the one-strand LoD invariant, level selection and the
oracle gradient."""
import math

import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import grad as G
from oracle import lod as L
from oracle import render as R

MAT = (1.55, math.radians(-3.0), 0.3, 0.3)


def _asset_from(verts, width=80e-6, sigma=(0.3, 0.6, 1.2)):
    n, V, _ = verts.shape
    xyz = np.ascontiguousarray(verts.reshape(n * V, 3).T.astype(np.float32))
    return hs.Asset(n, V - 1, xyz, np.full(n, width, np.float32),
                    np.repeat(np.asarray(sigma, np.float32)[:, None], n, 1))


def test_centres_are_member_means():
    asset = hs.make_asset(300, 8, 90.0, seed=3)
    assign = hs.kmeans_assign(asset, 12, seed=5)
    lod = L.build_level(asset, assign)
    pts = asset.xyz.T.reshape(300, 9, 3).astype(np.float64)
    for c in range(lod["n_total"].size):
        m = pts[assign == c].mean(0)
        assert np.allclose(lod["centers"][c], m, rtol=0, atol=1e-7)
        assert lod["n_total"][c] == (assign == c).sum()
        assert np.allclose(lod["sigma_a"][:, c], asset.sigma_a[:, assign == c].mean(1), rtol=1e-6)


def test_known_cross_section_recovers_axes():
    """Four members at (0, +-s1, 0) and (0, 0, +-s2) around a straight x-axis centre line:
    covariance diag(s1^2 / 2, s2^2 / 2), so |a| = r + 2 s1 / sqrt 2 along y, |b| likewise."""
    s1, s2 = 2e-3, 0.5e-3
    xs = np.linspace(0, 0.05, 6)
    offs = [(0, s1, 0), (0, -s1, 0), (0, 0, s2), (0, 0, -s2)]
    verts = np.stack([np.stack([xs + o[0], np.full(6, o[1]), np.full(6, o[2])], -1) for o in offs])
    lod = L.build_level(_asset_from(verts), np.zeros(4, np.int32))
    r = 40e-6
    assert np.allclose(lod["axes"][0, :, 0], r + 2 * s1 / math.sqrt(2), rtol=1e-6)
    assert np.allclose(lod["axes"][0, :, 1], r + 2 * s2 / math.sqrt(2), rtol=1e-6)
    assert np.allclose(np.abs(lod["ahat"][0, :, 1]), 1.0, atol=1e-6)
    assert np.allclose(lod["r"], r)


def test_single_member_cluster_is_circle_of_radius_r():
    asset = hs.make_asset(5, 6, 60.0, seed=1)
    lod = L.build_level(asset, np.arange(5, dtype=np.int32))
    assert np.all(lod["axes"] == np.float32(40e-6))
    assert np.all(lod["n_total"] == 1)
    assert np.allclose(lod["centers"].reshape(-1, 3), asset.xyz.T)


def test_one_strand_lod_reproduces_strand_render():
    """A level with one strand per cluster renders like the strands themselves: the thick
    hair is a circle of the strand radius, n = 1, no B^ lobe, S = 1 (Sec. 4)."""
    asset, cam, lights = hs.config(1, scale=0.08)
    lod = L.build_level(asset, np.arange(asset.n_strands, dtype=np.int32))
    img_s, ras_s = R.render(R.strand_level(asset), cam, lights, MAT)
    img_c, ras_c = R.render(R.cluster_level(lod), cam, lights, MAT)
    same_cov = (len(ras_s.seg) == len(ras_c.seg)) and np.array_equal(ras_s.pix, ras_c.pix)
    if same_cov:
        assert np.array_equal(ras_s.seg, ras_c.seg) and np.array_equal(ras_s.key, ras_c.key)
        # the two half-widths agree to a float32 ulp, not bit for bit (different formulas)
        assert np.allclose(img_c, img_s, rtol=1e-4, atol=1e-9)
    else:       # a float32 half-width sitting on a 1/16-pixel boundary: report, compare the rest
        diff = np.abs(img_c - img_s) > 1e-9 + 1e-6 * np.abs(img_s)
        assert diff.any(axis=-1).mean() < 0.01
    assert len(ras_s.seg) > 100


def test_level_selection_rule():
    asset, cam, _ = hs.config(1, scale=0.1)
    geoms = [R.strand_level(asset)]
    for k in (30, 5, 1):
        geoms.append(R.cluster_level(L.build_level(asset, hs.kmeans_assign(asset, k, seed=2))))
    widths = []
    for g in geoms:
        _, _, _, _, _, _, _, hw, _, vis = R.segment_records(g, cam)
        widths.append(2 * float(hw[vis].max()))
    lvl = R.select_level(geoms, cam, eps_w=2.0)
    ok = [lv for lv in range(1, 4) if widths[lv] <= 2.0]
    assert lvl == (max(ok) if ok else 0)
    assert R.select_level(geoms, cam, eps_w=1e9) == 3
    assert R.select_level(geoms, cam, eps_w=0.0) == 0


def _small_cluster_scene(seed=11):
    asset = hs.make_asset(400, 6, 90.0, seed=seed, sigma_spread=True)
    cam = hs.camera_for(asset, 96, 80)
    lights = hs.default_lights(asset, with_point=True)
    assign = hs.kmeans_assign(asset, 8, seed=seed)
    lod = L.build_level(asset, assign)
    return asset, cam, lights, lod


def test_oracle_gradient_matches_central_differences():
    """P13: autograd VJP vs central differences (h = 1e-3 in log space, one Richardson
    step against the h^2 truncation term) on 20 parameters."""
    asset, cam, lights, lod = _small_cluster_scene()
    K, S = lod["n_total"].size, asset.segs
    geom = R.cluster_level(lod)
    ras = R.rasterize(geom, cam)
    assert len(ras.seg) > 200
    rng = np.random.default_rng(0)
    d_rgba = rng.normal(size=(cam.height, cam.width, 4))
    g_axes, g_r, g_sig, rgba = G.cluster_vjp(geom, cam, lights, MAT, d_rgba, K, S, ras=ras)
    axes = lod["axes"].astype(np.float64)
    r = lod["r"].astype(np.float64)
    sig = lod["sigma_a"].astype(np.float64)

    def loss(ax, rr, sg):
        return float((G.cluster_render_with(geom, cam, lights, MAT, K, S, ax, rr, sg, ras) * d_rgba).sum())

    picks = []
    for _ in range(12):
        picks.append(("axes", (rng.integers(K), rng.integers(S), rng.integers(2))))
    for _ in range(4):
        picks.append(("r", (rng.integers(K),)))
    for _ in range(4):
        picks.append(("sig", (rng.integers(3), rng.integers(K))))
    h = 1e-3
    checked = 0
    for kind, idx in picks:
        base = {"axes": axes, "r": r, "sig": sig}[kind]
        grad = {"axes": g_axes, "r": g_r, "sig": g_sig}[kind][idx]
        def central(step):
            vals = []
            for sgn in (1, -1):
                p = {"axes": axes.copy(), "r": r.copy(), "sig": sig.copy()}
                p[kind][idx] = base[idx] * math.exp(sgn * step)
                vals.append(loss(p["axes"], p["r"], p["sig"]))
            return (vals[0] - vals[1]) / (2 * step), vals[0]
        # central differences at h and h/2 in log space, one Richardson step (error O(h^4))
        f1, v0 = central(h)
        f2, _ = central(0.5 * h)
        fd = (4.0 * f2 - f1) / 3.0
        an = grad * base[idx]
        assert abs(fd - an) <= 1e-4 * max(1e-6, abs(an)) + 1e-7 * (abs(v0) + 1e-12) + 1e-9, (kind, idx, fd, an)
        checked += 1
    assert checked == 20
