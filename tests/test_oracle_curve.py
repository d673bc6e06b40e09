"""Pins for curved thick hairs (oracle/curve.py): the Catmull-Rom basis (partition of unity,
interpolation, linear precision, the tangent (c_k+1 - c_k-1) / 2 at the control points and C1
joints), the tessellation count against brute force, and the reduction to the polyline
level when no segment is split."""
import math

import numpy as np

import hairsynth as hs
from oracle import curve as CV
from oracle import lod as OL
from oracle import render as R

F32 = np.float32


def test_basis_is_a_partition_of_unity_and_interpolates():
    u = np.linspace(0, 1, 101).astype(F32)
    w = CV.weights(u)
    assert np.allclose(sum(x.astype(np.float64) for x in w), 1.0, atol=3e-7)
    assert [float(x[0]) for x in w] == [0.0, 1.0, 0.0, 0.0]
    assert [float(x[-1]) for x in w] == [0.0, 0.0, 1.0, 0.0]
    c = np.random.default_rng(0).normal(size=(6, 3)).astype(F32)
    for k in range(5):
        assert np.array_equal(CV.point(c, k, F32(0.0)), c[k])
        assert np.array_equal(CV.point(c, k, F32(1.0)), c[k + 1])


def test_linear_precision_on_interior_segments():
    """Equally spaced collinear control points: P_k(u) = c_0 + (k + u) v (the spline
    reproduces straight lines), away from the clamped ends."""
    v = np.array([0.3, -0.2, 0.5])
    c = (np.arange(7)[:, None] * v[None, :]).astype(F32)
    for k in (1, 2, 3, 4):
        for u in np.linspace(0.05, 0.95, 19).astype(F32):
            p = CV.point(c, k, u).astype(np.float64)
            assert np.allclose(p, (k + float(u)) * v, atol=2e-6), (k, u)


def _deriv(c, k, u, h=1e-3):
    """Central difference of the spline in float64 (the basis evaluated in float64)."""
    def P(x):
        x2, x3 = x * x, x * x * x
        S = c.shape[0] - 1
        i = [min(max(k + d, 0), S) for d in (-1, 0, 1, 2)]
        w = (0.5 * ((2 * x2 - x3) - x), 0.5 * ((3 * x3 - 5 * x2) + 2), 0.5 * ((4 * x2 - 3 * x3) + x), 0.5 * (x3 - x2))
        return sum(wi * c[ii].astype(np.float64) for wi, ii in zip(w, i))
    return (P(u + h) - P(u - h)) / (2 * h)


def test_tangents_at_control_points_and_c1_joints():
    c = np.random.default_rng(1).normal(size=(7, 3)).astype(F32)
    for k in range(1, 5):
        t_end = _deriv(c, k, 1.0)
        t_start = _deriv(c, k + 1, 0.0)
        want = 0.5 * (c[k + 2].astype(np.float64) - c[k].astype(np.float64))
        assert np.allclose(t_end, want, atol=1e-5) and np.allclose(t_start, want, atol=1e-5)


def test_tessellation_count_matches_brute_force():
    asset = hs.make_asset(300, 8, 90.0, seed=5)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 20, seed=5))
    cam = hs.camera_for(asset, 256, 192)
    geom = R.cluster_level(lod)
    for max_px, max_sub in ((2, 16), (5, 4), (1, 16)):
        m = CV.tess_counts(geom, cam, max_px, max_sub)
        c = R.rs.cam_arrays(cam)
        XA, YA, _, _, okA = R.rs.project_points(geom.pA, c)
        XB, YB, _, _, okB = R.rs.project_points(geom.pB, c)
        for g in range(len(m)):
            if not (okA[g] and okB[g]):
                assert m[g] == 1
                continue
            L = math.hypot(int(XB[g]) - int(XA[g]), int(YB[g]) - int(YA[g])) / 16.0
            want = min(max_sub, max(1, math.ceil(L / max_px - 1e-12)))
            assert m[g] == want, (g, L, m[g], want)
        if max_px == 1:
            assert m.max() > 1


def test_no_split_reduces_to_the_polyline_level():
    asset = hs.make_asset(200, 6, 90.0, seed=6)
    lod = OL.build_level(asset, hs.kmeans_assign(asset, 12, seed=6))
    cam = hs.camera_for(asset, 128, 96)
    poly = R.cluster_level(lod)
    curved = CV.curved_geometry(lod, cam, 10 ** 6, 16)
    for f in ("pA", "pB", "ahat", "a_len", "b_len", "n_total", "r", "sigma_a"):
        assert np.array_equal(getattr(curved, f), getattr(poly, f)), f
    split = CV.curved_geometry(lod, cam, 1, 8)
    assert split.pA.shape[1] > poly.pA.shape[1]
    # consecutive rows of one segment share their joint; every segment's first and last row
    # start and end at its polyline vertices
    m = CV.tess_counts(poly, cam, 1, 8)
    start = np.concatenate([[0], np.cumsum(m)])
    for g in range(len(m)):
        rows = slice(start[g], start[g + 1])
        assert np.array_equal(split.pA[:, start[g]], poly.pA[:, g])
        assert np.array_equal(split.pB[:, start[g + 1] - 1], poly.pB[:, g])
        assert np.array_equal(split.pB[:, rows][:, :-1], split.pA[:, rows][:, 1:])
