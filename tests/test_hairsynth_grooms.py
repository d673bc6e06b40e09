"""The synthetic groom generators (inputs only): the default random-walk groom is unchanged by
the lock option, locked grooms keep each lock together, and the path features give the
clustering metric of Sec. 5.1 step 1 (sum of squared distances between corresponding points)."""
import numpy as np

import hairsynth as hs


def test_default_groom_unchanged_by_the_lock_option():
    a = hs.make_asset(200, 8, 90.0, seed=3, sigma_spread=True)
    b = hs.make_asset(200, 8, 90.0, seed=3, sigma_spread=True, clumps=0, flow=0.5)
    assert np.array_equal(a.xyz, b.xyz) and np.array_equal(a.sigma_a, b.sigma_a)


def test_locked_groom_is_seeded_and_keeps_locks_together():
    n, segs, K = 1600, 16, 100
    a = hs.make_asset(n, segs, 90.0, seed=11, clumps=K, flow=0.99)
    b = hs.make_asset(n, segs, 90.0, seed=11, clumps=K, flow=0.99)
    assert np.array_equal(a.xyz, b.xyz)
    pts = a.xyz.reshape(3, n, segs + 1).transpose(1, 2, 0).astype(np.float64)
    lock = (np.arange(n) * K) // n
    # roots on the sphere of radius 0.1 and within the lock radius of the lock's mean root
    assert np.allclose(np.linalg.norm(pts[:, 0], axis=1), 0.1, atol=1e-6)
    for c in range(0, K, 7):
        m = pts[lock == c]
        assert np.linalg.norm(m[:, 0] - m[:, 0].mean(0), axis=1).max() < 2.5e-3
        # members advance 0.01 per step and stay within a few millimetres of each other
        assert np.allclose(np.linalg.norm(np.diff(m, axis=1), axis=2), 0.01, atol=1e-6)
        assert np.linalg.norm(m[:, -1] - m[:, -1].mean(0), axis=1).max() < 1e-2
    # the lock structure is what distinguishes it from the random walk: tips of one lock are far
    # closer together than tips of random strands
    r = hs.make_asset(n, segs, 90.0, seed=11)
    rp = r.xyz.reshape(3, n, segs + 1).transpose(1, 2, 0).astype(np.float64)
    assert np.linalg.norm(rp[:16, -1] - rp[:16, -1].mean(0), axis=1).max() > 3e-2


def test_path_features_give_the_summed_point_distance():
    a = hs.make_asset(50, 12, 90.0, seed=5)
    f = hs.strand_features(a, "path")
    assert f.shape == (50, 12)
    pts = a.xyz.reshape(3, 50, 13).transpose(1, 2, 0).astype(np.float64)
    idx = [0, 4, 8, 12]
    i, j = 3, 17
    want = sum(float(((pts[i, k] - pts[j, k]) ** 2).sum()) for k in idx)
    assert abs(float(((f[i] - f[j]) ** 2).sum()) - want) < 1e-12


def test_path_kmeans_recovers_locks():
    n, K = 3200, 200
    a = hs.make_asset(n, 16, 90.0, seed=2, clumps=K, flow=0.99)
    lab = hs.kmeans_assign(a, K, seed=2, iters=20, features="path")
    lock = (np.arange(n) * K) // n
    # each cluster is mostly one lock
    pure = [np.bincount(lock[lab == c]).max() / np.count_nonzero(lab == c) for c in range(int(lab.max()) + 1)]
    assert np.mean(pure) > 0.9
