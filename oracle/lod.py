"""Thick-hair (elliptical cluster) construction for one LoD level (oracle).

Paper Sec. 5.1 step 3 builds a thick hair per cluster from the k-th control points of its
member strands: their mean is the cross-section centre, a PCA fit gives an ellipse, the
axis nearest the tangent is dropped.  The reading taken here works per segment: the PCA is
the 2x2 covariance of the member segment midpoints in the plane orthogonal to the centre
segment's tangent, and each semi-axis is the hair radius plus twice the standard deviation
along it (a 2-sigma envelope), so a single-strand cluster is a circle of the strand's radius.

  centres c_k        = mean over members of vertex k: float64 sums in member-index order,
                       divided by the member count, rounded to float32.
  u                  = normalize(c_{k+1} - c_k) (float64 from the float32 centres).
  basis of u-perp    = e1 = normalize(e_j - (e_j . u) u) with j the axis of smallest |u_j|
                       (lowest index on ties), e2 = u x e1.
  covariance         = (1/N) sum_j q_j q_j^T, q_j = ((m_j - mbar) . e1, (m_j - mbar) . e2),
                       m_j member midpoints, mbar = (c_k + c_{k+1}) / 2.
  eigenpairs         = lambda_1 >= lambda_2 >= 0 (clamped), a^ = eigenvector of lambda_1 in
                       the basis; a^ = e1 when lambda_1 - lambda_2 <= 1e-12 (lambda_1 + lambda_2)
                       (a circle).
  |a|, |b|           = r + 2 sqrt(lambda_1), r + 2 sqrt(lambda_2).
  per cluster        = n_total = member count, sigma_a = member mean, r = mean width / 2.
"""
from __future__ import annotations

import numpy as np

KAPPA = 2.0    # semi-axis = r + KAPPA * standard deviation


def _sequential_member_sums(values, members_sorted, cluster_of, K):
    """sum over members (in ascending member order) of values[member], per cluster; float64.

    values: [n_strands, ...] float64.  Adds one member per cluster per step so the order is
    exactly the member-index order.
    """
    out = np.zeros((K,) + values.shape[1:], dtype=np.float64)
    counts = np.bincount(cluster_of, minlength=K)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    for j in range(int(counts.max()) if K else 0):
        cl = np.nonzero(counts > j)[0]
        out[cl] += values[members_sorted[starts[cl] + j]]
    return out, counts


def build_level(asset, assign: np.ndarray):
    """Cluster arrays for one level from a dense assignment in [0, K).

    Returns dict: centers f32 [K, V, 3]; ahat f32 [K, S, 3]; axes f32 [K, S, 2] (|a|, |b|);
    n_total i32 [K]; sigma_a f32 [3, K]; r f32 [K].
    """
    assign = np.asarray(assign, dtype=np.int64)
    K = int(assign.max()) + 1
    V = asset.verts_per_strand
    S = asset.segs
    members = np.argsort(assign, kind="stable")            # ascending strand index per cluster
    pts = asset.xyz.T.reshape(asset.n_strands, V, 3).astype(np.float64)
    sums, counts = _sequential_member_sums(pts, members, assign, K)
    if np.any(counts == 0):
        raise ValueError("assignment leaves an empty cluster")
    centers = (sums / counts[:, None, None]).astype(np.float32)
    wsum, _ = _sequential_member_sums(asset.width.astype(np.float64), members, assign, K)
    r = ((wsum / counts) * 0.5).astype(np.float32)
    ssum, _ = _sequential_member_sums(asset.sigma_a.T.astype(np.float64), members, assign, K)
    sigma_a = (ssum / counts[:, None]).astype(np.float32).T.copy()

    c64 = centers.astype(np.float64)
    ahat = np.zeros((K, S, 3), dtype=np.float32)
    axes = np.zeros((K, S, 2), dtype=np.float32)
    mid = 0.5 * (pts[:, :-1] + pts[:, 1:])                   # [n, S, 3]
    for k in range(S):
        t = c64[:, k + 1] - c64[:, k]
        u = t / np.linalg.norm(t, axis=1, keepdims=True)
        j = np.argmin(np.abs(u), axis=1)
        e = np.zeros_like(u)
        e[np.arange(K), j] = 1.0
        e1 = e - (e * u).sum(1, keepdims=True) * u
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(u, e1)
        mbar = 0.5 * (c64[:, k] + c64[:, k + 1])
        q = mid[:, k] - mbar[assign]
        q1 = (q * e1[assign]).sum(1)
        q2 = (q * e2[assign]).sum(1)
        prods = np.stack([q1 * q1, q1 * q2, q2 * q2], axis=1)
        csum, _ = _sequential_member_sums(prods, members, assign, K)
        cov = csum / counts[:, None]
        C = np.stack([np.stack([cov[:, 0], cov[:, 1]], -1), np.stack([cov[:, 1], cov[:, 2]], -1)], -2)
        lam, vec = np.linalg.eigh(C)                          # ascending eigenvalues
        l1 = np.maximum(lam[:, 1], 0.0)
        l2 = np.maximum(lam[:, 0], 0.0)
        v = vec[:, :, 1]
        circle = (l1 - l2) <= 1e-12 * (l1 + l2)
        v = np.where(circle[:, None], np.array([1.0, 0.0]), v)
        a_dir = v[:, :1] * e1 + v[:, 1:2] * e2
        ahat[:, k] = a_dir.astype(np.float32)
        r64 = r.astype(np.float64)
        axes[:, k, 0] = (r64 + KAPPA * np.sqrt(l1)).astype(np.float32)
        axes[:, k, 1] = (r64 + KAPPA * np.sqrt(l2)).astype(np.float32)
    return dict(centers=centers, ahat=ahat, axes=axes, n_total=counts.astype(np.int32),
                sigma_a=sigma_a, r=r)
