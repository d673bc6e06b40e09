"""Seeded synthetic hair workloads shared by the oracle tests, the GPU tests and the benchmark.

This module only *makes inputs*: strand polylines, per-strand width and absorption, the
cluster assignment fed to the LoD builder, cameras and lights.  It holds none of the
rendering method's arithmetic (no projection, coverage, scattering or compositing), so both
the CPU oracle and the HIP path can consume its arrays without sharing method code.

The paper measures on artist and captured grooms that are not available here; these
generators stand in for them with the shapes and scales the paper describes (tens of
thousands to a few hundred thousand strands, 16-64 segments each, roots on a scalp-like
sphere cap, 1024^2-class images; paper Sec. 6 "Hairstyles", "Real-time performance").

Recipe (all float64, stored float32):
  * rng = numpy Generator(PCG64(seed)); draws in this order: U[n], V[n] for the roots,
    then for each step (step-major, all strands at once) a standard normal (n, 3) block,
    then (optionally) one standard normal z[n] for the absorption spread.
  * roots on a sphere cap of radius 0.1 about +y, area-uniform:
    cos(theta) = 1 - U (1 - cos(cap)), azimuth = 2 pi V; first direction = outward normal.
  * per step: d <- normalize(d + 0.3 N(0, I3) + (0, -0.2, 0)); x <- x + 0.01 d.
  * width 80e-6 m (a diameter); sigma_a = (0.3, 0.6, 1.2), optionally times exp(0.2 z).
  * material: eta 1.55, longitudinal shift -3 deg, beta_m = beta_n = 0.3 rad.

Clumped grooms (make_asset(..., clumps=K)): strands in K locks that follow a guide, the
structure of combed or styled hair.  Draws: U[K], V[K] for the guide roots (the cap as above),
then R[n], A[n] for the members' root offsets, then per step a standard normal (K, 3) block
for the guides followed by a standard normal (n, 3) block for the members, then the optional
absorption spread z[n].  Strand s belongs to lock s * K // n (consecutive strands share a
lock); its root is the guide's root plus an offset of radius clump_radius sqrt(R) at angle
2 pi A in the guide root's tangent plane, put back on the sphere of radius 0.1; it starts
along its own outward normal.  Per step the guide turns as above, and each member takes the
guide's new direction plus clump_noise N(0, I3), normalised, and advances 0.01.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Material", "Asset", "Camera", "Light", "make_asset", "kmeans_assign",
    "camera_for", "ring_cameras", "default_lights", "config", "CONFIGS",
]


@dataclass
class Material:
    """Fibre material.  model 0: near-field R / TT / TRT (eta, alpha, beta_m, beta_n and the
    strands' absorption); model 1: R / TT / D with constant attenuations, defaults inside the
    paper's stated ranges (Sec. 6: beta_R 0.08-0.15, beta_TT 0.12-0.3, gamma_TT 0.2-0.4,
    A_R 0.03-0.25, A_TT (0.25, 0.17, 0.07)-(0.38, 0.25, 0.18), A_D (0.2, 0.11, 0.1)-(0.4, 0.21, 0.08))."""
    eta: float = 1.55
    alpha: float = math.radians(-3.0)   # longitudinal shift (radians)
    beta_m: float = 0.3                  # longitudinal width (radians, std dev)
    beta_n: float = 0.3                  # azimuthal width (radians, std dev)
    model: int = 0
    beta_r: float = 0.1
    beta_tt: float = 0.2
    gamma_tt: float = 0.3
    a_r: tuple = (0.1, 0.1, 0.1)
    a_tt: tuple = (0.3, 0.2, 0.12)
    a_d: tuple = (0.3, 0.16, 0.09)

    @classmethod
    def rttd(cls, **kw) -> "Material":
        return cls(model=1, **kw)

    def as_array(self) -> np.ndarray:
        return np.array([self.eta, self.alpha, self.beta_m, self.beta_n], dtype=np.float32)


@dataclass
class Asset:
    """Strand polylines in structure-of-arrays form.

    xyz:     float32 [3, n_strands * (segs + 1)]  (x row, y row, z row), world metres.
             Vertex k of strand s sits at column s * (segs + 1) + k.
    width:   float32 [n_strands]  fibre diameter (m).
    sigma_a: float32 [3, n_strands] absorption per unit fibre radius (RGB rows).
    """
    n_strands: int
    segs: int
    xyz: np.ndarray
    width: np.ndarray
    sigma_a: np.ndarray
    material: Material = field(default_factory=Material)

    @property
    def verts_per_strand(self) -> int:
        return self.segs + 1

    @property
    def n_segments(self) -> int:
        return self.n_strands * self.segs

    def roots(self) -> np.ndarray:
        v = self.verts_per_strand
        return self.xyz[:, 0::v].T.astype(np.float64)

    def first_tangents(self) -> np.ndarray:
        v = self.verts_per_strand
        d = (self.xyz[:, 1::v] - self.xyz[:, 0::v]).T.astype(np.float64)
        return d / np.linalg.norm(d, axis=1, keepdims=True)

    def aabb(self):
        """(min, max) corners of the vertices, float64; cached per vertex array (assets are not
        modified in place)."""
        c = self.__dict__.get("_aabb_cache")
        if c is None or c[0] is not self.xyz:
            c = (self.xyz, self.xyz.min(axis=1).astype(np.float64), self.xyz.max(axis=1).astype(np.float64))
            self.__dict__["_aabb_cache"] = c
        return c[1], c[2]


@dataclass
class Camera:
    """Pinhole camera. rot is row-major world->view; the view looks along -z, y up.

    Pixel (i, j) has its centre at (i + 0.5, j + 0.5); x grows right, y grows down.
    """
    pos: np.ndarray          # float32 [3]
    rot: np.ndarray          # float32 [3, 3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.01

    def packed(self) -> np.ndarray:
        """float32[18]: pos(3) rot(9) fx fy cx cy z_near pad  (W, H travel as ints)."""
        out = np.zeros(18, dtype=np.float32)
        out[0:3] = self.pos
        out[3:12] = np.asarray(self.rot, dtype=np.float32).reshape(9)
        out[12:17] = (self.fx, self.fy, self.cx, self.cy, self.z_near)
        return out


@dataclass
class Light:
    kind: int                # 0 = directional (vec = unit direction toward the light), 1 = point (vec = position)
    vec: np.ndarray          # float32 [3]
    rgb: np.ndarray          # float32 [3]: irradiance E (directional) or intensity I (point)


def _normalize(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def make_asset(n_strands: int, segs: int, cap_deg: float = 90.0, seed: int = 0,
               sigma_spread: bool = False, material: Material | None = None, clumps: int = 0,
               clump_radius: float = 1e-3, clump_noise: float = 0.02, flow: float = 0.0) -> Asset:
    if clumps > 0:
        return _make_clumped(n_strands, segs, cap_deg, seed, sigma_spread, material, clumps, clump_radius,
                             clump_noise, flow)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(n_strands)
    U = rng.random(n)
    V = rng.random(n)
    cos_cap = math.cos(math.radians(cap_deg))
    cos_t = 1.0 - U * (1.0 - cos_cap)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    az = 2.0 * math.pi * V
    normal = np.stack([sin_t * np.cos(az), cos_t, sin_t * np.sin(az)], axis=1)
    x = 0.1 * normal
    d = normal.copy()
    verts = np.empty((n, segs + 1, 3), dtype=np.float64)
    verts[:, 0] = x
    drift = np.array([0.0, -0.2, 0.0])
    for k in range(segs):
        d = _normalize(d + 0.3 * rng.standard_normal((n, 3)) + drift)
        x = x + 0.01 * d
        verts[:, k + 1] = x
    xyz = np.ascontiguousarray(verts.reshape(n * (segs + 1), 3).T.astype(np.float32))
    width = np.full(n, 80e-6, dtype=np.float32)
    base = np.array([0.3, 0.6, 1.2])
    if sigma_spread:
        z = rng.standard_normal(n)
        sig = base[:, None] * np.exp(0.2 * z)[None, :]
    else:
        sig = np.repeat(base[:, None], n, axis=1)
    return Asset(n, segs, xyz, width, np.ascontiguousarray(sig.astype(np.float32)),
                 material or Material())


def _cap_points(U: np.ndarray, V: np.ndarray, cap_deg: float) -> np.ndarray:
    cos_cap = math.cos(math.radians(cap_deg))
    cos_t = 1.0 - U * (1.0 - cos_cap)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    az = 2.0 * math.pi * V
    return np.stack([sin_t * np.cos(az), cos_t, sin_t * np.sin(az)], axis=1)


def _make_clumped(n_strands, segs, cap_deg, seed, sigma_spread, material, clumps, clump_radius, clump_noise,
                  flow=0.0, flow_modes=8, flow_wavelength=0.15):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(n_strands)
    K = max(1, min(int(clumps), n))
    gU = rng.random(K)
    gV = rng.random(K)
    g_normal = _cap_points(gU, gV, cap_deg)
    R = rng.random(n)
    A = rng.random(n)
    if flow > 0.0:   # a smooth random field over the scalp: flow_modes plane waves per step
        w_dir = _normalize(rng.standard_normal((flow_modes, 3)))
        w_amp = rng.standard_normal((segs, flow_modes, 3)) / math.sqrt(flow_modes)
        w_phase = 2.0 * math.pi * rng.random((segs, flow_modes))
        w_proj = (0.1 * g_normal) @ w_dir.T * (2.0 * math.pi / flow_wavelength)   # [K, modes]
    lock = (np.arange(n, dtype=np.int64) * K) // n
    # an orthonormal tangent frame at each guide root
    ref = np.where(np.abs(g_normal[:, 1:2]) < 0.9, np.array([[0.0, 1.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    t1 = _normalize(np.cross(g_normal, ref))
    t2 = np.cross(g_normal, t1)
    rad = clump_radius * np.sqrt(R)
    ang = 2.0 * math.pi * A
    root = 0.1 * g_normal[lock] + (rad * np.cos(ang))[:, None] * t1[lock] + (rad * np.sin(ang))[:, None] * t2[lock]
    normal = _normalize(root)
    x = 0.1 * normal
    d = normal.copy()
    dg = g_normal.copy()
    verts = np.empty((n, segs + 1, 3), dtype=np.float64)
    verts[:, 0] = x
    drift = np.array([0.0, -0.2, 0.0])
    for k in range(segs):
        noise = rng.standard_normal((K, 3))
        if flow > 0.0:
            smooth = np.cos(w_proj + w_phase[k][None, :]) @ w_amp[k]                    # [K, 3]
            noise = math.sqrt(1.0 - flow * flow) * noise + flow * math.sqrt(2.0) * smooth
        dg = _normalize(dg + 0.3 * noise + drift)
        d = _normalize(dg[lock] + clump_noise * rng.standard_normal((n, 3)))
        x = x + 0.01 * d
        verts[:, k + 1] = x
    xyz = np.ascontiguousarray(verts.reshape(n * (segs + 1), 3).T.astype(np.float32))
    width = np.full(n, 80e-6, dtype=np.float32)
    base = np.array([0.3, 0.6, 1.2])
    if sigma_spread:
        z = rng.standard_normal(n)
        sig = base[:, None] * np.exp(0.2 * z)[None, :]
    else:
        sig = np.repeat(base[:, None], n, axis=1)
    return Asset(n, segs, xyz, width, np.ascontiguousarray(sig.astype(np.float32)),
                 material or Material())


def kmeans_assign(asset: Asset, k: int, seed: int, iters: int = 25, init: str = "kmeans++",
                  features: str = "root") -> np.ndarray:
    """Cluster assignment used as the LoD builder's input (int32 [n_strands], dense labels).

    Features (float64): "root" = [root / 0.1, first-segment tangent] (6-D); "path" = the
    positions of 4 vertices evenly spaced along the strand (root to tip, 12-D), so that the
    squared feature distance is the sum of squared distances between corresponding points of
    two strands (the clustering metric of Sec. 5.1 step 1 with 4 control points).  Seeding drawn from
    PCG64(seed): k-means++ (default) or, for large k, k distinct random strands
    (init="random"); then `iters` Lloyd iterations; distance ties go to the lower centre
    index (argmin; above 512 centres a k-d tree finds the exact nearest centre); empty
    clusters are dropped and labels renumbered densely in order.
    """
    return _kmeans(strand_features(asset, features), k, seed, iters, init)


def strand_features(asset: Asset, features: str = "root") -> np.ndarray:
    if features == "path":
        v = asset.verts_per_strand
        pts = asset.xyz.reshape(3, asset.n_strands, v).astype(np.float64)
        idx = np.round(np.linspace(0, v - 1, 4)).astype(np.int64)
        return np.ascontiguousarray(pts[:, :, idx].transpose(1, 2, 0).reshape(asset.n_strands, 12))
    return np.concatenate([asset.roots() / 0.1, asset.first_tangents()], axis=1)


def kmeans_hierarchy(asset: Asset, ks, seed: int, iters: int = 25, init: str = "kmeans++",
                     features: str = "root") -> list:
    """Nested assignments for the levels finer -> coarser (ks descending): the finest level is
    k-means on the strand features; each coarser level is k-means on the previous level's
    cluster mean features, so every cluster lies inside one cluster of each coarser level."""
    feats = strand_features(asset, features)
    lab = _kmeans(feats, ks[0], seed, iters, init)
    out = [lab]
    for li, k in enumerate(ks[1:], start=1):
        K = int(lab.max()) + 1
        cnt = np.bincount(lab, minlength=K).astype(np.float64)
        cf = np.zeros((K, feats.shape[1]))
        np.add.at(cf, lab, feats)
        cf /= cnt[:, None]
        top = _kmeans(cf, k, seed + li, iters, init)
        lab = top[lab].astype(np.int32)
        out.append(lab)
    return out


def _kmeans(feats: np.ndarray, k: int, seed: int, iters: int, init: str) -> np.ndarray:
    n = feats.shape[0]
    k = min(int(k), n)
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = np.empty((k, feats.shape[1]))
    if init == "random":
        centres[:] = feats[np.sort(rng.choice(n, size=k, replace=False))]
    else:
        first = int(rng.integers(n))
        centres[0] = feats[first]
        d2 = ((feats - centres[0]) ** 2).sum(1)
        for c in range(1, k):
            tot = d2.sum()
            if tot <= 0.0:
                idx = int(rng.integers(n))
            else:
                r = rng.random() * tot
                idx = int(np.searchsorted(np.cumsum(d2), r, side="right"))
                idx = min(idx, n - 1)
            centres[c] = feats[idx]
            d2 = np.minimum(d2, ((feats - centres[c]) ** 2).sum(1))

    def assign(cent):
        if k > 512:   # exact nearest centre through a k-d tree (same result up to exact ties)
            from scipy.spatial import cKDTree
            return cKDTree(cent).query(feats, k=1, workers=-1)[1].astype(np.int64)
        lab = np.empty(n, dtype=np.int64)
        cn = (cent ** 2).sum(1)
        step = max(1, int(2e7 // max(1, k)))
        for s in range(0, n, step):
            f = feats[s:s + step]
            dist = (f ** 2).sum(1)[:, None] - 2.0 * f @ cent.T + cn[None, :]
            lab[s:s + step] = np.argmin(dist, axis=1)
        return lab

    lab = assign(centres)
    for _ in range(iters):
        cnt = np.bincount(lab, minlength=k).astype(np.float64)
        sums = np.zeros_like(centres)
        np.add.at(sums, lab, feats)
        nz = cnt > 0
        centres[nz] = sums[nz] / cnt[nz, None]
        lab = assign(centres)
    used = np.unique(lab)
    remap = np.full(k, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return remap[lab].astype(np.int32)


def _look_at(pos: np.ndarray, target: np.ndarray) -> np.ndarray:
    back = _normalize(pos - target)
    up = np.array([0.0, 1.0, 0.0])
    right = _normalize(np.cross(up, back))
    up2 = np.cross(back, right)
    return np.stack([right, up2, back])


def camera_for(asset: Asset, width: int, height: int, azimuth: float = 0.0,
               fill: float = 0.9, fov_y_deg: float = 30.0) -> Camera:
    """Frame the asset's AABB: its bounding sphere spans `fill` of the half-height."""
    lo, hi = asset.aabb()
    centre = 0.5 * (lo + hi)
    radius = 0.5 * float(np.linalg.norm(hi - lo))
    half = math.radians(fov_y_deg) / 2.0
    dist = radius / (fill * math.tan(half))
    pos = centre + dist * np.array([math.sin(azimuth), 0.0, math.cos(azimuth)])
    rot = _look_at(pos, centre)
    fy = (height / 2.0) / math.tan(half)
    return Camera(pos.astype(np.float32), rot.astype(np.float32), float(np.float32(fy)),
                  float(np.float32(fy)), width / 2.0, height / 2.0, width, height, 0.01)


def camera_occupancy(asset: Asset, width: int, height: int, occupancy: float, azimuth: float = 0.0) -> Camera:
    """Camera whose projected bounding sphere covers `occupancy` of the image area."""
    fill = math.sqrt(occupancy * width * height / math.pi) / (height / 2.0)
    return camera_for(asset, width, height, azimuth=azimuth, fill=fill)


def ring_cameras(asset: Asset, n: int, width: int, height: int) -> list[Camera]:
    return [camera_for(asset, width, height, azimuth=2.0 * math.pi * k / n) for k in range(n)]


def default_lights(asset: Asset, with_point: bool) -> list[Light]:
    lo, hi = asset.aabb()
    centre = 0.5 * (lo + hi)
    d = np.array([0.5, 0.6, 0.6])
    d = d / np.linalg.norm(d)
    lights = [Light(0, d.astype(np.float32), np.ones(3, dtype=np.float32))]
    if with_point:
        p = centre + np.array([-0.3, 0.1, -0.4])
        lights.append(Light(1, p.astype(np.float32), np.full(3, 0.25, dtype=np.float32)))
    return lights


# The five workloads, numbered (the number also offsets the generator seed: 1000 + n).  Sizes
# follow the paper's scales (Sec. 6); the generator recipe is above.
CONFIGS = {
    # 1: small frame, 1k strands x 16 segments at 256x256, one directional light
    1: dict(strands=1_000, segs=16, cap=60.0, res=(256, 256), point=False, spread=False),
    # 2: full frame, 100k strands x 32 segments at 1920x1080, directional + point light
    2: dict(strands=100_000, segs=32, cap=90.0, res=(1920, 1080), point=True, spread=True),
    # 3: LoD sweep, 150k strands x 64 segments at 1080p with 10k / 1k / 100 thick hairs
    3: dict(strands=150_000, segs=64, cap=90.0, res=(1920, 1080), point=True, spread=True,
            levels=(10_000, 1_000, 100)),
    # 4: fitting, 50k strands x 32 segments -> 500 thick hairs, 8 views at 512x512
    4: dict(strands=50_000, segs=32, cap=90.0, res=(512, 512), point=False, spread=False,
            levels=(500,), views=8),
    # 5: serving, three resident assets at 720p / 1080p / 2160p
    5: dict(assets=((10_000, 16), (100_000, 32), (300_000, 48)), cap=90.0, point=True, spread=True,
            resolutions=((1280, 720), (1920, 1080), (3840, 2160))),
}


def config(cfg: int, scale: float = 1.0):
    """(asset, camera, lights) for workloads 1-4; `scale` shrinks the strand count for tests."""
    c = CONFIGS[cfg]
    n = max(1, int(round(c["strands"] * scale)))
    asset = make_asset(n, c["segs"], c["cap"], seed=1000 + cfg, sigma_spread=c["spread"])
    w, h = c["res"]
    cam = camera_for(asset, w, h)
    return asset, cam, default_lights(asset, c["point"])
