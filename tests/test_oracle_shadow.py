"""Pins for the deep opacity map (oracle/shadow.py): light frame, grid coverage, the DOM
against brute force with Python integers, closed-form hair counts (thin strands stacked in a
texel column; a thick hair's chord count integrating to rho kappa times its cross-section
area), the layered lookup (bias, interpolation, continuity, monotonicity, bilinear), and the
shadowed render's reductions (no occluder: unchanged; an occluder: darker, and exactly the
f_ours forward attenuation)."""
import math

import numpy as np
import torch

import hairsynth as hs
from oracle import raster as rs
from oracle import render as R
from oracle import shadow as SH

F32 = np.float32


def test_light_basis_is_orthonormal_and_right_handed():
    for w in ([0.5, 0.6, 0.6], [0.0, 1.0, 0.0], [0.1, -0.95, 0.2], [1.0, 0.0, 0.0]):
        e1, e2, d, om = (x.astype(np.float64) for x in SH.light_basis(w))
        wn = np.asarray(w) / np.linalg.norm(w)
        assert np.allclose(om, wn, atol=1e-7) and np.allclose(d, -wn, atol=1e-7)
        for a, b in ((e1, e2), (e1, om), (e2, om)):
            assert abs(a @ b) < 1e-6
        for a in (e1, e2):
            assert abs(a @ a - 1.0) < 1e-6
        assert np.allclose(np.cross(e1, e2), om, atol=1e-6)


def _geom_strands(pA, pB, width):
    pA = np.asarray(pA, F32).T.copy()
    pB = np.asarray(pB, F32).T.copy()
    n = pA.shape[1]
    return R.LevelGeom("strand", pA, pB, np.zeros((n, 3), F32), width=np.full(n, width, F32))


def test_grid_holds_every_segment():
    asset, _, lights = hs.config(1, scale=0.3)
    geom = R.strand_level(asset)
    g = SH.dom_grid(geom, lights[0].vec, 128)
    XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = SH.light_records(geom, g)
    assert vis.all()
    for X in (XA, XB, YA, YB):
        assert X.min() >= 16 and X.max() <= 16 * 127
    assert izA.min() >= 1.0 and izB.min() >= 1.0


def _brute_dom(geom, omega, R, K, delta):
    """The DOM definition with Python integers for coverage and explicit loops."""
    g = SH.dom_grid(geom, omega, R)
    XA, YA, XB, YB, izA, izB, hw, hw_fx, vis = SH.light_records(geom, g)
    frags = {}
    for s in range(len(XA)):
        ax, ay, bx, by = int(XA[s]), int(YA[s]), int(XB[s]), int(YB[s])
        dx, dy = bx - ax, by - ay
        den = dx * dx + dy * dy
        Rr = int(hw_fx[s]) + 8
        for j in range(R):
            for i in range(R):
                ex, ey = 16 * i + 8 - ax, 16 * j + 8 - ay
                num = ex * dx + ey * dy
                cr = ex * dy - ey * dx
                if den > 0 and 0 <= num < den and cr * cr < Rr * Rr * den:
                    t = F32(num) / F32(den)
                    iz = F32(izA[s] + t * F32(izB[s] - izA[s]))
                    dl = abs(cr) / math.sqrt(den) / 16.0
                    h = float(hw[s])
                    alpha = min(max(min(dl + h, 0.5) - max(dl - h, -0.5), 0.0), 1.0)
                    frags.setdefault(j * R + i, []).append((iz, alpha))
    iz0 = np.zeros(R * R, F32)
    C = np.zeros((R * R, K))
    for q, fl in frags.items():
        top = max(f[0] for f in fl)
        iz0[q] = top
        for iz, a in fl:
            k = min(K - 1, int(math.floor(F32(F32(top - iz) / F32(delta)))))
            C[q, k:] += a
    return iz0, C


def test_dom_matches_brute_force():
    rng = np.random.default_rng(3)
    pA = rng.uniform(-0.05, 0.05, size=(7, 3))
    pB = pA + rng.normal(size=(7, 3)) * 0.03
    geom = _geom_strands(pA, pB, 4e-3)
    omega = [0.3, 0.5, 0.8]
    dom = SH.build_dom(geom, omega, 24, 3, 0.01)
    iz0, C = _brute_dom(geom, omega, 24, 3, 0.01)
    assert np.array_equal(dom.iz0.view(np.uint32), iz0.view(np.uint32))
    assert np.allclose(dom.C, C, rtol=1e-12, atol=1e-15)
    assert (iz0 > 0).sum() > 20 and C[:, -1].max() > 1.0


def test_stacked_thin_strands_count_their_coverage():
    """N thin strands along e1, one behind another toward the light, all through the same row
    of texel centres: every texel of that row holds N strands of box coverage w / s, and the
    layers split them by depth."""
    omega = np.array([0.0, 0.0, 1.0])
    e1, e2, d, _ = SH.light_basis(omega)
    e1, e2 = e1.astype(np.float64), e2.astype(np.float64)
    N, w, R = 5, 2e-4, 64
    anchors_A = [0.05 * e2 - 0.05 * e1, -0.05 * e2 - 0.05 * e1]
    anchors_B = [0.05 * e2 + 0.05 * e1, -0.05 * e2 + 0.05 * e1]
    g = SH.dom_grid(_geom_strands(anchors_A, anchors_B, w), omega, R)
    j = R // 2
    v = float(g["v0"]) + (j + 0.5) * float(g["s"])          # the centres of texel row j
    pA = [v * e2 - 0.04 * e1 - 0.02 * k * omega for k in range(N)]
    pB = [v * e2 + 0.04 * e1 - 0.02 * k * omega for k in range(N)]
    geom = _geom_strands(pA + anchors_A, pB + anchors_B, w)
    dom = SH.build_dom(geom, omega, R, 4, 0.015)
    assert dom.grid["s"] == g["s"] and dom.grid["v0"] == g["v0"]
    row = dom.C[j * R:(j + 1) * R]
    full = row[row[:, -1] > 0]
    s = float(g["s"])
    assert len(full) > R // 2
    assert np.allclose(full[:, -1], N * w / s, rtol=1e-5)
    # layers of depth 0.015 from the first strand: the strands sit 0.02 apart
    assert np.allclose(full[:, 0], w / s, rtol=1e-5)
    assert np.allclose(full[:, 1], 2 * w / s, rtol=1e-5)
    assert np.allclose(full[:, 2], 3 * w / s, rtol=1e-5)


def test_thick_hair_chord_count_integrates_to_area():
    """Across a thick hair seen edge-on by the light, sum_texels count * s = rho kappa pi |a||b|
    (the chord l_max sqrt(1 - h^2) integrates to the ellipse's area)."""
    omega = np.array([0.0, 0.0, 1.0])
    e1, e2, d, _ = SH.light_basis(omega)
    a, b, n_total, r = 0.004, 0.0025, 40, 4e-5
    ahat = e2.astype(np.float64)          # |a| across the light, |b| along it
    pA = (-0.05 * e1).astype(F32)[:, None]
    pB = (0.05 * e1).astype(F32)[:, None]
    geom = R.LevelGeom("cluster", pA, pB, np.zeros((1, 3), F32), ahat=ahat.astype(F32)[:, None],
                       a_len=np.array([a], F32), b_len=np.array([b], F32), n_total=np.array([n_total], np.int32),
                       r=np.array([r], F32))
    Rg = 160
    dom = SH.build_dom(geom, omega, Rg, 2, 1.0)
    g = dom.grid
    s = float(g["s"])
    col = int(Rg // 2)
    total = dom.C[col::Rg, -1].sum() * s
    rho = min(1.0, n_total * r * r / (a * b))
    kappa = math.sqrt(n_total / (math.pi * a * b))
    assert abs(total / (rho * kappa * math.pi * a * b) - 1.0) < 0.01


def _dom_one_texel(K=4, delta=0.1, C=(1.0, 3.0, 4.0, 6.0)):
    e1, e2, d, w = SH.light_basis([0.0, 0.0, 1.0])
    g = dict(e1=e1, e2=e2, d=d, omega=w, u0=F32(-1.5), v0=F32(-1.5), s=F32(1.0), k16=F32(16.0), z_ref=F32(10.0), R=3)
    iz0 = np.zeros(9, F32)
    Cm = np.zeros((9, K))
    iz0[4] = F32(9.0)          # centre texel: first hair at z = 1
    Cm[4] = C
    return SH.Dom(g, K, delta, iz0, Cm)


def _pt(u, v, z):
    e1, e2, d, _ = SH.light_basis([0.0, 0.0, 1.0])
    p = u * e1.astype(np.float64) + v * e2.astype(np.float64) + z * d.astype(np.float64)
    return p.astype(F32)[:, None]


def test_lookup_bias_interpolation_and_limits():
    dom = _dom_one_texel()
    n = lambda z: SH.dom_count(dom, _pt(0.0, 0.0, z))[0]
    close = lambda a, b: abs(a - b) < 1e-4    # float32 depths: z = 1 + x Delta to ~1e-6
    assert n(0.5) == 0.0                      # in front of the first hair
    assert n(1.05) == 0.0                     # inside the first layer: one layer of bias
    assert close(n(1.1), 0.0) and close(n(1.15), 0.5)   # half of layer 0 behind the bias
    assert close(n(1.2), 1.0) and close(n(1.25), 2.0)
    assert close(n(1.45), 5.0) and n(1.6) == 6.0 and n(5.0) == 6.0
    zs = np.linspace(0.0, 2.0, 2001)
    vals = np.array([n(z) for z in zs])
    assert np.all(np.diff(vals) >= -1e-9)                  # monotone in depth
    assert np.max(np.abs(np.diff(vals))) < 0.03             # continuous (slope <= 20 per unit)


def test_lookup_bilinear_between_texel_centres():
    dom = _dom_one_texel()
    dom.iz0[5] = F32(9.0)                     # the texel at +e1 holds 2 hairs
    dom.C[5] = (2.0, 2.0, 2.0, 2.0)
    z = 1.6                                   # saturated: texel values 6 and 2
    at = lambda u, v: SH.dom_count(dom, _pt(u, v, z))[0]
    assert abs(at(0.0, 0.0) - 6.0) < 1e-6     # the texel centre
    assert abs(at(0.5, 0.0) - 4.0) < 1e-5     # halfway to the +e1 neighbour
    assert abs(at(0.0, 0.5) - 3.0) < 1e-5     # halfway to an empty neighbour
    assert abs(at(-0.25, 0.25) - 6.0 * 0.75 * 0.75) < 1e-5
    assert abs(at(0.25, 0.25) - (6.0 * 0.75 + 2.0 * 0.25) * 0.75) < 1e-5
    assert at(0.0, 1.0) == 0.0 and at(5.0, 5.0) == 0.0


def test_shadowed_render_reductions():
    """One strand: its own DOM never shadows it (bias), so the shadowed render is the plain
    one.  A second strand between it and the light darkens it, and the darkened fragments are
    f_ours with n_F = 1 + n_s."""
    omega = np.array([0.0, 0.0, 1.0], np.float32)
    light = hs.Light(0, omega, np.ones(3, F32))
    cam = hs.Camera(np.array([0.0, 0.0, 1.0], F32), np.eye(3, dtype=F32), 400.0, 400.0, 32.0, 32.0, 64, 64, 0.01)
    back = _geom_strands([[-0.05, 0.0, 0.0]], [[0.05, 0.001, 0.0]], 2e-3)
    mat = (1.55, math.radians(-3.0), 0.3, 0.3)
    a, _ = R.render(back, cam, [light], mat)
    b, _ = R.render(back, cam, [light], mat, shadow=(64, 4, 0.01))
    assert np.array_equal(a, b)
    both = _geom_strands([[-0.05, 0.0, 0.0], [0.0, -0.05, 0.05]], [[0.05, 0.001, 0.0], [0.001, 0.05, 0.05]], 2e-3)
    ras = R.rasterize(both, cam)
    ns = SH.shadow_counts(both, ras, cam, [light], 64, 4, 0.01)[0]
    shaded = ns > 0
    assert shaded.any() and bool(np.all(ras.seg[shaded.numpy()] == 0))
    _, L0 = R.fragment_radiance(both, ras, cam, [light], mat)
    _, L1 = R.fragment_radiance(both, ras, cam, [light], mat, shadow=[ns])
    assert torch.all(L1[shaded].sum(-1) < L0[shaded].sum(-1))
    assert torch.equal(L1[~shaded], L0[~shaded])
