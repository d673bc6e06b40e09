"""Pins for the aggregated thick-hair scattering function (oracle/aggregate.py)."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import aggregate as ag
from oracle import fiber as fb

T = lambda x: torch.as_tensor(x, dtype=torch.float64)
MAT = (1.55, math.radians(-3.0), 0.3, 0.3)
SIG = torch.tensor([[0.3, 0.6, 1.2]], dtype=torch.float64)


def test_printed_constants():
    assert ag.D_1PLUS == 0.6          # Sec. 4, d_1+
    assert ag.C_M == 0.2              # Sec. 4, c_m


def test_front_mass_matches_quadrature():
    s = fb.logistic_scale(0.3)
    for mu in (-3.0, -1.6, -0.4, 0.0, 0.9, 1.57, 2.8, 5.0, -7.0):
        val = 0.0
        for a, b in ((-math.pi, -math.pi / 2), (math.pi / 2, math.pi)):
            kink = [k for k in ((mu + math.pi) % (2 * math.pi) - math.pi, mu % (2 * math.pi) - math.pi) if a < k < b]
            v, _ = integrate.quad(lambda x: float(fb.trimmed_logistic(fb.wrap_pi(T(x - mu)), s)), a, b, limit=200,
                                  epsabs=1e-14, epsrel=1e-12, points=kink or None)
            val += v
        assert abs(val - float(ag.front_mass(T(mu), s))) < 1e-10, mu


def test_hemisphere_albedos_match_dense_h_quadrature():
    """a_F + a_B is the h-averaged total albedo; 8-node GL agrees with dense quadrature."""
    x = T([0.1, 0.6, 1.1])
    sig = SIG.expand(3, 3)
    a_F, a_B, var_f, var_b = ag.hemisphere_stats(x, sig, MAT)
    hs = np.linspace(-1, 1, 4001)
    for i in range(3):
        A, go, gt = fb.attenuation(T(np.full_like(hs, float(x[i]))), T(hs), sig[i:i + 1].expand(len(hs), 3), 1.55)
        s = fb.logistic_scale(0.3)
        PF = torch.stack([ag.front_mass(fb.exit_azimuth(p, go, gt), s) for p in range(3)], -1)
        front = (A * PF[..., None]).sum(-2).numpy()
        ref = 0.5 * np.trapezoid(front, hs, axis=0)
        assert np.allclose(a_F[i].numpy(), ref, rtol=2.5e-2)   # 8 nodes vs the sqrt edge at |h| -> 1
        tot = 0.5 * np.trapezoid(A.sum(-2).numpy(), hs, axis=0)
        assert np.allclose((a_F[i] + a_B[i]).numpy(), tot, rtol=2.5e-2)
    assert torch.all((a_F > 0) & (a_F < 1) & (a_B > 0))
    b_p = fb.lobe_shifts_widths(MAT[1], MAT[2])[1]
    lo, hi = min(b_p) ** 2, max(b_p) ** 2
    assert torch.all((var_f >= lo) & (var_f <= hi) & (var_b >= lo) & (var_b <= hi))


def test_a1plus_closed_form_equals_explicit_sum():
    """A_1+ = d_1+ a_B sum_{i=1..n} a_F^{2i-1} (Sec. 4) at integer n."""
    a_F = T([[0.3, 0.5, 0.8]])
    a_B = T([[0.2, 0.1, 0.05]])
    for n in (1, 2, 3, 7):
        AB, _ = ag.back_lobe(a_F, a_B, T([0.01]), T([0.02]), T([float(n)]))
        explicit = sum(a_F ** (2 * i - 1) for i in range(1, n + 1)) * a_B * 0.6
        A1 = a_B * a_F ** 2 / (1 - a_F ** 2)
        A3 = a_B ** 3 * a_F ** 2 / (1 - a_F ** 2) ** 3
        assert torch.allclose(AB, explicit + A1 + A3, rtol=1e-12)


def test_a1_a3_are_dual_scattering_path_series():
    """The closed forms are the dual-scattering path series (Sec. 3.2): A_1 sums one
    backward event with 2k >= 2 forward events, a_B sum_k a_F^{2k}; A_3 sums three backward
    events, a_B^3 sum_j j (j + 1) / 2 a_F^{2j} (a triangular count of forward-pair
    placements).  Guards the exponents of the closed forms against slips."""
    aF, aB = 0.7, 0.15
    A1_series = sum(aB * aF ** (2 * k) for k in range(1, 400))
    A3_series = aB ** 3 * sum(0.5 * j * (j + 1) * aF ** (2 * j) for j in range(1, 600))
    AB, _ = ag.back_lobe(T([[aF] * 3]), T([[aB] * 3]), T([0.0]), T([0.0]), T([1.0]))
    A1p = 0.6 * aB * aF
    assert abs(float(AB[0, 0]) - (A1p + A1_series + A3_series)) < 1e-12


def test_shadowing_masking_reductions():
    phi = T([0.0, 0.4, -1.2, 2.0])
    n_total = T([5.0, 5.0, 5.0, 5.0])
    a_F = T([[0.4, 0.5, 0.6]] * 4)
    # phi = 0 => S = 1 - c_m (1 - rho)
    S = ag.shadowing_masking(phi, T([0.3] * 4), a_F, n_total)
    assert torch.allclose(S[0], T([1 - 0.2 * 0.7] * 3))
    # rho = 1 => S = 1
    assert torch.allclose(ag.shadowing_masking(phi, T([1.0] * 4), a_F, n_total), torch.ones(4, 3, dtype=torch.float64))
    # front hemisphere and single hairs => S = 1
    assert torch.allclose(S[3], torch.ones(3, dtype=torch.float64))
    S1 = ag.shadowing_masking(phi, T([0.3] * 4), a_F, T([1.0] * 4))
    assert torch.allclose(S1, torch.ones(4, 3, dtype=torch.float64))
    # P_n clamps at zero: rho = 0, phi near pi/2 => S = P_s a_F
    S2 = ag.shadowing_masking(T([1.5]), T([0.0]), a_F[:1], T([5.0]))
    assert torch.allclose(S2, (1 - math.cos(1.5)) * a_F[:1])


def _random_dirs(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_single_hair_cluster_reduces_to_single_fibre():
    """n_total = 1: n = 1, A_B^ = 0, S = 1, so f_ours = f_single (Sec. 4: 'exactly the same
    as their counterparts in the single hair BCSDF')."""
    rng = np.random.default_rng(0)
    n = 64
    th = T(rng.uniform(-1.2, 1.2, n))
    xd = T(rng.uniform(0, 1.2, n))
    phi = T(rng.uniform(-math.pi, math.pi, n))
    h = T(rng.uniform(-1, 1, n))
    sig = SIG.expand(n, 3)
    one = torch.ones(n, dtype=torch.float64)
    fo = ag.f_ours(th, xd, phi, h, sig, MAT, one, T(rng.uniform(0, 1, n)), one, T(rng.uniform(1, 5, n)))
    fs = fb.f_single(th, xd, phi, h, sig, MAT)
    assert torch.allclose(fo, fs, rtol=1e-13, atol=0)


def test_back_hemisphere_has_n_equal_one():
    phi = T([0.3, -1.0, 2.0, -2.9])
    rho, nF, nB = ag.hair_counts(phi, T([0.02, 0.02, 0.02, 0.02]), T([50.0] * 4), T([4e-5] * 4),
                                 T([1e-3] * 4), T([5e-4] * 4))
    assert torch.equal(nF[:2], torch.ones(2, dtype=torch.float64))
    assert torch.all(nF[2:] > 1.0)
    # rho is the hair area fraction: n pi r^2 / (pi |a| |b|)
    assert torch.allclose(rho, T([50 * math.pi * 16e-10 / (math.pi * 5e-7)] * 4))


def _march_chord(P, D, a, b, step):
    """Brute force: walk from P along D until the point leaves the ellipse."""
    s = step
    while True:
        q = P + s * D
        if (q[0] / a) ** 2 + (q[1] / b) ** 2 > 1.0:
            return s - 0.5 * step
        s += step


def test_chord_against_brute_force_march():
    rng = np.random.default_rng(7)
    for a, b in ((4.0, 1.0), (1.0, 1.0), (2.5, 1.7)):            # 4:1 ellipse of the ablation
        ahat = np.array([1.0, 0.0, 0.0]); bhat = np.array([0.0, 1.0, 0.0])
        for _ in range(12):
            ang = rng.uniform(0, 2 * math.pi)
            xh = np.array([math.cos(ang), math.sin(ang), 0.0])
            yh = np.array([-math.sin(ang), math.cos(ang), 0.0])
            h = rng.uniform(-0.95, 0.95)
            W = float(ag.ellipse_support(T(a), T(b), T(ahat), T(bhat), T(yh)))
            dang = rng.uniform(0, 2 * math.pi)
            D = np.array([math.cos(dang), math.sin(dang), 0.0])
            s_star = float(ag.ellipse_chord(T(h), T(W), T(xh), T(yh), T(ahat), T(bhat), T(a), T(b), T(D)))
            # entry point: first hit of the line h W yh - t xh with the ellipse, by dense scan
            ts = np.linspace(-10, 10, 400001)
            pts = h * W * yh[None, :2] - ts[:, None] * xh[None, :2]
            inside = (pts[:, 0] / a) ** 2 + (pts[:, 1] / b) ** 2 <= 1.0
            assert inside.any()
            P = pts[np.argmax(inside)]
            if s_star > 1e-6:
                assert abs(_march_chord(P, D[:2], a, b, 1e-5 * a) - s_star) < 2e-3 * a
            elif s_star < -1e-6:
                assert abs(_march_chord(P, -D[:2], a, b, 1e-5 * a) + s_star) < 2e-3 * a


def test_chord_circle_closed_form():
    R = 1.3
    for h in (-0.8, 0.0, 0.5):
        for dang in (0.3, 2.0, 4.0):
            ahat = np.array([1.0, 0.0, 0.0]); bhat = np.array([0.0, 1.0, 0.0])
            xh = np.array([1.0, 0.0, 0.0]); yh = np.array([0.0, 1.0, 0.0])
            D = np.array([math.cos(dang), math.sin(dang), 0.0])
            s = float(ag.ellipse_chord(T(h), T(R), T(xh), T(yh), T(ahat), T(bhat), T(R), T(R), T(D)))
            P = np.array([math.sqrt(R * R - (h * R) ** 2), h * R])
            q = abs(P[0] * D[1] - P[1] * D[0])                       # distance centre -> line
            assert abs(abs(s) - 2 * math.sqrt(R * R - q * q)) < 1e-12


def test_support_width_is_max_projection():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a, b = rng.uniform(0.5, 3, 2)
        ang = rng.uniform(0, 2 * math.pi)
        yh = np.array([math.cos(ang), math.sin(ang), 0.0])
        W = float(ag.ellipse_support(T(a), T(b), T([1.0, 0, 0]), T([0, 1.0, 0]), T(yh)))
        ts = np.linspace(0, 2 * math.pi, 200001)
        proj = (a * np.cos(ts)) * yh[0] + (b * np.sin(ts)) * yh[1]
        assert abs(W - proj.max()) < 1e-8


def test_reciprocity_at_fixed_counts():
    """h-averaged f_ours(omega_i, omega_o) = f_ours(omega_o, omega_i) at fixed n, rho."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        ti, to = rng.uniform(-1.3, 1.3, 2)
        phi = rng.uniform(0.6 * math.pi, math.pi) * rng.choice([-1, 1])   # front: n from the chord
        nF = T([rng.uniform(1, 4)]); nB = T([rng.uniform(1, 3)]); rho = T([0.4]); nt = T([30.0])

        def avg(a, b, ph):
            tot = 0
            for hk, wk in zip(ag.GL_NODES, ag.GL_WEIGHTS):
                tot = tot + 0.5 * wk * ag.f_ours(T([0.5 * (a + b)]), T([0.5 * abs(a - b)]), T([ph]), hk.reshape(1),
                                                 SIG, MAT, nt, rho, nF, nB)[0]
            return tot
        assert torch.allclose(avg(ti, to, phi), avg(to, ti, -phi), rtol=1e-11)


def test_gauss_legendre_average_symmetric_in_h():
    """Nodes h and -h contribute equally to a_F / a_B (same attenuation, same front mass by
    F(-x) = 1 - F(x) of the periodic logistic CDF); the device sums the four h > 0 nodes with
    doubled weights."""
    import oracle.fiber as Fb
    s = Fb.logistic_scale(0.3)
    xd = torch.linspace(0.0, 1.4, 9, dtype=torch.float64)
    sig = torch.tensor([0.3, 0.6, 1.2], dtype=torch.float64)
    h = ag.GL_NODES.to(torch.float64)
    for i in range(4):
        hp, hm = h[7 - i], h[i]
        assert float(hp) == -float(hm)
        Ap, gop, gtp = Fb.attenuation(xd, hp * torch.ones_like(xd), sig, 1.55)
        Am, gom, gtm = Fb.attenuation(xd, hm * torch.ones_like(xd), sig, 1.55)
        assert torch.allclose(Ap, Am, rtol=0, atol=1e-15)
        for p in range(3):
            fp = ag.front_mass(Fb.exit_azimuth(p, gop, gtp), s)
            fm = ag.front_mass(Fb.exit_azimuth(p, gom, gtm), s)
            assert torch.allclose(fp, fm, rtol=0, atol=1e-12)
