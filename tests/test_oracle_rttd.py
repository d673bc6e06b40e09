"""Pins for the R / TT / D single-fibre model and its aggregated form (oracle/rttd.py).

Every pin integrates or probes the scattering function numerically; none retypes a formula:
lobe normalisations over (theta_o, phi), hemisphere albedos against quadrature, the variance
reductions to a single Gaussian lobe, widened lobes that keep their mass and whose azimuthal
variance grows by (n - 1) sigma_f^2, and the single-hair reduction f_ours = f_single.
"""
import math

import numpy as np
import torch

from oracle import aggregate as ag
from oracle import rttd as rt

MAT = rt.RTTD(0.1, 0.2, 0.3, (0.1, 0.1, 0.1), (0.3, 0.2, 0.12), (0.3, 0.16, 0.09))
NARROW = rt.RTTD(0.08, 0.12, 0.3, (0.1, 0.1, 0.1), (0.3, 0.2, 0.12), (0.3, 0.16, 0.09))
PI = math.pi


def _gl(a, b, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (a + b), 0.5 * (b - a) * w


def _grid(theta_i, phi_parts, n_t=300, n_p=200, t_half=0.5 * PI):
    """Tensor-product Gauss-Legendre grid over theta_o in [-t_half, t_half] and the phi intervals."""
    to, wt = _gl(-t_half, t_half, n_t)
    ps, wp = [], []
    for a, b in phi_parts:
        x, w = _gl(a, b, n_p)
        ps.append(x)
        wp.append(w)
    ph, wph = np.concatenate(ps), np.concatenate(wp)
    TO, PH = np.meshgrid(to, ph, indexing="ij")
    W = np.outer(wt, wph)
    th = torch.tensor(0.5 * (theta_i + TO))
    return th, torch.tensor(PH), torch.tensor(W)


FULL = [(-PI, -0.5 * PI), (-0.5 * PI, 0.0), (0.0, 0.5 * PI), (0.5 * PI, PI)]
FRONT = [(-PI, -0.5 * PI), (0.5 * PI, PI)]
BACK = [(-0.5 * PI, 0.0), (0.0, 0.5 * PI)]


def _integrate(f, W):
    return (f * W[..., None]).sum(dim=(0, 1)).numpy()


def test_single_fibre_lobes_are_normalised():
    """Integral of f over theta_o and phi is A_R + A_TT + A_D (each lobe has unit mass; the
    narrow widths keep the longitudinal Gaussians' tails beyond theta_o = +-pi/2 below 1e-9)."""
    tot = np.array(NARROW.a_r) + np.array(NARROW.a_tt) + np.array(NARROW.a_d)
    for theta_i in (0.0, 0.1, -0.1):
        th, ph, W = _grid(theta_i, FULL)
        got = _integrate(rt.f_single(th, ph, NARROW), W)
        assert np.allclose(got, tot, rtol=1e-9, atol=0), (theta_i, got, tot)


def test_each_lobe_alone_has_its_attenuation_as_mass():
    th, ph, W = _grid(0.1, FULL)
    zero = (0.0, 0.0, 0.0)
    for name in ("a_r", "a_tt", "a_d"):
        m = NARROW._replace(**{k: (getattr(NARROW, k) if k == name else zero) for k in ("a_r", "a_tt", "a_d")})
        got = _integrate(rt.f_single(th, ph, m), W)
        assert np.allclose(got, getattr(NARROW, name), rtol=1e-9, atol=0), name


def test_hemisphere_albedos_match_quadrature():
    for m in (NARROW, NARROW._replace(gamma_tt=1.2)):
        a_F, a_B, _, _ = rt.hemisphere_stats(m)
        th, ph, W = _grid(0.0, FRONT)
        assert np.allclose(_integrate(rt.f_single(th, ph, m), W), a_F.numpy(), rtol=1e-9, atol=0)
        th, ph, W = _grid(0.0, BACK)
        assert np.allclose(_integrate(rt.f_single(th, ph, m), W), a_B.numpy(), rtol=1e-9, atol=0)
    # TT is a forward lobe: its front share dominates
    assert float(a_F[0]) > float(a_B[0])


def test_hemisphere_variances_reduce_to_single_lobes():
    zero = (0.0, 0.0, 0.0)
    _, _, vf, vb = rt.hemisphere_stats(MAT._replace(a_tt=zero))
    assert math.isclose(vf, MAT.beta_r ** 2, rel_tol=1e-14) and math.isclose(vb, MAT.beta_r ** 2, rel_tol=1e-14)
    _, _, vf, vb = rt.hemisphere_stats(MAT._replace(a_r=zero))
    assert math.isclose(vf, MAT.beta_tt ** 2, rel_tol=1e-14) and math.isclose(vb, MAT.beta_tt ** 2, rel_tol=1e-14)
    # D carries no variance weight; TT's mass sits in front, so the back mean leans to R
    _, _, vf0, vb0 = rt.hemisphere_stats(MAT._replace(a_d=zero))
    _, _, vf1, vb1 = rt.hemisphere_stats(MAT)
    assert vf0 == vf1 and vb0 == vb1
    assert MAT.beta_r ** 2 < vb1 < vf1 < MAT.beta_tt ** 2


def test_lobe_shapes():
    th = torch.zeros(721, dtype=torch.float64)
    ph = torch.linspace(-PI, PI, 721, dtype=torch.float64)
    zero = (0.0, 0.0, 0.0)
    flat = rt.f_single(th, ph, MAT._replace(a_tt=zero))
    assert torch.allclose(flat, flat[0].expand_as(flat), rtol=1e-15, atol=0)
    tt = rt.f_single(th, ph, MAT._replace(a_r=zero, a_d=zero))[:, 0]
    assert abs(float(ph[int(torch.argmax(tt))])) == PI                       # TT peaks at phi = pi
    assert torch.allclose(tt, tt.flip(0), rtol=1e-12, atol=0)                # symmetric in phi
    lon = rt.f_single(torch.linspace(-0.7, 0.7, 141, dtype=torch.float64), torch.zeros(141, dtype=torch.float64),
                      MAT._replace(a_tt=zero, a_d=zero))[:, 0]
    assert int(torch.argmax(lon)) == 70                                      # R: no longitudinal shift


def test_reciprocity():
    g = torch.Generator().manual_seed(5)
    ti = (torch.rand(200, generator=g, dtype=torch.float64) - 0.5) * 2.0
    to = (torch.rand(200, generator=g, dtype=torch.float64) - 0.5) * 2.0
    ph = (torch.rand(200, generator=g, dtype=torch.float64) - 0.5) * 2 * PI
    a = rt.f_single(0.5 * (ti + to), ph, MAT)
    b = rt.f_single(0.5 * (to + ti), -ph, MAT)
    assert torch.allclose(a, b, rtol=1e-14, atol=0)


def test_single_hair_cluster_is_the_single_fibre():
    g = torch.Generator().manual_seed(6)
    th = (torch.rand(300, generator=g, dtype=torch.float64) - 0.5) * 1.5
    ph = (torch.rand(300, generator=g, dtype=torch.float64) - 0.5) * 2 * PI
    one = torch.ones_like(th)
    for rho in (0.0, 0.3, 1.0):
        got = rt.f_ours(th, ph, MAT, one, rho * one, one, 3.0 * one)
        assert torch.allclose(got, rt.f_single(th, ph, MAT), rtol=1e-14, atol=0)


def test_widened_forward_lobes_keep_mass_and_add_variance():
    """With n_F hairs crossed (single-hair cluster: no B^, S = 1) the R^, TT^, D^ lobes hold
    a_F^{n_F - 1} of the single-fibre mass, and the TT^ azimuthal variance about pi grows by
    (n_F - 1) sigma_f^2."""
    a_F, _, var_f, _ = rt.hemisphere_stats(NARROW)
    tot = np.array(NARROW.a_r) + np.array(NARROW.a_tt) + np.array(NARROW.a_d)
    for nF in (1.5, 2.0):
        th, ph, W = _grid(0.0, FULL)
        one = torch.ones_like(th)
        got = _integrate(rt.f_ours(th, ph, NARROW, one, one, nF * one, one), W)
        want = a_F.numpy() ** (nF - 1.0) * tot
        assert np.allclose(got, want, rtol=2e-5, atol=0), (nF, got, want)
    zero = (0.0, 0.0, 0.0)
    tt_only = NARROW._replace(a_r=zero, a_d=zero)
    _, _, var_tt, _ = rt.hemisphere_stats(tt_only)
    th, ph, W = _grid(0.0, [(0.0, PI), (PI, 2 * PI)], n_p=400)
    one = torch.ones_like(th)
    for nF in (1.0, 3.0):
        f = rt.f_ours(th, ph, tt_only, one, one, nF * one, one)[..., 0]
        mass = float((f * W).sum())
        m2 = float((f * W * (ph - PI) ** 2).sum()) / mass
        assert math.isclose(m2, tt_only.gamma_tt ** 2 + (nF - 1.0) * var_tt, rel_tol=1e-6), (nF, m2)


def test_back_lobe_mass_and_hemisphere():
    """Dense cluster (rho = 1: S = 1), n_F = 1: in the back hemisphere f_ours - f_single is
    the B^ lobe, whose integral over that hemisphere and over theta_o (taken over the whole
    line, |theta_o| < 4 pi, so the Gaussian's full mass counts) is A_B^ = A_1 + A_3 + A_1+;
    in the front hemisphere the B^ lobe is absent."""
    a_F, a_B, vf, vb = rt.hemisphere_stats(MAT)
    nB = 4.0
    th, ph, W = _grid(0.0, BACK, n_t=600, t_half=4.0 * PI)
    one = torch.ones_like(th)
    diff = rt.f_ours(th, ph, MAT, 5.0 * one, one, one, nB * one) - rt.f_single(th, ph, MAT)
    AB, _ = ag.back_lobe(a_F, a_B, torch.tensor(vf), torch.tensor(vb), torch.tensor(nB))
    assert np.allclose(_integrate(diff, W), AB.numpy(), rtol=1e-8, atol=0)
    th, ph, W = _grid(0.0, FRONT)
    one = torch.ones_like(th)
    diff = rt.f_ours(th, ph, MAT, 5.0 * one, one, one, nB * one) - rt.f_single(th, ph, MAT)
    assert float(diff.abs().max()) == 0.0


def test_widened_reflection_lobe_longitudinal_variance():
    """At phi = 0 the TT^ lobe is negligible (its Gaussian sits at phi = pi) and D^ is constant
    in theta, so f - f(theta_h = 3) is the R^ lobe alone; over the theta_h line its variance
    is beta_R^2 + (n_F - 1) sigma_f^2 with sigma_f^2 of the whole material."""
    _, _, var_f, var_b = rt.hemisphere_stats(NARROW)
    assert var_f != var_b
    x, w = _gl(-3.0, 3.0, 800)
    th = torch.tensor(np.append(x, 3.0))
    w = torch.tensor(w)
    ph = torch.zeros_like(th)
    one = torch.ones_like(th)
    for nF in (1.0, 2.5, 4.0):
        f = rt.f_ours(th, ph, NARROW, one, one, nF * one, one)[:, 1]
        g = f[:-1] - f[-1]
        m0 = float((g * w).sum())
        m2 = float((g * w * th[:-1] ** 2).sum()) / m0
        assert math.isclose(m2, NARROW.beta_r ** 2 + (nF - 1.0) * var_f, rel_tol=1e-9), (nF, m2)
