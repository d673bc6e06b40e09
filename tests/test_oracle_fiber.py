"""Pins for the single-fibre scattering function (oracle/fiber.py).

Each test checks the oracle against something other than its own formula: textbook closed
forms written differently, brute-force geometry, quadrature, or invariants.
"""
import math

import numpy as np
import pytest
import torch
from scipy import integrate, stats

from oracle import fiber as fb

T = lambda x: torch.as_tensor(x, dtype=torch.float64)
MAT = (1.55, math.radians(-3.0), 0.3, 0.3)


# ---- P1: Gaussian, Fresnel, Bravais index -------------------------------------------------

def test_gaussian_matches_normal_pdf():
    x = np.linspace(-2, 2, 41)
    for beta in (0.05, 0.3, 1.1):
        assert np.allclose(fb.gaussian(beta, T(x)).numpy(), stats.norm.pdf(x, scale=beta), rtol=1e-12)


def _fresnel_angles(theta_i, eta):
    """Textbook Fresnel in terms of the incidence and refraction angles."""
    theta_t = math.asin(math.sin(theta_i) / eta)
    if theta_i == 0.0:
        return ((eta - 1) / (eta + 1)) ** 2
    rs = -math.sin(theta_i - theta_t) / math.sin(theta_i + theta_t)
    rp = math.tan(theta_i - theta_t) / math.tan(theta_i + theta_t)
    return 0.5 * (rs * rs + rp * rp)


@pytest.mark.parametrize("eta", [1.33, 1.55, 2.0])
def test_fresnel_textbook(eta):
    for th in np.linspace(0.0, 1.5, 16):
        ours = float(fb.fresnel_dielectric(T(math.cos(th)), eta))
        assert abs(ours - _fresnel_angles(th, eta)) < 1e-12
    assert abs(float(fb.fresnel_dielectric(T(0.0), eta)) - 1.0) < 1e-12          # grazing
    brewster = math.atan(eta)                                                  # rp = 0 there
    th_t = math.asin(math.sin(brewster) / eta)
    rs = math.sin(brewster - th_t) / math.sin(brewster + th_t)
    assert abs(float(fb.fresnel_dielectric(T(math.cos(brewster)), eta)) - 0.5 * rs * rs) < 1e-12


def _refract3(d, n, eta):
    """Vector Snell refraction of unit direction d (travelling) at unit normal n (facing d)."""
    c = -np.dot(d, n)
    k = 1.0 - (1.0 - c * c) / (eta * eta)
    return d / eta + (c / eta - math.sqrt(k)) * n


@pytest.mark.parametrize("x_long", [0.0, 0.3, 0.8, 1.2])
def test_bravais_index_from_3d_snell(x_long):
    """A ray at longitudinal angle x hitting a cylinder refracts, in projection onto the
    normal plane, as a 2-D Snell law with index eta' = sqrt(eta^2 - sin^2 x) / cos x."""
    eta = 1.55
    eta_p = math.sqrt(eta * eta - math.sin(x_long) ** 2) / math.cos(x_long)
    for gam in np.linspace(-1.4, 1.4, 9):
        # cylinder axis = z; surface normal in the x-y plane at angle gam from the ray's azimuth
        d = np.array([-math.cos(x_long), 0.0, math.sin(x_long)])     # azimuth along -x
        n = np.array([math.cos(gam), math.sin(gam), 0.0])
        t = _refract3(d, n, eta)
        tp = t[:2] / np.linalg.norm(t[:2])
        g_t = math.asin(abs(tp[0] * n[1] - tp[1] * n[0]))          # angle to the inward normal
        assert abs(math.sin(abs(gam)) - eta_p * math.sin(g_t)) < 1e-12
        # the longitudinal angle inside follows sin(theta_t) = sin(x) / eta
        assert abs(t[2] - math.sin(x_long) / eta) < 1e-12


# ---- P2: exit azimuth by brute-force 2-D ray tracing through a disc ------------------------

def _trace_disc(h, eta_p, p):
    """Camera ray travelling along -x at offset y = h hits the unit disc; follow p internal
    segments (R: p=0).  Returns the exit direction (the direction toward the light)."""
    pos = np.array([math.sqrt(1 - h * h), h])
    d = np.array([-1.0, 0.0])
    n = pos.copy()
    if p == 0:
        return d - 2 * np.dot(d, n) * n

    def refract2(d, n, eta):
        c = -np.dot(d, n)
        k = 1.0 - (1.0 - c * c) / (eta * eta)
        return d / eta + (c / eta - math.sqrt(k)) * n

    d = refract2(d, n, eta_p)
    for seg in range(p):
        # next intersection with the unit circle from inside
        b = np.dot(pos, d)
        s = -2.0 * b
        pos = pos + s * d
        n = pos / np.linalg.norm(pos)
        if seg < p - 1:
            d = d - 2 * np.dot(d, n) * n                          # internal reflection
    # exit: refract from inside (index eta_p -> 1)
    c = np.dot(d, n)
    k = 1.0 - eta_p * eta_p * (1.0 - c * c)
    return eta_p * d + (math.sqrt(k) - eta_p * c) * n


@pytest.mark.parametrize("p", [0, 1, 2])
def test_exit_azimuth_matches_ray_trace(p):
    eta_p = 1.7
    for h in np.linspace(-0.95, 0.95, 39):
        out = _trace_disc(h, eta_p, p)
        # omega_o is +x (toward the camera); the exit direction is omega_i.  phi = -azimuth(omega_i)
        phi_traced = -math.atan2(out[1], out[0])
        g_o = math.asin(h)
        g_t = math.asin(h / eta_p)
        phi_model = float(fb.exit_azimuth(p, T(g_o), T(g_t)))
        diff = (phi_traced - phi_model + math.pi) % (2 * math.pi) - math.pi
        assert abs(diff) < 1e-9, (p, h, phi_traced, phi_model)


# ---- P3/P4: normalisation -----------------------------------------------------------------

@pytest.mark.parametrize("beta_n", [0.1, 0.3, 0.9])
def test_azimuthal_lobe_normalised(beta_n):
    s = fb.logistic_scale(beta_n)
    for mu in (0.0, 1.0, 3.0, -2.5):
        val, _ = integrate.quad(lambda x: float(fb.trimmed_logistic(fb.wrap_pi(T(x - mu)), s)),
                                -math.pi, math.pi, limit=200, points=[mu if abs(mu) < math.pi else 0.0])
        assert abs(val - 1.0) < 1e-8


def test_logistic_std_dev_is_beta_n():
    beta = 0.05                       # narrow so the trimming is negligible
    s = fb.logistic_scale(beta)
    var, _ = integrate.quad(lambda x: x * x * float(fb.trimmed_logistic(T(x), s)), -math.pi, math.pi,
                            points=[0.0], limit=200)
    assert abs(math.sqrt(var) - beta) < 1e-6


def test_trimmed_cdf_is_integral_of_density():
    s = fb.logistic_scale(0.4)
    for x in (-2.0, -0.3, 0.0, 1.1, 3.0):
        val, _ = integrate.quad(lambda y: float(fb.trimmed_logistic(T(y), s)), -math.pi, x, limit=200)
        assert abs(val - float(fb.trimmed_logistic_cdf(T(x), s))) < 1e-10


@pytest.mark.parametrize("beta", [0.15, 0.3, 0.6])
def test_longitudinal_lobe_is_density_in_theta_o(beta):
    theta_i = 0.4
    val, _ = integrate.quad(lambda to: 0.5 * float(fb.gaussian(beta, T(0.5 * (theta_i + to) - 0.1))),
                            -np.inf, np.inf)
    assert abs(val - 1.0) < 1e-9
    val2, _ = integrate.quad(lambda to: 0.5 * float(fb.gaussian(beta, T(0.5 * (theta_i + to))))
                             * math.cos(to) ** 2, -math.pi / 2, math.pi / 2)
    assert val2 <= 1.0


# ---- P5: white furnace -------------------------------------------------------------------

def test_attenuation_white_furnace_closed_form():
    x = T(np.linspace(0.0, 1.4, 8))[:, None].expand(8, 9)
    h = T(np.linspace(-0.99, 0.99, 9))[None, :].expand(8, 9)
    A, _, _ = fb.attenuation(x, h, torch.zeros(8, 9, 3, dtype=torch.float64), 1.55)
    cos_xd, _, cos_go, _, _, _ = fb.fiber_geometry(x, h, 1.55)
    F = fb.fresnel_dielectric(cos_xd * cos_go, 1.55)
    total = A.sum(dim=-2)[..., 0]
    assert torch.allclose(total, 1.0 - F * F + F ** 3, atol=1e-14)
    assert float(total.max()) <= 1.0


@pytest.mark.parametrize("theta_i,h", [(0.0, 0.0), (0.5, 0.6), (-0.9, -0.3), (1.2, 0.95)])
def test_directional_albedo_at_most_one(theta_i, h):
    """Integral of f cos^2(theta_o) over the sphere of outgoing directions, sigma_a = 0."""
    to = np.linspace(-math.pi / 2, math.pi / 2, 721)
    ph = np.linspace(-math.pi, math.pi, 721)
    TO, PH = np.meshgrid(to, ph, indexing="ij")
    ti = np.full_like(TO, theta_i)
    f = fb.f_single(T(0.5 * (ti + TO)), T(0.5 * np.abs(ti - TO)), T(PH), T(np.full_like(TO, h)),
                    torch.zeros(*TO.shape, 3, dtype=torch.float64), MAT)[..., 0].numpy()
    alb = np.trapezoid(np.trapezoid(f * np.cos(TO) ** 2, ph, axis=1), to)
    assert 0.0 < alb <= 1.0


# ---- P6: reciprocity ---------------------------------------------------------------------

def test_h_averaged_reciprocity():
    from oracle.aggregate import GL_NODES, GL_WEIGHTS
    rng = np.random.default_rng(3)
    sig = torch.tensor([[0.3, 0.6, 1.2]], dtype=torch.float64)
    for _ in range(20):
        ti, to = rng.uniform(-1.4, 1.4, 2)
        phi = rng.uniform(-math.pi, math.pi)

        def avg(a, b, ph):
            tot = torch.zeros(3, dtype=torch.float64)
            for hk, wk in zip(GL_NODES, GL_WEIGHTS):
                tot = tot + 0.5 * wk * fb.f_single(T([0.5 * (a + b)]), T([0.5 * abs(a - b)]), T([ph]),
                                                   hk.reshape(1), sig, MAT)[0]
            return tot
        # swapping omega_i and omega_o negates the relative azimuth phi_o - phi_i
        assert torch.allclose(avg(ti, to, phi), avg(to, ti, -phi), rtol=1e-12, atol=1e-15)
