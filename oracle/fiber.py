"""Single-fibre scattering function: near-field Marschner-style R / TT / TRT lobes (float64).

The paper states its single-hair BCSDF as a sum over lobes p of A_p M_p(theta_h) N_p(phi)
with theta_h = (theta_i + theta_o) / 2 and phi = phi_o - phi_i (Sec. 3.1, eq. bcsdf), and
says the framework carries over to Marschner's R / TT / TRT lobes (Sec. 2 and Sec. 6,
"Extending to Marschner model with TRT term") without printing their formulas.  The lobe
definitions below are the reading this implementation fixes:

  * Gaussian G(beta, x) with beta a standard deviation (Sec. 3.2, definition of G).
  * M_p = 1/2 G(beta_p, theta_h - alpha_p): a density over theta_o (the 1/2 is the
    Jacobian of theta_h), alpha_p = (a, -a/2, -3a/2), beta_p = (bm, bm/2, 2 bm).
  * N_p = trimmed logistic about the exit azimuth Phi(p, h) = 2 p gamma_t - 2 gamma_o + p pi,
    standard deviation beta_n, normalised on (-pi, pi].
  * A_0 = F, A_1 = (1-F)^2 T, A_2 = (1-F)^2 F T^2 with unpolarised dielectric Fresnel F at
    cos(x_d) cos(gamma_o), modified index eta' = sqrt(eta^2 - sin^2 x_d) / cos x_d
    (Bravais), T = exp(-sigma_a 2 cos(gamma_t) / cos(theta_t)), sin(theta_t) = sin(x_d)/eta.
  * x_d = |theta_i - theta_o| / 2 in every attenuation term, so f is reciprocal.

All functions take torch float64 tensors and broadcast.
"""
from __future__ import annotations

import math

import torch

PI = math.pi
SQRT_2PI = math.sqrt(2.0 * PI)


def gaussian(beta, x):
    """G(beta, x) = exp(-x^2 / 2 beta^2) / (sqrt(2 pi) beta)  (Sec. 3.2)."""
    return torch.exp(-(x * x) / (2.0 * beta * beta)) / (SQRT_2PI * beta)


def fresnel_dielectric(cos_i, eta):
    """Unpolarised Fresnel reflectance entering a dielectric of relative index eta > 1."""
    sin2_t = (1.0 - cos_i * cos_i) / (eta * eta)
    cos_t = torch.sqrt(1.0 - sin2_t)
    rs = (cos_i - eta * cos_t) / (cos_i + eta * cos_t)
    rp = (eta * cos_i - cos_t) / (eta * cos_i + cos_t)
    return 0.5 * (rs * rs + rp * rp)


def lobe_shifts_widths(alpha: float, beta_m: float):
    """(alpha_p, beta_p) for p = R, TT, TRT."""
    return (alpha, -0.5 * alpha, -1.5 * alpha), (beta_m, 0.5 * beta_m, 2.0 * beta_m)


def logistic_scale(beta):
    """Scale s of a logistic whose standard deviation is beta: s = sqrt(3) beta / pi."""
    return math.sqrt(3.0) * beta / PI


def trimmed_logistic(x, s):
    """Logistic density of scale s restricted to [-pi, pi] and renormalised there.

    Untrimmed density: e^{-|x|/s} / (s (1 + e^{-|x|/s})^2); its mass on [-pi, pi] is
    tanh(pi / 2s).
    """
    s = torch.as_tensor(s, dtype=x.dtype)
    e = torch.exp(-torch.abs(x) / s)
    return e / (s * (1.0 + e) ** 2) / torch.tanh(PI / (2.0 * s))


def trimmed_logistic_cdf(x, s):
    """Cumulative of trimmed_logistic on [-pi, pi] (0 at -pi, 1 at pi)."""
    s = torch.as_tensor(s, dtype=x.dtype)
    lo = 1.0 / (1.0 + torch.exp(PI / s))
    hi = 1.0 / (1.0 + torch.exp(-PI / s))
    return (1.0 / (1.0 + torch.exp(-x / s)) - lo) / (hi - lo)


def wrap_pi(x):
    """Map an angle to [-pi, pi)."""
    return x - 2.0 * PI * torch.floor((x + PI) / (2.0 * PI))


def fiber_geometry(x_d, h, eta):
    """Refraction geometry for half-difference angle x_d and cross-section offset h.

    Returns (cos_xd, gamma_o, cos_gamma_o, gamma_t, cos_gamma_t, cos_theta_t).
    """
    sin_xd = torch.sin(x_d)
    cos_xd = torch.cos(x_d)
    eta_p = torch.sqrt(eta * eta - sin_xd * sin_xd) / cos_xd
    gamma_o = torch.asin(h)
    cos_go = torch.sqrt((1.0 - h) * (1.0 + h))
    sin_gt = h / eta_p
    gamma_t = torch.asin(sin_gt)
    cos_gt = torch.sqrt(1.0 - sin_gt * sin_gt)
    sin_tt = sin_xd / eta
    cos_tt = torch.sqrt(1.0 - sin_tt * sin_tt)
    return cos_xd, gamma_o, cos_go, gamma_t, cos_gt, cos_tt


def attenuation(x_d, h, sigma_a, eta):
    """A_p for p = R, TT, TRT.

    x_d, h: [...];  sigma_a: [..., 3].  Returns (A [..., 3 lobes, 3 rgb], gamma_o, gamma_t).
    """
    cos_xd, gamma_o, cos_go, gamma_t, cos_gt, cos_tt = fiber_geometry(x_d, h, eta)
    F = fresnel_dielectric(cos_xd * cos_go, eta)[..., None]
    T = torch.exp(-sigma_a * (2.0 * cos_gt / cos_tt)[..., None])
    one_f2 = (1.0 - F) ** 2
    A0 = F.expand_as(T)
    A1 = one_f2 * T
    A2 = one_f2 * F * T * T
    return torch.stack([A0, A1, A2], dim=-2), gamma_o, gamma_t


def exit_azimuth(p: int, gamma_o, gamma_t):
    """Phi(p, h) = 2 p gamma_t - 2 gamma_o + p pi (relative azimuth phi_o - phi_i)."""
    return 2.0 * p * gamma_t - 2.0 * gamma_o + p * PI


def angles(sin_ti, sin_to):
    """theta_i, theta_o, theta_h, x_d from the sines (clamped to [-1, 1])."""
    ti = torch.asin(torch.clamp(sin_ti, -1.0, 1.0))
    to = torch.asin(torch.clamp(sin_to, -1.0, 1.0))
    return ti, to, 0.5 * (ti + to), 0.5 * torch.abs(ti - to)


def f_single(theta_h, x_d, phi, h, sigma_a, mat):
    """Single-fibre BCSDF sum_p A_p M_p N_p (RGB, [..., 3]).

    mat = (eta, alpha, beta_m, beta_n) as floats.
    """
    eta, alpha, beta_m, beta_n = mat
    A, gamma_o, gamma_t = attenuation(x_d, h, sigma_a, eta)
    a_p, b_p = lobe_shifts_widths(alpha, beta_m)
    s = logistic_scale(beta_n)
    out = torch.zeros_like(A[..., 0, :])
    for p in range(3):
        M = 0.5 * gaussian(b_p[p], theta_h - a_p[p])
        N = trimmed_logistic(wrap_pi(phi - exit_azimuth(p, gamma_o, gamma_t)), s)
        out = out + A[..., p, :] * (M * N)[..., None]
    return out
