"""Aggregated thick-hair scattering function f_ours (paper Sec. 4, eq. our_bcsdf), float64.

f_ours = S(phi, theta_d) * ( sum_{p in R^, TT^, TRT^} A_p M_p N_p  +  A_B^ M_B^ N_B^ )

The paper's own single-fibre model is R / TT / D; this implementation runs the Marschner
R / TT / TRT variant the paper says the framework generalises to, so the hatted lobes are
R^, TT^ and TRT^ (no D^).  The pieces, with the reading each one takes:

  * A_p = a_F^{n-1} a_p (Sec. 4, modified lobes), a_p the single-fibre attenuation at the
    view ray's cross-section offset h.
  * Variances add: beta_bar_p^2 = beta_p^2 + (n-1) sigma_f^2 for both the longitudinal M_p
    and the azimuthal N_p width (Sec. 4, accumulated variances; the paper mixes a
    variance and a standard deviation there, the sum is taken over variances).
  * a_F, a_B: h-averaged (8-node Gauss-Legendre) hemispherical albedos of the single fibre,
    front = |phi| > pi/2, with the longitudinal integral taken as 1 (Sec. 3.3: a_F sums
    the single-fibre lobes toward the front hemisphere).  sigma_f^2 (sigma_b^2) is the
    attenuation-weighted mean of the lobe variances beta_p^2 over the front (back)
    hemisphere, weights averaged over RGB.
  * A_1, A_3: dual-scattering local back-scattering paths (Sec. 3.2), in their closed
    geometric-series forms a_B a_F^2 / (1 - a_F^2) and a_B^3 a_F^2 / (1 - a_F^2)^3.
  * A_1+ = d_1+ a_B sum_{i=1..n} a_F^{2i-1} with d_1+ = 0.6 (Sec. 4, extra path series),
    summed in closed form for real n: a_F (1 - a_F^{2n}) / (1 - a_F^2).
  * A_B^ = A_1+ + A_1 + A_3;  M_B^ = 1/2 G(beta_bar_B, theta_h) with beta_bar_B^2 the
    attenuation-weighted mean path variance;  N_B^ = I_B(phi) / pi, I_B = [|phi| < pi/2].
  * rho = n_total r^2 / (|a||b|), n = rho l sqrt(n_total / (pi |a||b|)) (Sec. 4, hair
    number), rho clamped to [0, 1]; l is the 2-D chord through the cross-section ellipse
    from the view ray's entry point toward (n_F) or away from (n_B) the light.
  * n = 1 in the back hemisphere |phi| < pi/2 (Sec. 4), and for a single-hair cluster.
  * S = P_s a_F + P_n with P_s = (1 - rho)(1 - cos phi), P_m = c_m (1 - rho), c_m = 0.2,
    P_n = 1 - P_m - P_s clamped at 0, applied only for |phi| < pi/2 (Sec. 4,
    eq. shadowmasking).
  * A single-hair cluster (n_total = 1) has A_B^ = 0 and S = 1, so f_ours = f_single.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .fiber import (PI, attenuation, exit_azimuth, gaussian, logistic_scale, lobe_shifts_widths,
                    trimmed_logistic, trimmed_logistic_cdf, wrap_pi)

D_1PLUS = 0.6     # Sec. 4, constant of the extra path series A_1+
C_M = 0.2         # Sec. 4, multiple-hair shadowing constant c_m

_GL_X, _GL_W = np.polynomial.legendre.leggauss(8)
GL_NODES = torch.tensor(_GL_X, dtype=torch.float64)
GL_WEIGHTS = torch.tensor(_GL_W, dtype=torch.float64)


def periodic_cdf(x, s):
    """Antiderivative of the 2 pi-periodic trimmed logistic: k + C(x - 2 pi k)."""
    k = torch.floor((x + PI) / (2.0 * PI))
    return k + trimmed_logistic_cdf(x - 2.0 * PI * k, s)


def front_mass(mu, s):
    """Mass of the trimmed logistic centred at mu over the front hemisphere |phi| > pi/2."""
    back = periodic_cdf(0.5 * PI - mu, s) - periodic_cdf(-0.5 * PI - mu, s)
    return 1.0 - back


def hemisphere_stats(x_d, sigma_a, mat):
    """a_F, a_B ([..., 3]) and sigma_f^2, sigma_b^2 ([...]) for half-difference angle x_d."""
    eta, alpha, beta_m, beta_n = mat
    _, b_p = lobe_shifts_widths(alpha, beta_m)
    s = logistic_scale(beta_n)
    h = GL_NODES.to(x_d.dtype)
    w = GL_WEIGHTS.to(x_d.dtype)
    xk = x_d[..., None].expand(*x_d.shape, 8)
    hk = h.expand_as(xk)
    A, gamma_o, gamma_t = attenuation(xk, hk, sigma_a[..., None, :], eta)   # [..., 8, 3p, 3c]
    PF = torch.stack([front_mass(exit_azimuth(p, gamma_o, gamma_t), s) for p in range(3)], dim=-1)
    wk = (0.5 * w)[:, None, None]
    front = (wk * A * PF[..., None]).sum(dim=-3)          # [..., 3p, 3c]
    back = (wk * A * (1.0 - PF[..., None])).sum(dim=-3)
    a_F = front.sum(dim=-2)
    a_B = back.sum(dim=-2)
    bp2 = torch.tensor([b * b for b in b_p], dtype=x_d.dtype)
    wF = front.mean(dim=-1)
    wB = back.mean(dim=-1)
    var_f = (wF * bp2).sum(-1) / wF.sum(-1)
    var_b = (wB * bp2).sum(-1) / wB.sum(-1)
    return a_F, a_B, var_f, var_b


def back_lobe(a_F, a_B, var_f, var_b, n_B):
    """A_B^ (before the n_total = 1 switch) and beta_bar_B^2 of the B^ lobe."""
    aF2 = a_F * a_F
    A1 = a_B * aF2 / (1.0 - aF2)
    A3 = a_B ** 3 * aF2 / (1.0 - aF2) ** 3
    A1p = D_1PLUS * a_B * a_F * (1.0 - a_F ** (2.0 * n_B[..., None])) / (1.0 - aF2)
    m1, m3, m1p = A1.mean(-1), A3.mean(-1), A1p.mean(-1)
    varB = (m1 * (var_b + 2.0 * var_f) + m3 * (3.0 * var_b + 2.0 * var_f)
            + m1p * (var_b + (2.0 * n_B - 1.0) * var_f)) / (m1 + m3 + m1p)
    return A1p + A1 + A3, varB


def shadowing_masking(phi, rho, a_F, n_total):
    """S(phi, theta_d), RGB."""
    P_s = (1.0 - rho) * (1.0 - torch.cos(phi))
    P_m = C_M * (1.0 - rho)
    P_n = torch.clamp(1.0 - P_m - P_s, min=0.0)
    S = P_s[..., None] * a_F + P_n[..., None]
    active = (torch.abs(phi) < 0.5 * PI) & (n_total >= 2)
    return torch.where(active[..., None], S, torch.ones_like(S))


def f_ours(theta_h, x_d, phi, h, sigma_a, mat, n_total, rho, n_F, n_B):
    """Aggregated BCSDF (RGB [..., 3]).  n_total, rho, n_F, n_B: [...] float64."""
    eta, alpha, beta_m, beta_n = mat
    a_p, b_p = lobe_shifts_widths(alpha, beta_m)
    a_F, a_B, var_f, var_b = hemisphere_stats(x_d, sigma_a, mat)
    A, gamma_o, gamma_t = attenuation(x_d, h, sigma_a, eta)
    fwd = a_F ** (n_F - 1.0)[..., None]
    extra = (n_F - 1.0) * var_f
    s_bar = math.sqrt(3.0) * torch.sqrt(beta_n * beta_n + extra) / PI
    out = torch.zeros_like(a_F)
    for p in range(3):
        M = 0.5 * gaussian(torch.sqrt(b_p[p] * b_p[p] + extra), theta_h - a_p[p])
        N = trimmed_logistic(wrap_pi(phi - exit_azimuth(p, gamma_o, gamma_t)), s_bar)
        out = out + fwd * A[..., p, :] * (M * N)[..., None]
    AB, varB = back_lobe(a_F, a_B, var_f, var_b, n_B)
    AB = torch.where((n_total >= 2)[..., None], AB, torch.zeros_like(AB))
    MB = 0.5 * gaussian(torch.sqrt(varB), theta_h)
    NB = (torch.abs(phi) < 0.5 * PI).to(theta_h.dtype) / PI
    out = out + AB * (MB * NB)[..., None]
    return shadowing_masking(phi, rho, a_F, n_total) * out


def ellipse_support(a_len, b_len, ahat, bhat, yh):
    """Half-width W of the ellipse (semi-axes a_len along ahat, b_len along bhat) along yh."""
    pa = a_len * (ahat * yh).sum(-1)
    pb = b_len * (bhat * yh).sum(-1)
    return torch.sqrt(pa * pa + pb * pb)


def ellipse_chord(h, W, xh, yh, ahat, bhat, a_len, b_len, D):
    """Signed chord s* from the view ray's entry point along D (unit, in the cross-section).

    The view ray runs along -xh at offset h W along yh; its first hit P on the ellipse is
    the smaller root of |o' - t x'|^2 = 1 in axis-scaled coordinates.  The line P + s D meets
    the ellipse again at s* = -2 (P' . D') / (D' . D').
    """
    o_a = h * W * (yh * ahat).sum(-1) / a_len
    o_b = h * W * (yh * bhat).sum(-1) / b_len
    x_a = (xh * ahat).sum(-1) / a_len
    x_b = (xh * bhat).sum(-1) / b_len
    qa = x_a * x_a + x_b * x_b
    qb = o_a * x_a + o_b * x_b
    qc = o_a * o_a + o_b * o_b - 1.0
    disc = torch.clamp(qb * qb - qa * qc, min=0.0)
    t = (qb - torch.sqrt(disc)) / qa
    P_a = o_a - t * x_a
    P_b = o_b - t * x_b
    D_a = (D * ahat).sum(-1) / a_len
    D_b = (D * bhat).sum(-1) / b_len
    return -2.0 * (P_a * D_a + P_b * D_b) / (D_a * D_a + D_b * D_b)


def hair_counts(phi, s_star, n_total, r, a_len, b_len):
    """rho, n_F, n_B for a fragment of a thick hair (Sec. 4, hair number)."""
    rho = torch.clamp(n_total * r * r / (a_len * b_len), 0.0, 1.0)
    kappa = torch.sqrt(n_total / (PI * a_len * b_len))
    l_F = torch.clamp(s_star, min=0.0)
    l_B = torch.clamp(-s_star, min=0.0)
    one = torch.ones_like(rho)
    back = torch.abs(phi) < 0.5 * PI
    n_F = torch.where(back | (n_total < 2), one, torch.clamp(rho * kappa * l_F, min=1.0))
    n_B = torch.clamp(rho * kappa * l_B, min=1.0)
    return rho, n_F, n_B
