"""R / TT / D single-fibre model and its aggregated thick-hair form (float64, oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper's own single-fibre model (Sec. 3.1, eq. bcsdf) has three lobes with constant RGB
attenuations: reflection R, transmission TT and a diffuse lobe D standing in for multiple
scattering inside the fibre.  Its aggregated counterparts R^, TT^, D^ (Sec. 4, modified
lobes) are the same lobes after n - 1 forward passes.  Readings taken here:

  * M_R = 1/2 G(beta_R, theta_h) and M_TT = 1/2 G(beta_TT, theta_h): the paper prints the
    lobes with no longitudinal shift; the factor 1/2 normalises them over theta_o (theta_h
    moves at half the rate of theta_o), the same convention as M_D = 1/pi, which the paper
    prints and which integrates to 1 over theta_o in [-pi/2, pi/2].
  * N_R = N_D = 1 / (2 pi) (uniform); N_TT = G(gamma_TT, phi - pi) with phi - pi wrapped
    to [-pi, pi) (not renormalised: for the paper's widths 0.2-0.4 the wrapped Gaussian's
    mass differs from 1 by less than 1e-14).
  * a_F, a_B (Sec. 3.3: the single-fibre lobes summed toward the front / back hemisphere,
    front = |phi| > pi/2), longitudinal integral taken as 1: R and D split evenly, TT puts
    erf(pi / (2 sqrt2 gamma_TT)) of its mass in the front hemisphere.  No h-average is
    needed: none of the lobes depends on the cross-section offset.
  * sigma_f^2 (sigma_b^2): the attenuation-weighted mean (RGB-mean weights) of the
    longitudinal variances beta_R^2, beta_TT^2 of the lobes' front (back) mass.  The D lobe
    is uniform in both angles and has no spread to accumulate, so it carries no weight.
  * Variances add: beta_bar^2 = beta^2 + (n_F - 1) sigma_f^2 in M_R^, M_TT^ and N_TT^; the
    D^ lobe keeps M = 1/pi, N = 1/(2 pi).  A_p = a_F^{n_F - 1} A_p.
  * The B^ lobe (A_1 + A_3 + A_1+, its path variance) and the shadowing-masking term S are the
    same as for the Marschner variant (oracle.aggregate.back_lobe, shadowing_masking).
"""
from __future__ import annotations

import math
from typing import NamedTuple

import torch

from .aggregate import back_lobe, shadowing_masking
from .fiber import PI, gaussian, wrap_pi


class RTTD(NamedTuple):
    """Material of the R / TT / D model: widths in radians, attenuations RGB."""
    beta_r: float
    beta_tt: float
    gamma_tt: float
    a_r: tuple
    a_tt: tuple
    a_d: tuple


def _rgb(v, like):
    return torch.as_tensor(v, dtype=like.dtype)


def lobes(theta_h, phi, m: RTTD, extra=None):
    """Per-lobe (M N) of R, TT, D ([..., 3] over lobes) with variances widened by `extra`."""
    if extra is None:
        extra = torch.zeros_like(theta_h)
    bR = torch.sqrt(m.beta_r * m.beta_r + extra)
    bT = torch.sqrt(m.beta_tt * m.beta_tt + extra)
    gT = torch.sqrt(m.gamma_tt * m.gamma_tt + extra)
    mnR = 0.5 * gaussian(bR, theta_h) / (2.0 * PI)
    mnT = 0.5 * gaussian(bT, theta_h) * gaussian(gT, wrap_pi(phi - PI))
    mnD = torch.full_like(theta_h, 1.0 / (PI * 2.0 * PI))
    return torch.stack([mnR, mnT, mnD], dim=-1)


def f_single(theta_h, phi, m: RTTD):
    """Single-fibre f = A_R M_R N_R + A_TT M_TT N_TT + A_D M_D N_D, RGB [..., 3]."""
    A = torch.stack([_rgb(m.a_r, theta_h), _rgb(m.a_tt, theta_h), _rgb(m.a_d, theta_h)])  # [lobe, rgb]
    return lobes(theta_h, phi, m) @ A


def hemisphere_stats(m: RTTD):
    """a_F, a_B (RGB, float64 tensors [3]) and sigma_f^2, sigma_b^2 (floats)."""
    fT = math.erf(0.5 * PI / (math.sqrt(2.0) * m.gamma_tt))      # TT mass with |phi - pi| < pi/2
    bT = math.erf(PI / (math.sqrt(2.0) * m.gamma_tt)) - fT       # the rest of the wrapped Gaussian
    aR = torch.tensor(m.a_r, dtype=torch.float64)
    aT = torch.tensor(m.a_tt, dtype=torch.float64)
    aD = torch.tensor(m.a_d, dtype=torch.float64)
    a_F = 0.5 * aR + fT * aT + 0.5 * aD
    a_B = 0.5 * aR + bT * aT + 0.5 * aD
    wR_F, wT_F = 0.5 * float(aR.mean()), fT * float(aT.mean())
    wR_B, wT_B = 0.5 * float(aR.mean()), bT * float(aT.mean())
    b2R, b2T = m.beta_r * m.beta_r, m.beta_tt * m.beta_tt

    def mean_var(wR, wT):
        return (wR * b2R + wT * b2T) / (wR + wT) if wR + wT > 0.0 else 0.0

    return a_F, a_B, mean_var(wR_F, wT_F), mean_var(wR_B, wT_B)


def f_ours(theta_h, phi, m: RTTD, n_total, rho, n_F, n_B):
    """Aggregated f (Sec. 4, eq. our_bcsdf) with R^, TT^, D^ and B^ lobes, RGB [..., 3]."""
    a_F, a_B, var_f, var_b = hemisphere_stats(m)
    shape = theta_h.shape
    aF = a_F.expand(*shape, 3)
    aB = a_B.expand(*shape, 3)
    vf = torch.full(shape, var_f, dtype=theta_h.dtype)
    vb = torch.full(shape, var_b, dtype=theta_h.dtype)
    A = torch.stack([_rgb(m.a_r, theta_h), _rgb(m.a_tt, theta_h), _rgb(m.a_d, theta_h)])
    out = (aF ** (n_F - 1.0)[..., None]) * (lobes(theta_h, phi, m, (n_F - 1.0) * vf) @ A)
    AB, varB = back_lobe(aF, aB, vf, vb, n_B)
    AB = torch.where((n_total >= 2)[..., None], AB, torch.zeros_like(AB))
    MB = 0.5 * gaussian(torch.sqrt(varB), theta_h)
    NB = (torch.abs(phi) < 0.5 * PI).to(theta_h.dtype) / PI
    out = out + AB * (MB * NB)[..., None]
    return shadowing_masking(phi, rho, aF, n_total) * out
