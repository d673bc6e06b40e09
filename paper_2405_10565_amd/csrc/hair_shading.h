// Per-fragment scattering on the device: single fibre (R / TT / TRT) and the aggregated
// thick-hair model.  Written once as templates over the scalar type so the forward pass
// (float) and the backward pass (forward-mode dual numbers) share the definition.
//
//   f_single = sum_p A_p M_p N_p                      (Sec. 3.1, eq. bcsdf; Marschner lobes)
//   f_ours   = S (sum_p A_p M_p N_p + A_B M_B N_B)     (Sec. 4, eq. our_bcsdf)
//
// Lobe definitions (the readings the library fixes where the paper prints none):
//   M_p = 1/2 G(beta_p, theta_h - alpha_p), G a Gaussian with standard deviation beta;
//   N_p = logistic of standard deviation beta_n about Phi(p, h) = 2 p gamma_t - 2 gamma_o + p pi,
//         trimmed to [-pi, pi] and renormalised;
//   A_R = F, A_TT = (1 - F)^2 T, A_TRT = (1 - F)^2 F T^2 with Fresnel F at cos(x_d) cos(gamma_o),
//         Bravais index eta' = sqrt(eta^2 - sin^2 x_d) / cos x_d, T = exp(-sigma_a 2 cos gamma_t / cos theta_t),
//         x_d = |theta_i - theta_o| / 2.
// Thick hairs (Sec. 4): A_p = a_F^{n-1} a_p, variances add (beta^2 + (n-1) sigma_f^2), a_F / a_B
// are 8-node Gauss-Legendre h-averages of the single-fibre albedos toward |phi| > pi/2 /
// |phi| < pi/2, A_B = A_1+ + A_1 + A_3 with d_1+ = 0.6, N_B = [|phi| < pi/2] / pi,
// S = P_s a_F + max(0, 1 - P_m - P_s) for |phi| < pi/2 with c_m = 0.2, and n = 1 for
// |phi| < pi/2 or a single-hair cluster.
//
// R / TT / D model (Sec. 3.1 eq. bcsdf with constant RGB attenuations A_R, A_TT, A_D; Sec. 4
// modified lobes): M_R = 1/2 G(beta_R, theta_h), N_R = 1 / (2 pi); M_TT = 1/2 G(beta_TT,
// theta_h), N_TT = G(gamma_TT, phi - pi); M_D = 1 / pi, N_D = 1 / (2 pi).  For thick hairs the
// three lobes take a_F^{n-1} and variances widened by (n-1) sigma_f^2; a_F, a_B, sigma_f^2 and
// sigma_b^2 do not depend on the view and are folded on the host.  The B lobe and S are shared
// with the Marschner variant.
//
// Float arithmetic: the scattering terms use the hardware exp2 / reciprocal / square-root
// instructions and fitted polynomials for arcsine and arctangent (coefficients and error
// bounds in hair_fastmath_coef.h); every such step is within a few float32 ulps, far inside the
// renderer's radiance tolerance.  The view angles enter through sin / cos products (x_d from
// cos(theta_i - theta_o) by the half-angle identities), so no trigonometric call remains.
#pragma once

#include "hair_internal.h"
#include "hair_fastmath_coef.h"

// Multiply-adds in the scattering terms may fuse (one rounding instead of two); nothing here
// decides an integer.  The library's other code is compiled without contraction.
#pragma clang fp contract(fast)

namespace hair {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kHalfPi = 1.57079632679489661923f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.15915494309189533577f;
constexpr float kInvTwoPi2 = 0.05066059182116888572f;   // 1 / (2 pi^2) = M_D N_D
constexpr float kInvSqrt2Pi = 0.39894228040143267794f;
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kSqrt3 = 1.73205080756887729353f;
constexpr float kD1Plus = 0.6f;     // Sec. 4, A_1+ path-series constant
constexpr float kCm = 0.2f;         // Sec. 4, multiple-hair shadowing constant

// ---- float function set; the dual-number type provides the same names ----
__device__ inline float m_exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ inline float m_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float m_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float m_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float m_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// arcsine on [-1, 1]: polynomial on [0, 1/2], asin(x) = pi/2 - 2 asin(sqrt((1 - x) / 2)) above
__device__ inline float m_asin(float x) {
    const float ax = fabsf(x);
    const bool big = ax > 0.5f;
    const float t = big ? 0.5f * (1.0f - ax) : ax * ax;
    const float z = big ? __builtin_amdgcn_sqrtf(t) : ax;
    float p = kAsinP[4];
    p = p * t + kAsinP[3];
    p = p * t + kAsinP[2];
    p = p * t + kAsinP[1];
    p = p * t + kAsinP[0];
    float r = z + (z * t) * p;
    r = big ? kHalfPi - 2.0f * r : r;
    return copysignf(r, x);
}

// atan2 by octant reduction to atan(a), a in [0, 1]
__device__ inline float m_atan2(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float t = a * a;
    float q = kAtanQ[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) q = q * t + kAtanQ[i];
    float r = a * q;
    r = ay > ax ? kHalfPi - r : r;
    r = x < 0.0f ? kPi - r : r;
    return copysignf(r, y);
}

__device__ inline float m_tanh(float x) { return tanhf(x); }
__device__ inline float m_abs(float x) { return fabsf(x); }
// x^y for x >= 0 (0^0 = 1)
__device__ inline float m_pow(float x, float y) {
    if (y == 0.0f) return 1.0f;
    if (x == 0.0f) return 0.0f;
    return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
}
__device__ inline float m_min(float a, float b) { return fminf(a, b); }
__device__ inline float m_max(float a, float b) { return fmaxf(a, b); }
__device__ inline float m_val(float x) { return x; }

template <class T> struct V3 { T x, y, z; };
template <class T> __device__ inline V3<T> v3(T x, T y, T z) { return {x, y, z}; }
template <class T> __device__ inline T dot(const V3<T>& a, const V3<T>& b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
template <class T> __device__ inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> __device__ inline V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S> __device__ inline V3<T> scale(const V3<T>& a, S s) { return {a.x * s, a.y * s, a.z * s}; }

template <class T> __device__ inline T clampv(T x, float lo, float hi) { return m_min(m_max(x, T(lo)), T(hi)); }

// Gaussian of standard deviation beta at x
template <class T> __device__ inline T gaussian(T beta, T x) {
    const T ib = m_rcp(beta);
    return m_exp(-0.5f * (x * x) * (ib * ib)) * kInvSqrt2Pi * ib;
}

__device__ inline float wrap_pi(float x) { return x - kTwoPi * floorf((x + kPi) * kInvTwoPi); }

template <class T> __device__ inline T wrap_pi(T x) {
    float k = floorf((m_val(x) + kPi) * kInvTwoPi);
    return x - kTwoPi * k;
}

// logistic density of scale s trimmed to [-pi, pi]; k = log2(e) / s, norm = 1 / (s tanh(pi / 2s))
template <class T> __device__ inline T trimmed_logistic(T x, T k, T norm) {
    T e = m_exp2(-m_abs(x) * k);
    T one_e = 1.0f + e;
    return e * norm * m_rcp(one_e * one_e);
}

// Antiderivative of the 2 pi-periodic trimmed logistic of the material's scale s:
// k + (sigmoid(y / s) - lo) / (hi - lo), y = x - 2 pi k in [-pi, pi).
template <class T> __device__ inline T periodic_cdf(T x, const MatConst& m) {
    float k = floorf((m_val(x) + kPi) * kInvTwoPi);
    T y = x - kTwoPi * k;
    return T(k) + (m_rcp(1.0f + m_exp2(-y * m.inv_s_l2)) - m.cdf_lo) * m.cdf_scale;
}

// (one reciprocal of the product of the two denominators, both at least cos theta_t > 0)
template <class T> __device__ inline T fresnel(T cos_i, const MatConst& m) {
    T sin2_t = (1.0f - cos_i * cos_i) * m.inv_eta2;
    T cos_t = m_sqrt(1.0f - sin2_t);
    T ec = m.eta * cos_t, ei = m.eta * cos_i;
    T ds = cos_i + ec, dp = ei + cos_t;
    T inv = m_rcp(ds * dp);
    T rs = (cos_i - ec) * dp * inv;
    T rp = (ei - cos_t) * ds * inv;
    return 0.5f * (rs * rs + rp * rp);
}

// View/light geometry of one fragment and light (independent of the fitted parameters).
struct LightView {
    float theta_h;     // (theta_i + theta_o) / 2
    float cos_ti;      // cos theta_i (irradiance foreshortening)
    float phi;         // relative azimuth
    float cos_phi;
    float sxd2, cxd;   // sin^2 x_d, cos x_d
    float inv_eta_p;   // 1 / eta' (Bravais index at x_d)
    float inv_ctt;     // 1 / cos theta_t, sin theta_t = sin x_d / eta
};

// sin_ti / sin_to: sines of the longitudinal angles (cos_to = cos theta_o >= 0); wx, wy: light
// direction in the normal plane, so that cos theta_i = |(wx, wy)| (taken from the components,
// not from 1 - sin^2).  theta_h = (theta_i + theta_o) / 2 is half the angle whose sine and
// cosine the sum formulas give (one arctangent per light; theta_o itself is not needed).
// 1 / eta' = cos x_d / sqrt(eta^2 - sin^2 x_d) and 1 / cos theta_t = eta / sqrt(eta^2 - sin^2 x_d)
// share their square root.
__device__ inline LightView light_view(float sin_ti, float sin_to, float cos_to, float wx, float wy, bool degen,
                                       const MatConst& m) {
    LightView v;
    const float si = fminf(fmaxf(sin_ti, -1.0f), 1.0f);
    const float r2 = wx * wx + wy * wy;
    const float r_w = m_rsqrt(r2);
    const float ci = r2 > 0.0f ? r2 * r_w : 0.0f;
    v.cos_ti = ci;
    v.theta_h = 0.5f * m_atan2(si * cos_to + ci * sin_to, ci * cos_to - si * sin_to);
    const float c = fminf(fmaxf(ci * cos_to + si * sin_to, -1.0f), 1.0f);   // cos(theta_i - theta_o)
    v.sxd2 = 0.5f * (1.0f - c);
    v.cxd = m_sqrt(0.5f * (1.0f + c));
    const float r_e = m_rsqrt(m.eta * m.eta - v.sxd2);
    v.inv_eta_p = v.cxd * r_e;
    v.inv_ctt = m.eta * r_e;
    if (degen || !(r2 > 0.0f)) {
        v.phi = 0.0f;
        v.cos_phi = 1.0f;
    } else {
        v.phi = -m_atan2(wy, wx);
        v.cos_phi = wx * r_w;
    }
    return v;
}

// Attenuations of R, TT, TRT (RGB) and the refraction angle at offset h (incidence angle
// gamma_o = asin h, cos gamma_o given).
template <class T> struct Atten {
    T A[3][3];      // [lobe][channel]
    T gamma_t;
};

// sigl: absorption times log2(e)
template <class T>
__device__ inline Atten<T> attenuation(const LightView& v, T h, T cgo, const T sigl[3], const MatConst& m) {
    Atten<T> o;
    T sgt = h * v.inv_eta_p;
    o.gamma_t = m_asin(sgt);
    T cgt = m_sqrt(1.0f - sgt * sgt);
    T F = fresnel(v.cxd * cgo, m);
    T path = 2.0f * cgt * v.inv_ctt;
    T one_f = 1.0f - F;
    T one_f2 = one_f * one_f;
    for (int c = 0; c < 3; ++c) {
        T Tc = m_exp2(-sigl[c] * path);
        o.A[0][c] = F;
        o.A[1][c] = one_f2 * Tc;
        o.A[2][c] = one_f2 * F * Tc * Tc;
    }
    return o;
}

template <class T> __device__ inline T exit_azimuth(int p, T gamma_o, T gamma_t) {
    const T g2 = -2.0f * gamma_o;
    return p == 0 ? g2 : (p == 1 ? (g2 + 2.0f * gamma_t) + kPi : (g2 + 4.0f * gamma_t) + kTwoPi);
}

// Single-fibre BCSDF, RGB (gamma_o = asin h, cgo = cos gamma_o).  With the absorption
// transmittance T_c of channel c, A_R = F, A_TT = (1 - F)^2 T_c and A_TRT = (1 - F)^2 F T_c^2,
// so the three lobes sum per channel as q_R + T_c (q_TT + T_c q_TRT) with q_p the lobe's M_p N_p
// times its channel-independent factor; M_p N_p's two amplitudes are one host constant.
template <class T>
__device__ inline void f_single(const LightView& v, T h, T gamma_o, T cgo, const T sigl[3], const MatConst& m,
                                T out[3]) {
    const T sgt = h * v.inv_eta_p;
    const T gamma_t = m_asin(sgt);
    const T cgt = m_sqrt(1.0f - sgt * sgt);
    const T F = fresnel(v.cxd * cgo, m);
    const T path = 2.0f * cgt * v.inv_ctt;
    const T one_f = 1.0f - F;
    const T one_f2 = one_f * one_f;
    const T ks = T(m.inv_s_l2);
    T mn[3];
    for (int p = 0; p < 3; ++p) {
        const float x = v.theta_h - m.alpha_p[p];
        const float M = m_exp2(-m.g_k2[p] * (x * x));
        const T e = m_exp2(-m_abs(wrap_pi(v.phi - exit_azimuth(p, gamma_o, gamma_t))) * ks);
        const T one_e = 1.0f + e;
        mn[p] = (m.mn_amp[p] * M) * (e * m_rcp(one_e * one_e));
    }
    const T q0 = F * mn[0], q1 = one_f2 * mn[1], q2 = (one_f2 * F) * mn[2];
    for (int c = 0; c < 3; ++c) {
        const T Tc = m_exp2(-sigl[c] * path);
        out[c] = q0 + Tc * (q1 + Tc * q2);
    }
}

// Hemisphere albedos a_F, a_B (RGB) and variances sigma_f^2, sigma_b^2 at the light's x_d.
// The 8-node rule is symmetric in h and so is each node's contribution (h -> -h flips the
// sign of gamma_o, gamma_t and of every exit azimuth, which leaves the attenuations and, by
// F(-x) = 1 - F(x) of the periodic CDF, the back-hemisphere mass unchanged): the four nodes
// h > 0 are evaluated with doubled weights.
template <class T>
__device__ inline void hemisphere_stats(const LightView& v, const T sigl[3], const MatConst& m, T aF[3], T aB[3],
                                        T& var_f, T& var_b) {
    T wF[3], wB[3];
    for (int c = 0; c < 3; ++c) aF[c] = aB[c] = T(0.0f);
    for (int p = 0; p < 3; ++p) wF[p] = wB[p] = T(0.0f);
    for (int k = 4; k < 8; ++k) {
        const T go = T(kGLgo[k]);
        Atten<T> at = attenuation(v, T(kGLx[k]), T(kGLcgo[k]), sigl, m);
        float wk = kGLw[k];   // 2 x (1/2 of the node weight on [-1, 1])
        for (int p = 0; p < 3; ++p) {
            T mu = exit_azimuth(p, go, at.gamma_t);
            T back = periodic_cdf(T(kHalfPi) - mu, m) - periodic_cdf(T(-kHalfPi) - mu, m);
            T PF = 1.0f - back;
            T sumF = T(0.0f), sumB = T(0.0f);
            for (int c = 0; c < 3; ++c) {
                T f = wk * at.A[p][c] * PF;
                T b = wk * at.A[p][c] * back;
                aF[c] = aF[c] + f;
                aB[c] = aB[c] + b;
                sumF = sumF + f;
                sumB = sumB + b;
            }
            wF[p] = wF[p] + sumF * (1.0f / 3.0f);
            wB[p] = wB[p] + sumB * (1.0f / 3.0f);
        }
    }
    T nf = T(0.0f), df = T(0.0f), nb = T(0.0f), db = T(0.0f);
    for (int p = 0; p < 3; ++p) {
        float b2 = m.beta_p[p] * m.beta_p[p];
        nf = nf + wF[p] * b2;
        df = df + wF[p];
        nb = nb + wB[p] * b2;
        db = db + wB[p];
    }
    var_f = nf / df;
    var_b = nb / db;
}

// Thick-hair inputs of one fragment and light.
template <class T> struct ClusterFrag {
    T n_total;     // members
    T rho;         // hair density
    T n_F, n_B;    // hair counts toward / away from the light
};

// B lobe (A_1+ + A_1 + A_3 toward the back hemisphere) added to out, then the
// shadowing-masking factor S applied (Sec. 4; both only for clusters of two or more hairs).
template <class T>
__device__ inline void back_lobe_shadow(const LightView& v, const T aF[3], const T aB[3], const T& var_f,
                                        const T& var_b, const ClusterFrag<T>& cf, bool back_hemi, bool multi,
                                        T out[3]) {
    if (multi) {
        T A1[3], A3[3], A1p[3];
        T m1 = T(0.0f), m3 = T(0.0f), m1p = T(0.0f);
        for (int c = 0; c < 3; ++c) {
            T aF2 = aF[c] * aF[c];
            T iom = m_rcp(1.0f - aF2);
            A1[c] = aB[c] * aF2 * iom;
            A3[c] = aB[c] * aB[c] * aB[c] * aF2 * (iom * iom * iom);
            A1p[c] = kD1Plus * aB[c] * aF[c] * (1.0f - m_pow(aF[c], 2.0f * cf.n_B)) * iom;
            m1 = m1 + A1[c] * (1.0f / 3.0f);
            m3 = m3 + A3[c] * (1.0f / 3.0f);
            m1p = m1p + A1p[c] * (1.0f / 3.0f);
        }
        T varB = (m1 * (var_b + 2.0f * var_f) + m3 * (3.0f * var_b + 2.0f * var_f) +
                  m1p * (var_b + (2.0f * cf.n_B - 1.0f) * var_f)) / (m1 + m3 + m1p);
        if (back_hemi) {
            T MB = 0.5f * gaussian(m_sqrt(varB), T(v.theta_h)) * (1.0f / kPi);
            for (int c = 0; c < 3; ++c) out[c] = out[c] + (A1p[c] + A1[c] + A3[c]) * MB;
        }
    }
    if (back_hemi && multi) {
        T one_rho = 1.0f - cf.rho;
        T Ps = one_rho * (1.0f - v.cos_phi);
        T Pn = m_max(1.0f - kCm * one_rho - Ps, T(0.0f));
        for (int c = 0; c < 3; ++c) out[c] = (Ps * aF[c] + Pn) * out[c];
    }
}

// Aggregated BCSDF, RGB.
template <class T>
__device__ inline void f_ours(const LightView& v, T h, T gamma_o, T cgo, const T sigl[3], const MatConst& m,
                              const ClusterFrag<T>& cf, T out[3]) {
    const bool back_hemi = fabsf(v.phi) < 0.5f * kPi;
    const bool multi = m_val(cf.n_total) >= 2.0f;
    T aF[3], aB[3], var_f, var_b;
    hemisphere_stats(v, sigl, m, aF, aB, var_f, var_b);
    Atten<T> at = attenuation(v, h, cgo, sigl, m);
    T nm1 = cf.n_F - 1.0f;
    T extra = nm1 * var_f;
    T s_bar = kSqrt3 * m_sqrt(T(m.beta_n * m.beta_n) + extra) / kPi;
    T inv_sb = m_rcp(s_bar);
    T norm = m_rcp(s_bar * m_tanh(kPi * 0.5f * inv_sb));
    T fwd[3];
    for (int c = 0; c < 3; ++c) fwd[c] = m_pow(aF[c], nm1);
    for (int c = 0; c < 3; ++c) out[c] = T(0.0f);
    for (int p = 0; p < 3; ++p) {
        T M = 0.5f * gaussian(m_sqrt(T(m.beta_p[p] * m.beta_p[p]) + extra), T(v.theta_h - m.alpha_p[p]));
        T N = trimmed_logistic(wrap_pi(v.phi - exit_azimuth(p, gamma_o, at.gamma_t)), inv_sb * kLog2e, norm);
        T MN = M * N;
        for (int c = 0; c < 3; ++c) out[c] = out[c] + fwd[c] * at.A[p][c] * MN;
    }
    back_lobe_shadow(v, aF, aB, var_f, var_b, cf, back_hemi, multi, out);
}

// R / TT / D single fibre, RGB.  |phi - pi| wrapped into [0, pi] is pi - |phi|.
template <class T>
__device__ inline void f_single_rttd(const LightView& v, const MatConst& m, T out[3]) {
    const float th2 = v.theta_h * v.theta_h;
    const float psi = kPi - fabsf(v.phi);
    const float MNR = m.d_amp[0] * m_exp2(-m.d_k2[0] * th2) * kInvTwoPi;
    const float MNT = m.d_amp[1] * m_exp2(-(m.d_k2[1] * th2 + m.n_k2 * (psi * psi))) * m.n_amp;
    for (int c = 0; c < 3; ++c) out[c] = T(m.A[0][c] * MNR + m.A[1][c] * MNT + m.A[2][c] * kInvTwoPi2);
}

// Aggregated R^ / TT^ / D^ / B^ model, RGB.
template <class T>
__device__ inline void f_ours_rttd(const LightView& v, const MatConst& m, const ClusterFrag<T>& cf, T out[3]) {
    const bool back_hemi = fabsf(v.phi) < 0.5f * kPi;
    const bool multi = m_val(cf.n_total) >= 2.0f;
    const float psi = kPi - fabsf(v.phi);
    T nm1 = cf.n_F - 1.0f;
    T extra = nm1 * m.var_f;
    T MNR = 0.5f * gaussian(m_sqrt(T(m.d_beta2[0]) + extra), T(v.theta_h)) * kInvTwoPi;
    T MNT = 0.5f * gaussian(m_sqrt(T(m.d_beta2[1]) + extra), T(v.theta_h)) *
            gaussian(m_sqrt(T(m.gamma2) + extra), T(psi));
    T aF[3], aB[3];
    for (int c = 0; c < 3; ++c) {
        aF[c] = T(m.aF[c]);
        aB[c] = T(m.aB[c]);
        out[c] = m_pow(aF[c], nm1) * (m.A[0][c] * MNR + m.A[1][c] * MNT + m.A[2][c] * kInvTwoPi2);
    }
    back_lobe_shadow(v, aF, aB, T(m.var_f), T(m.var_b), cf, back_hemi, multi, out);
}

}  // namespace hair

#pragma clang fp contract(off)
