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
#pragma once

#include "hair_internal.h"

namespace hair {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvSqrt2Pi = 0.39894228040143267794f;
constexpr float kSqrt3 = 1.73205080756887729353f;
constexpr float kD1Plus = 0.6f;     // Sec. 4, A_1+ path-series constant
constexpr float kCm = 0.2f;         // Sec. 4, multiple-hair shadowing constant

// 8-point Gauss-Legendre rule on [-1, 1] (standard published nodes and weights).
__constant__ static const float kGLx[8] = {-0.9602898564975363f, -0.7966664774136267f, -0.5255324099163290f,
                                           -0.1834346424956498f, 0.1834346424956498f,  0.5255324099163290f,
                                           0.7966664774136267f,  0.9602898564975363f};
__constant__ static const float kGLw[8] = {0.1012285362903763f, 0.2223810344533745f, 0.3137066458778873f,
                                           0.3626837833783620f, 0.3626837833783620f, 0.3137066458778873f,
                                           0.2223810344533745f, 0.1012285362903763f};

// ---- scalar function set; the dual-number type provides the same names ----
__device__ inline float m_exp(float x) { return expf(x); }
__device__ inline float m_sqrt(float x) { return sqrtf(x); }
__device__ inline float m_asin(float x) { return asinf(x); }
__device__ inline float m_atan2(float y, float x) { return atan2f(y, x); }
__device__ inline float m_sin(float x) { return sinf(x); }
__device__ inline float m_cos(float x) { return cosf(x); }
__device__ inline float m_tanh(float x) { return tanhf(x); }
__device__ inline float m_abs(float x) { return fabsf(x); }
__device__ inline float m_pow(float x, float y) { return powf(x, y); }
__device__ inline float m_min(float a, float b) { return fminf(a, b); }
__device__ inline float m_max(float a, float b) { return fmaxf(a, b); }
__device__ inline float m_val(float x) { return x; }
__device__ inline float m_const(float x, float) { return x; }

template <class T> struct V3 { T x, y, z; };
template <class T> __device__ inline V3<T> v3(T x, T y, T z) { return {x, y, z}; }
template <class T> __device__ inline T dot(const V3<T>& a, const V3<T>& b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
template <class T> __device__ inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> __device__ inline V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S> __device__ inline V3<T> scale(const V3<T>& a, S s) { return {a.x * s, a.y * s, a.z * s}; }

template <class T> __device__ inline T clampv(T x, float lo, float hi) { return m_min(m_max(x, T(lo)), T(hi)); }

template <class T> __device__ inline T gaussian(T beta, T x) {
    return m_exp(-(x * x) / (2.0f * beta * beta)) * kInvSqrt2Pi / beta;
}

__device__ inline float wrap_pi(float x) { return x - kTwoPi * floorf((x + kPi) / kTwoPi); }

template <class T> __device__ inline T wrap_pi(T x) {
    float k = floorf((m_val(x) + kPi) / kTwoPi);
    return x - kTwoPi * k;
}

template <class T> __device__ inline T trimmed_logistic(T x, T s, T inv_tanh) {
    T e = m_exp(-m_abs(x) / s);
    T one_e = 1.0f + e;
    return e / (s * one_e * one_e) * inv_tanh;
}

template <class T> __device__ inline T logistic_cdf_trimmed(T x, T s) {
    T lo = 1.0f / (1.0f + m_exp(kPi / s));
    T hi = 1.0f / (1.0f + m_exp(-kPi / s));
    return (1.0f / (1.0f + m_exp(-x / s)) - lo) / (hi - lo);
}

// Antiderivative of the 2 pi-periodic trimmed logistic.
template <class T> __device__ inline T periodic_cdf(T x, T s) {
    float k = floorf((m_val(x) + kPi) / kTwoPi);
    return T(k) + logistic_cdf_trimmed(x - kTwoPi * k, s);
}

template <class T> __device__ inline T fresnel(T cos_i, float eta) {
    T sin2_t = (1.0f - cos_i * cos_i) / (eta * eta);
    T cos_t = m_sqrt(1.0f - sin2_t);
    T rs = (cos_i - eta * cos_t) / (cos_i + eta * cos_t);
    T rp = (eta * cos_i - cos_t) / (eta * cos_i + cos_t);
    return 0.5f * (rs * rs + rp * rp);
}

// Attenuations of R, TT, TRT (RGB) and the refraction angles at offset h.
template <class T> struct Atten {
    T A[3][3];      // [lobe][channel]
    T gamma_o, gamma_t;
};

template <class T>
__device__ inline Atten<T> attenuation(T x_d, T h, const T sig[3], float eta) {
    Atten<T> o;
    T sxd = m_sin(x_d);
    T cxd = m_max(m_cos(x_d), T(0.0f));
    T eta_p = m_sqrt(eta * eta - sxd * sxd) / cxd;
    o.gamma_o = m_asin(h);
    T cgo = m_sqrt((1.0f - h) * (1.0f + h));
    T sgt = h / eta_p;
    o.gamma_t = m_asin(sgt);
    T cgt = m_sqrt(1.0f - sgt * sgt);
    T stt = sxd / eta;
    T ctt = m_sqrt(1.0f - stt * stt);
    T F = fresnel(cxd * cgo, eta);
    T path = 2.0f * cgt / ctt;
    T one_f = 1.0f - F;
    T one_f2 = one_f * one_f;
    for (int c = 0; c < 3; ++c) {
        T Tc = m_exp(-sig[c] * path);
        o.A[0][c] = F;
        o.A[1][c] = one_f2 * Tc;
        o.A[2][c] = one_f2 * F * Tc * Tc;
    }
    return o;
}

template <class T> __device__ inline T exit_azimuth(int p, T gamma_o, T gamma_t) {
    return (2.0f * p) * gamma_t - 2.0f * gamma_o + p * kPi;
}

// Single-fibre BCSDF, RGB.
template <class T>
__device__ inline void f_single(T theta_h, T x_d, T phi, T h, const T sig[3], const MatConst& m, T out[3]) {
    Atten<T> at = attenuation(x_d, h, sig, m.eta);
    T s = T(m.s), inv_tanh = T(m.inv_tanh);
    out[0] = out[1] = out[2] = T(0.0f);
    for (int p = 0; p < 3; ++p) {
        T M = 0.5f * gaussian(T(m.beta_p[p]), theta_h - m.alpha_p[p]);
        T N = trimmed_logistic(wrap_pi(phi - exit_azimuth(p, at.gamma_o, at.gamma_t)), s, inv_tanh);
        T MN = M * N;
        for (int c = 0; c < 3; ++c) out[c] = out[c] + at.A[p][c] * MN;
    }
}

// Hemisphere albedos a_F, a_B (RGB) and variances sigma_f^2, sigma_b^2 at x_d.
template <class T>
__device__ inline void hemisphere_stats(T x_d, const T sig[3], const MatConst& m, T aF[3], T aB[3], T& var_f,
                                        T& var_b) {
    T s = T(m.s);
    T wF[3], wB[3];
    for (int c = 0; c < 3; ++c) aF[c] = aB[c] = T(0.0f);
    for (int p = 0; p < 3; ++p) wF[p] = wB[p] = T(0.0f);
    for (int k = 0; k < 8; ++k) {
        T hk = T(kGLx[k]);
        Atten<T> at = attenuation(x_d, hk, sig, m.eta);
        float wk = 0.5f * kGLw[k];
        for (int p = 0; p < 3; ++p) {
            T mu = exit_azimuth(p, at.gamma_o, at.gamma_t);
            T back = periodic_cdf(T(0.5f * kPi) - mu, s) - periodic_cdf(T(-0.5f * kPi) - mu, s);
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

// Aggregated BCSDF, RGB.
template <class T>
__device__ inline void f_ours(T theta_h, T x_d, T phi, T h, const T sig[3], const MatConst& m,
                              const ClusterFrag<T>& cf, T out[3]) {
    const bool back_hemi = m_abs(m_val(phi)) < 0.5f * kPi;
    const bool multi = m_val(cf.n_total) >= 2.0f;
    T aF[3], aB[3], var_f, var_b;
    hemisphere_stats(x_d, sig, m, aF, aB, var_f, var_b);
    Atten<T> at = attenuation(x_d, h, sig, m.eta);
    T nm1 = cf.n_F - 1.0f;
    T extra = nm1 * var_f;
    T s_bar = kSqrt3 * m_sqrt(T(m.beta_n * m.beta_n) + extra) / kPi;
    T inv_tanh = 1.0f / m_tanh(kPi / (2.0f * s_bar));
    T fwd[3];
    for (int c = 0; c < 3; ++c) fwd[c] = m_pow(aF[c], nm1);
    for (int c = 0; c < 3; ++c) out[c] = T(0.0f);
    for (int p = 0; p < 3; ++p) {
        T M = 0.5f * gaussian(m_sqrt(T(m.beta_p[p] * m.beta_p[p]) + extra), theta_h - m.alpha_p[p]);
        T N = trimmed_logistic(wrap_pi(phi - exit_azimuth(p, at.gamma_o, at.gamma_t)), s_bar, inv_tanh);
        T MN = M * N;
        for (int c = 0; c < 3; ++c) out[c] = out[c] + fwd[c] * at.A[p][c] * MN;
    }
    if (multi) {
        T A1[3], A3[3], A1p[3];
        T m1 = T(0.0f), m3 = T(0.0f), m1p = T(0.0f);
        for (int c = 0; c < 3; ++c) {
            T aF2 = aF[c] * aF[c];
            T om = 1.0f - aF2;
            A1[c] = aB[c] * aF2 / om;
            A3[c] = aB[c] * aB[c] * aB[c] * aF2 / (om * om * om);
            A1p[c] = kD1Plus * aB[c] * aF[c] * (1.0f - m_pow(aF[c], 2.0f * cf.n_B)) / om;
            m1 = m1 + A1[c] * (1.0f / 3.0f);
            m3 = m3 + A3[c] * (1.0f / 3.0f);
            m1p = m1p + A1p[c] * (1.0f / 3.0f);
        }
        T varB = (m1 * (var_b + 2.0f * var_f) + m3 * (3.0f * var_b + 2.0f * var_f) +
                  m1p * (var_b + (2.0f * cf.n_B - 1.0f) * var_f)) / (m1 + m3 + m1p);
        if (back_hemi) {
            T MB = 0.5f * gaussian(m_sqrt(varB), theta_h) * (1.0f / kPi);
            for (int c = 0; c < 3; ++c) out[c] = out[c] + (A1p[c] + A1[c] + A3[c]) * MB;
        }
    }
    if (back_hemi && multi) {
        T one_rho = 1.0f - cf.rho;
        T Ps = one_rho * (1.0f - m_cos(phi));
        T Pn = m_max(1.0f - kCm * one_rho - Ps, T(0.0f));
        for (int c = 0; c < 3; ++c) out[c] = (Ps * aF[c] + Pn) * out[c];
    }
}

}  // namespace hair
