// Forward-mode dual numbers for the backward pass: a value and N partial derivatives.
// Provides the same scalar function set as the float path in hair_shading.h (m_exp, m_sqrt,
// ...), so the scattering functions, written once as templates, differentiate themselves.
#pragma once

#include <hip/hip_runtime.h>

namespace hair {

template <int N>
struct Dual {
    float v;
    float d[N];
    __device__ Dual() : v(0.0f) {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0f;
    }
    __device__ Dual(float x) : v(x) {  // NOLINT: implicit from constants
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0f;
    }
    __device__ static Dual seed(float x, int k) {
        Dual r(x);
        r.d[k] = 1.0f;
        return r;
    }
};

// chain rule helper: f(x) with f'(x) = g
template <int N> __device__ inline Dual<N> chain(const Dual<N>& x, float fx, float g) {
    Dual<N> r;
    r.v = fx;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = g * x.d[i];
    return r;
}

template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N> __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    const float inv = 1.0f / b.v;
    r.v = a.v * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
    return r;
}
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, float b) { return a + Dual<N>(b); }
template <int N> __device__ inline Dual<N> operator+(float a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, float b) { return a - Dual<N>(b); }
template <int N> __device__ inline Dual<N> operator-(float a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> __device__ inline Dual<N> operator*(const Dual<N>& a, float b) {
    Dual<N> r;
    r.v = a.v * b;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N> __device__ inline Dual<N> operator*(float a, const Dual<N>& b) { return b * a; }
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, float b) { return a * (1.0f / b); }
template <int N> __device__ inline Dual<N> operator/(float a, const Dual<N>& b) { return Dual<N>(a) / b; }

template <int N> __device__ inline Dual<N> m_exp(const Dual<N>& x) {
    const float e = expf(x.v);
    return chain(x, e, e);
}
template <int N> __device__ inline Dual<N> m_exp2(const Dual<N>& x) {
    const float e = exp2f(x.v);
    return chain(x, e, e * 0.69314718055994530942f);
}
template <int N> __device__ inline Dual<N> m_sqrt(const Dual<N>& x) {
    const float s = sqrtf(x.v);
    return chain(x, s, s > 0.0f ? 0.5f / s : 0.0f);
}
template <int N> __device__ inline Dual<N> m_asin(const Dual<N>& x) {
    const float c = sqrtf(fmaxf((1.0f - x.v) * (1.0f + x.v), 0.0f));
    return chain(x, asinf(x.v), c > 0.0f ? 1.0f / c : 0.0f);
}
template <int N> __device__ inline Dual<N> m_rcp(const Dual<N>& x) {
    const float r = 1.0f / x.v;
    return chain(x, r, -r * r);
}
template <int N> __device__ inline Dual<N> m_sin(const Dual<N>& x) { return chain(x, sinf(x.v), cosf(x.v)); }
template <int N> __device__ inline Dual<N> m_cos(const Dual<N>& x) { return chain(x, cosf(x.v), -sinf(x.v)); }
template <int N> __device__ inline Dual<N> m_tanh(const Dual<N>& x) {
    const float t = tanhf(x.v);
    return chain(x, t, 1.0f - t * t);
}
template <int N> __device__ inline Dual<N> m_abs(const Dual<N>& x) { return x.v < 0.0f ? -x : x; }
template <int N> __device__ inline Dual<N> m_min(const Dual<N>& a, const Dual<N>& b) { return b.v < a.v ? b : a; }
template <int N> __device__ inline Dual<N> m_max(const Dual<N>& a, const Dual<N>& b) { return b.v > a.v ? b : a; }
template <int N> __device__ inline Dual<N> m_pow(const Dual<N>& x, const Dual<N>& y) {
    // x^y = exp(y ln x) for x > 0
    const float lx = logf(x.v);
    const float p = expf(y.v * lx);
    Dual<N> r;
    r.v = p;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = p * (y.d[i] * lx + y.v * x.d[i] / x.v);
    return r;
}
template <int N> __device__ inline Dual<N> m_atan2(const Dual<N>& y, const Dual<N>& x) {
    const float r2 = x.v * x.v + y.v * y.v;
    Dual<N> r;
    r.v = atan2f(y.v, x.v);
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = r2 > 0.0f ? (x.v * y.d[i] - y.v * x.d[i]) / r2 : 0.0f;
    return r;
}
template <int N> __device__ inline float m_val(const Dual<N>& x) { return x.v; }

}  // namespace hair
