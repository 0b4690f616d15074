// rt_dual.h -- forward-mode dual numbers for the per-ray adjoint's small
// pieces (emission, observer setup): a value and N directional derivatives,
// with the elementary functions the spacetime and emission formulas use.
// Host and device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "rt_math.h"

namespace rt {

// The double overloads stay visible beside the dual ones inside rt.
using ::pow;
using ::sqrt;
using ::tanh;

template <int N>
struct Dual {
    double v;
    double d[N];
    __host__ __device__ Dual() : v(0.0) {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __host__ __device__ Dual(double x) : v(x) {  // NOLINT: constants promote
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    // Variable number `dir` (derivative 1 along it).
    __host__ __device__ static Dual var(double x, int dir) {
        Dual r(x);
        r.d[dir] = 1.0;
        return r;
    }
};

template <int N>
__host__ __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v + b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v - b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r(-a.v);
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v * b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    const double inv = 1.0 / b.v;
    Dual<N> r(a.v * inv);
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N>
__host__ __device__ inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N>
__host__ __device__ inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N>
__host__ __device__ inline Dual<N> operator*(const Dual<N>& a, double b) {
    Dual<N> r(a.v * b);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N>
__host__ __device__ inline Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N>
__host__ __device__ inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

template <int N>
__host__ __device__ inline Dual<N> chain(const Dual<N>& a, double value, double deriv) {
    Dual<N> r(value);
    for (int i = 0; i < N; ++i) r.d[i] = deriv * a.d[i];
    return r;
}

template <int N>
__host__ __device__ inline Dual<N> sqrt(const Dual<N>& a) {
    const double s = ::sqrt(a.v);
    return chain(a, s, 0.5 / s);
}
template <int N>
__host__ __device__ inline Dual<N> tanh(const Dual<N>& a) {
    const double t = ::tanh(a.v);
    return chain(a, t, 1.0 - t * t);
}
template <int N>
__host__ __device__ inline Dual<N> pow(const Dual<N>& a, double b) {
    const double p = ::pow(a.v, b);
    return chain(a, p, b * p / a.v);
}

__host__ __device__ inline double value_of(double x) { return x; }
template <int N>
__host__ __device__ inline double value_of(const Dual<N>& x) { return x.v; }

namespace dm {
template <int N>
__host__ __device__ inline Dual<N> recip(const Dual<N>& a) {
    return 1.0 / a;
}
template <int N>
__host__ __device__ inline Dual<N> recip1(const Dual<N>& a) {
    return 1.0 / a;
}
template <int N>
__host__ __device__ inline Dual<N> exp(const Dual<N>& a) {
    const double e = dm::exp(a.v);
    return chain(a, e, e);
}
template <int N>
__host__ __device__ inline Dual<N> expm1(const Dual<N>& a) {
    return chain(a, dm::expm1(a.v), dm::exp(a.v));
}
template <int N>
__host__ __device__ inline Dual<N> log1p(const Dual<N>& a) {
    return chain(a, dm::log1p(a.v), 1.0 / (1.0 + a.v));
}
template <int N>
__host__ __device__ inline Dual<N> log1p_fast(const Dual<N>& a) {
    return chain(a, dm::log1p_fast(a.v), 1.0 / (1.0 + a.v));
}
template <int N>
__host__ __device__ inline void sincos(const Dual<N>& a, Dual<N>* s, Dual<N>* c) {
    double sv, cv;
    dm::sincos(a.v, &sv, &cv);
    *s = chain(a, sv, cv);
    *c = chain(a, cv, -sv);
}
}  // namespace dm

}  // namespace rt
