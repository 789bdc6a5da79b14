// fv_physics.h -- device-side Euler user terms and the Rusanov face flux,
// shared by the patch-update kernels (library-private).
//
//   p      = (gamma - 1) (E - |m|^2 / (2 rho)),   c = sqrt(gamma p / rho)
//   F_n(Q) = (m_n, m_a u_n + p delta_an (each stored momentum a), (E + p) u_n)
//   l_n(Q) = |u_n| + c                                  (Sec. 2.2, Sec. 5)
//   Fhat   = 1/2 (F_n(Q_L) + F_n(Q_R)) - 1/2 max(l_n(Q_L), l_n(Q_R)) (Q_R - Q_L)   (Eq. 2)
//
// Every expression is written with explicit fused multiply-adds and
// contraction is disabled, so all kernels and code paths round identically.
// 1/rho and sqrt use the hardware approximations refined by Newton steps
// (deterministic, within about one ulp of the correctly rounded values).
#pragma once

#include <hip/hip_runtime.h>

namespace fv {

#pragma clang fp contract(off)

// NaN-propagating maximum: a NaN in either argument gives NaN.
__device__ __forceinline__ double nanmax(double a, double b) { return (a != a || a > b) ? a : b; }

// 1/x: v_rcp_f64 refined by two Newton-Raphson steps.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// sqrt(x) for x >= 0 (NaN for x < 0): v_rsq_f64 refined by coupled
// Newton iterations on the root and half the inverse root.
__device__ __forceinline__ double root(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double hh = 0.5 * y;
    const double t = __builtin_fma(-g, hh, 0.5);
    g = __builtin_fma(g, t, g);
    hh = __builtin_fma(hh, t, hh);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, hh, g);
    d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, hh, g);
    return x == 0.0 ? 0.0 : g;
}

struct Prim {
    double rinv;  // 1 / rho
    double p;     // pressure
    double c;     // speed of sound
};

template <int NQ>
__device__ __forceinline__ Prim primitives(const double (&q)[NQ], double gamma) {
    Prim a;
    a.rinv = recip(q[0]);
    double m2 = q[1] * q[1] + q[2] * q[2];
    if constexpr (NQ == 5) m2 = m2 + q[3] * q[3];
    const double e = __builtin_fma(-0.5 * m2, a.rinv, q[NQ - 1]);  // E - |m|^2 / (2 rho)
    a.p = (gamma - 1.0) * e;
    a.c = root(gamma * a.p * a.rinv);
    return a;
}

template <int NQ>
__device__ __forceinline__ void euler_flux(const double (&q)[NQ], const Prim &a, int n, double (&f)[NQ],
                                           double &lam) {
    const double un = q[1 + n] * a.rinv;
    f[0] = q[1 + n];
#pragma unroll
    for (int b = 0; b < NQ - 2; ++b) f[1 + b] = (b == n) ? __builtin_fma(q[1 + b], un, a.p) : q[1 + b] * un;
    f[NQ - 1] = (q[NQ - 1] + a.p) * un;
    lam = __builtin_fabs(un) + a.c;
}

template <int NQ>
__device__ __forceinline__ void rusanov(const double (&qL)[NQ], const double (&fL)[NQ], double lL,
                                        const double (&qR)[NQ], const double (&fR)[NQ], double lR,
                                        double (&fh)[NQ]) {
    const double s = 0.5 * nanmax(lL, lR);
#pragma unroll
    for (int k = 0; k < NQ; ++k) fh[k] = __builtin_fma(-s, qR[k] - qL[k], 0.5 * (fL[k] + fR[k]));
}

// Largest wave speed of a volume over the axes n < D.
template <int D, int NQ>
__device__ __forceinline__ double volume_lambda(const double (&q)[NQ], double gamma) {
    const Prim a = primitives<NQ>(q, gamma);
    double l = 0.0;
#pragma unroll
    for (int n = 0; n < D; ++n) l = nanmax(l, __builtin_fabs(q[1 + n] * a.rinv) + a.c);
    return l;
}

// new state: Q + r * D, with D the difference-first sum of the axis terms
template <int NQ>
__device__ __forceinline__ void advance(const double (&q)[NQ], const double (&d)[NQ], double r, double (&qn)[NQ]) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) qn[k] = __builtin_fma(r, d[k], q[k]);
}

#pragma clang fp contract(on)

template <int NQ>
__device__ __forceinline__ void load_volume(const double *__restrict__ src, double (&q)[NQ]) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[k] = src[k];
}

template <int NQ>
__device__ __forceinline__ void store_volume(double *__restrict__ dst, const double (&q)[NQ]) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) dst[k] = q[k];
}

// Benign state for lanes with nothing to load (keeps their arithmetic finite).
template <int NQ>
__device__ __forceinline__ void rest_state(double (&q)[NQ]) {
    q[0] = 1.0;
#pragma unroll
    for (int k = 1; k < NQ - 1; ++k) q[k] = 0.0;
    q[NQ - 1] = 2.5;
}

}  // namespace fv
