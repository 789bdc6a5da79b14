// fv_pde.h -- user terms of the PDEs the generic patch-update kernel solves
// (library-private; the built-in instances of the microkernel interface).
//
// The paper's engine assembles its solver from user-supplied terms of Eq. 1:
// the flux F_n, the non-conservative product B_n(Q) dQ/dx_n, the source S and
// the largest wave speed lambda_max,n (Sec. 2.2).  A PDE type for the generic
// kernel supplies them as static device functions:
//
//   NQ                unknowns stored per volume; the first NV are evolved,
//   NV                the rest are parameters carried along unchanged (the
//                     bathymetry of the shallow water equations)
//   kFlux, kNcp, kSource   which terms exist
//   Params            trivially copyable parameters (kernel argument)
//   Cache             what the terms of one volume share (Euler: 1/rho, p, c)
//   prepare(q, prm)                      -> Cache
//   flux(q, cache, n, f[NV], lam, prm)   F_n(q) (zeros without a flux) and lambda_n(q)
//   ncp(qbar, dq, n, b[NV], prm)         B_n(qbar) dq
//   source(q, s[NV], prm)                S(q)
//   max_lambda<D>(q, prm)                max over n < D of lambda_n(q)
//
// The face terms the kernel forms from them (the central jump reading of the
// non-conservative product; with B = 0 this is exactly Eq. 2):
//   Fhat = 1/2 (F_n(Q_L) + F_n(Q_R)) - 1/2 max(lambda_L, lambda_R) (Q_R - Q_L)
//   G+   = Fhat - 1/2 B_n(Qbar) (Q_R - Q_L)      received by the volume right of the face
//   G-   = Fhat + 1/2 B_n(Qbar) (Q_R - Q_L)      lost by the volume left of it
//   Q_new = Q + (dt/h) sum_n [G+(c - e_n/2) - G-(c + e_n/2)] + dt S(Q)
//
// A new PDE is a new type of this shape; instantiating the kernel template on
// it (fv_update.hip) gives its solver.
#pragma once

#include <hip/hip_runtime.h>

#include "fv_physics.h"

namespace fv {

#pragma clang fp contract(off)

// The compressible Euler equations (the paper's experiments), N = 5 or 4.
template <int NQ_>
struct EulerPDE {
    static constexpr int NQ = NQ_, NV = NQ_;
    static constexpr bool kFlux = true, kNcp = false, kSource = false;
    struct Params {
        double gamma;
    };
    using Cache = Prim;
    __device__ static Cache prepare(const double (&q)[NQ], const Params &pr) { return primitives<NQ>(q, pr.gamma); }
    __device__ static void flux(const double (&q)[NQ], const Cache &a, int n, double (&f)[NV], double &lam,
                                const Params &) {
        euler_flux<NQ>(q, a, n, f, lam);
    }
    __device__ static void ncp(const double (&)[NQ], const double (&)[NQ], int, double (&b)[NV], const Params &) {
#pragma unroll
        for (int k = 0; k < NV; ++k) b[k] = 0.0;
    }
    __device__ static void source(const double (&)[NQ], double (&s)[NV], const Params &) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] = 0.0;
    }
    template <int D>
    __device__ static double max_lambda(const double (&q)[NQ], const Params &pr) {
        return volume_lambda<D, NQ>(q, pr.gamma);
    }
};

// 2D shallow water over a bathymetry b: Q = (h, hu, hv, b), b not evolved.
//   F_x = (hu, hu u, hv u), F_y = (hv, hu v, hv v); hydrostatic pressure as the
//   non-conservative product B_n dQ/dx_n = g h d(h + b)/dx_n in the n-momentum;
//   Coriolis S = (0, f hv, -f hu); lambda_n = |u_n| + sqrt(g h).
struct ShallowWaterPDE {
    static constexpr int NQ = 4, NV = 3;
    static constexpr bool kFlux = true, kNcp = true, kSource = true;
    struct Params {
        double g;
        double f;
    };
    struct Cache {
        double hinv;  // 1 / h
        double c;     // sqrt(g h)
    };
    __device__ static Cache prepare(const double (&q)[NQ], const Params &pr) {
        Cache a;
        a.hinv = recip(q[0]);
        a.c = root(pr.g * q[0]);
        return a;
    }
    __device__ static void flux(const double (&q)[NQ], const Cache &a, int n, double (&f)[NV], double &lam,
                                const Params &) {
        const double un = q[1 + n] * a.hinv;
        f[0] = q[1 + n];
        f[1] = q[1] * un;
        f[2] = q[2] * un;
        lam = __builtin_fabs(un) + a.c;
    }
    __device__ static void ncp(const double (&qbar)[NQ], const double (&dq)[NQ], int n, double (&b)[NV],
                               const Params &pr) {
        const double hydro = pr.g * qbar[0] * (dq[0] + dq[3]);
        b[0] = 0.0;
        b[1] = (n == 0) ? hydro : 0.0;
        b[2] = (n == 1) ? hydro : 0.0;
    }
    __device__ static void source(const double (&q)[NQ], double (&s)[NV], const Params &pr) {
        s[0] = 0.0;
        s[1] = pr.f * q[2];
        s[2] = -pr.f * q[1];
    }
    template <int D>
    __device__ static double max_lambda(const double (&q)[NQ], const Params &pr) {
        const Cache a = prepare(q, pr);
        double l = 0.0;
#pragma unroll
        for (int n = 0; n < D; ++n) l = nanmax(l, __builtin_fabs(q[1 + n] * a.hinv) + a.c);
        return l;
    }
};

// Linear advection dq/dt + a . grad q = 0: F_n = a_n q, lambda_n = |a_n|.
struct AdvectionPDE {
    static constexpr int NQ = 1, NV = 1;
    static constexpr bool kFlux = true, kNcp = false, kSource = false;
    struct Params {
        double a[3];
    };
    struct Cache {};
    __device__ static Cache prepare(const double (&)[NQ], const Params &) { return Cache{}; }
    __device__ static void flux(const double (&q)[NQ], const Cache &, int n, double (&f)[NV], double &lam,
                                const Params &pr) {
        f[0] = pr.a[n] * q[0];
        lam = __builtin_fabs(pr.a[n]);
    }
    __device__ static void ncp(const double (&)[NQ], const double (&)[NQ], int, double (&b)[NV], const Params &) {
        b[0] = 0.0;
    }
    __device__ static void source(const double (&)[NQ], double (&s)[NV], const Params &) { s[0] = 0.0; }
    template <int D>
    __device__ static double max_lambda(const double (&)[NQ], const Params &pr) {
        double l = 0.0;
#pragma unroll
        for (int n = 0; n < D; ++n) l = nanmax(l, __builtin_fabs(pr.a[n]));
        return l;
    }
};

// Linear acoustics, Q = (p, u_1 .. u_D): dp/dt + K0 div u = 0, du/dt + grad p / rho0 = 0.
// NCP_FORM = false: F_n = (K0 u_n, p / rho0 e_n); true: the same system written as
// B_n dQ/dx_n with F = 0.  lambda_n = c = sqrt(K0 / rho0) (a parameter).
template <int D, bool NCP_FORM>
struct AcousticsPDE {
    static constexpr int NQ = 1 + D, NV = 1 + D;
    static constexpr bool kFlux = !NCP_FORM, kNcp = NCP_FORM, kSource = false;
    struct Params {
        double rho0;
        double K0;
        double c;  // sqrt(K0 / rho0)
    };
    struct Cache {};
    __device__ static Cache prepare(const double (&)[NQ], const Params &) { return Cache{}; }
    __device__ static void flux(const double (&q)[NQ], const Cache &, int n, double (&f)[NV], double &lam,
                                const Params &pr) {
        if constexpr (NCP_FORM) {
#pragma unroll
            for (int k = 0; k < NV; ++k) f[k] = 0.0;
        } else {
            f[0] = pr.K0 * q[1 + n];
#pragma unroll
            for (int a = 0; a < D; ++a) f[1 + a] = (a == n) ? q[0] / pr.rho0 : 0.0;
        }
        lam = pr.c;
    }
    __device__ static void ncp(const double (&)[NQ], const double (&dq)[NQ], int n, double (&b)[NV],
                               const Params &pr) {
        b[0] = pr.K0 * dq[1 + n];
#pragma unroll
        for (int a = 0; a < D; ++a) b[1 + a] = (a == n) ? dq[0] / pr.rho0 : 0.0;
    }
    __device__ static void source(const double (&)[NQ], double (&s)[NV], const Params &) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] = 0.0;
    }
    template <int DD>
    __device__ static double max_lambda(const double (&)[NQ], const Params &pr) {
        return pr.c;
    }
};

// The two face values of one face from the user terms of its two volumes
// (F and lambda already evaluated): gp for the right volume, gm for the left.
template <class PDE>
__device__ __forceinline__ void face_terms(const double (&qL)[PDE::NQ], const double (&fL)[PDE::NV], double lL,
                                           const double (&qR)[PDE::NQ], const double (&fR)[PDE::NV], double lR,
                                           int n, const typename PDE::Params &pr, double (&gp)[PDE::NV],
                                           double (&gm)[PDE::NV]) {
    const double s = 0.5 * nanmax(lL, lR);
#pragma unroll
    for (int k = 0; k < PDE::NV; ++k) gp[k] = __builtin_fma(-s, qR[k] - qL[k], 0.5 * (fL[k] + fR[k]));
    if constexpr (PDE::kNcp) {
        double qbar[PDE::NQ], dq[PDE::NQ], b[PDE::NV];
#pragma unroll
        for (int k = 0; k < PDE::NQ; ++k) {
            qbar[k] = 0.5 * (qL[k] + qR[k]);
            dq[k] = qR[k] - qL[k];
        }
        PDE::ncp(qbar, dq, n, b, pr);
#pragma unroll
        for (int k = 0; k < PDE::NV; ++k) {
            gm[k] = __builtin_fma(0.5, b[k], gp[k]);
            gp[k] = __builtin_fma(-0.5, b[k], gp[k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < PDE::NV; ++k) gm[k] = gp[k];
    }
}

// New state of a volume: Q + r D over the evolved unknowns (+ dt S(Q)); the
// parameter unknowns keep their values.
template <class PDE>
__device__ __forceinline__ void advance_pde(const double (&q)[PDE::NQ], const double (&d)[PDE::NV], double r,
                                            double dt, const typename PDE::Params &pr, double (&qn)[PDE::NQ]) {
#pragma unroll
    for (int k = 0; k < PDE::NV; ++k) qn[k] = __builtin_fma(r, d[k], q[k]);
    if constexpr (PDE::kSource) {
        double s[PDE::NV];
        PDE::source(q, s, pr);
#pragma unroll
        for (int k = 0; k < PDE::NV; ++k) qn[k] = __builtin_fma(dt, s[k], qn[k]);
    }
#pragma unroll
    for (int k = PDE::NV; k < PDE::NQ; ++k) qn[k] = q[k];
}

#pragma clang fp contract(on)

}  // namespace fv
