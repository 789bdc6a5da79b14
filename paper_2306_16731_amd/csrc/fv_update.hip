// fv_update.hip -- fused patch-update kernel for gfx950 (CDNA4, wave64).
//
// One explicit Euler step of the Rusanov Finite Volume scheme for the
// compressible Euler equations over a batch of halo-padded patches, FP64:
//   Q_new(c) = Q(c) + (dt/h) ((D_x + D_y) + D_z),
//   D_n      = Fhat_n(c - e_n/2) - Fhat_n(c + e_n/2)                (Sec. 2.2, Alg. 1)
//   Fhat     = 1/2 (F_n(Q_L) + F_n(Q_R)) - 1/2 max(l_n(Q_L), l_n(Q_R)) (Q_R - Q_L)  (Eq. 2)
//   l_n      = |u_n| + c                                            (Sec. 2.2)
// plus the per-patch maximum of l_n over the new interior (end of Sec. 2.2).
//
// Work mapping.  A patch's lanes cover its cross-section plane, halo volumes
// included: (p+2) lanes along x in 2D, (p+2)^2 lanes over (x, y) in 3D.  Each
// lane marches along the last axis (y in 2D, z in 3D) through the p+2 layers
// of the patch.  At every layer a lane
//   1. reads its volume (the next layer's read is already in flight),
//   2. evaluates the user terms once: 1/rho, p, c, then F_n and l_n for the
//      axes its volume's faces need,
//   3. publishes (Q, F_n, l_n) of the in-plane axes in LDS and computes the
//      in-plane face to its left from its neighbour's entry -- every face flux
//      is formed exactly once and read back by the volume on its other side,
//   4. forms the marching-axis face below it from the previous layer, kept in
//      registers, and
//   5. completes the volume of the previous layer, stores it, and folds its
//      wave speeds into a running maximum.
// Only interior and face-halo volumes are ever read; corner / edge halo
// volumes are skipped.  Several patches share a block when they fit.
//
// Arithmetic.  The Euler terms are written with explicit fused multiply-adds
// and contraction disabled, so every code path (in-plane or marching axis,
// halo or interior lane) rounds identically: constant states are reproduced
// bitwise, mirror images and x/y swaps give bitwise mirrored results.  The
// kernel is HBM bound (no dense contraction, no MFMA).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_internal.h"
#include "fv_pde.h"
#include "fv_physics.h"

namespace fv {
namespace {

constexpr uint32_t kPeriodic = 0x2u;

// Barrier for LDS traffic only: waits for this wave's LDS operations, not for
// its outstanding global loads (the next layer's prefetch stays in flight).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS per lane (structure of arrays over the block's lanes, so consecutive
// lanes hit consecutive 8-byte words):
//   XQ[NQ], XF[D-1][NV], XL[D-1]   the volume's state and in-plane user terms
//   FP[D-1][NV]                    G+ of the in-plane face to the lane's left
//   FM[D-1][NV]                    G- of that face (PDEs with a non-conservative
//                                  product; otherwise G- = G+ and FP serves both)
template <int D, class PDE>
struct Lds {
    static constexpr int kXQ = 0;
    static constexpr int kXF = PDE::NQ;
    static constexpr int kXL = kXF + (D - 1) * PDE::NV;
    static constexpr int kFP = kXL + (D - 1);
    static constexpr int kFM = kFP + (D - 1) * PDE::NV;
    static constexpr int kWords = kFM + (PDE::kNcp ? (D - 1) * PDE::NV : 0);
};

// The kernel for any PDE type of fv_pde.h (the generic solver of Eq. 1); the
// Euler instance is the Euler block kernel.
template <int D, class PDE, int MAXB>
__global__ void __launch_bounds__(MAXB)
update_kernel(const double *__restrict__ in, double *__restrict__ out,
              const int64_t *__restrict__ offsets, const int64_t *__restrict__ out_offsets,
              const int32_t *__restrict__ ids,
              int32_t num_items, int32_t P, int64_t stride, double r_host, const double *__restrict__ r_dev,
              typename PDE::Params prm, double dt, uint32_t flags, double *__restrict__ lambda_out) {
    constexpr int NQ = PDE::NQ, NV = PDE::NV;
    extern __shared__ double lds[];
    const double r = r_dev ? *r_dev : r_host;
    using L = Lds<D, PDE>;
    const int B = blockDim.x;
    const int W = P + 2;
    const int S = (D == 2) ? W : W * W;
    const int ppb = B / S;
    const int tid = threadIdx.x;
    const int slot = tid / S;
    const int l = tid - slot * S;
    const int i = (D == 2) ? l : l % W;
    const int j = (D == 2) ? 1 : l / W;
    const int64_t item = (int64_t)blockIdx.x * ppb + slot;
    const bool active = slot < ppb && item < num_items;

    const bool xin = i >= 1 && i <= P;
    const bool yin = j >= 1 && j <= P;
    const bool pint = xin && yin;                 // plane-interior lane
    const bool xhalo = !xin && yin;               // x face-halo lane
    const bool yhalo = (D == 3) && xin && !yin;   // y face-halo lane (3D)
    const bool used = active && (pint || xhalo || yhalo);

    const int64_t off = active ? (offsets ? offsets[item] : item * stride) : 0;
    const int64_t off_out = active ? (out_offsets ? out_offsets[item] : off) : 0;
    const int64_t lane_off = (D == 2) ? (int64_t)i * NQ : ((int64_t)j * W + i) * NQ;
    const int64_t layer = (int64_t)S * NQ;        // doubles between marching layers
    const double *src = in + off + lane_off;
    double *dst = out + off_out + lane_off;
    const bool periodic = (flags & kPeriodic) != 0;

    // Registers carried from one layer to the next (marching axis m = D-1).
    double qprev[NQ], fmprev[NV], lmprev = 0.0, gpprev[NV], dinprev[NV];
#pragma unroll
    for (int k = 0; k < NQ; ++k) qprev[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) { fmprev[k] = gpprev[k] = dinprev[k] = 0.0; }
    double lmax = 0.0;

    double qnext[NQ];
    if (used && pint) load_volume<NQ>(src, qnext);     // layer 0: only the plane interior

    for (int k = 0; k < W; ++k) {
        const bool inner = k >= 1 && k <= P;           // layer k is an interior layer
        const bool live = used && (pint || inner);
        double q[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) q[c] = qnext[c];
        // prefetch layer k + 1
        if (k + 1 < W) {
            const bool live1 = used && (pint || (k + 1 <= P));
            if (live1) load_volume<NQ>(src + (k + 1) * layer, qnext);
        }

        typename PDE::Cache a;
        double fm[NV], lm = 0.0;
        if (live) {
            a = PDE::prepare(q, prm);
            // in-plane user terms, published for the neighbours
            if (inner) {
#pragma unroll
                for (int c = 0; c < NQ; ++c) lds[(L::kXQ + c) * B + tid] = q[c];
#pragma unroll
                for (int n = 0; n < D - 1; ++n) {
                    const bool need = pint || (n == 0 ? xhalo : yhalo);
                    if (need) {
                        double f[NV], lam;
                        PDE::flux(q, a, n, f, lam, prm);
#pragma unroll
                        for (int c = 0; c < NV; ++c) lds[(L::kXF + n * NV + c) * B + tid] = f[c];
                        lds[(L::kXL + n) * B + tid] = lam;
                    }
                }
            }
            if (pint) PDE::flux(q, a, D - 1, fm, lm, prm);
        }
        lds_barrier();

        // in-plane face to the lane's left (faces at coordinate - 1/2, for
        // coordinates 1 .. p+1), formed once and published
        if (active && inner) {
#pragma unroll
            for (int n = 0; n < D - 1; ++n) {
                const int cn = (n == 0) ? i : j;
                const bool other_in = (n == 0) ? yin : xin;
                if (other_in && cn >= 1 && cn <= P + 1) {
                    const int nb = tid - ((n == 0) ? 1 : W);
                    double qL[NQ], fL[NV], fR[NV], lR, gp[NV], gm[NV];
#pragma unroll
                    for (int c = 0; c < NQ; ++c) qL[c] = lds[(L::kXQ + c) * B + nb];
#pragma unroll
                    for (int c = 0; c < NV; ++c) {
                        fL[c] = lds[(L::kXF + n * NV + c) * B + nb];
                        fR[c] = lds[(L::kXF + n * NV + c) * B + tid];
                    }
                    const double lL = lds[(L::kXL + n) * B + nb];
                    lR = lds[(L::kXL + n) * B + tid];
                    face_terms<PDE>(qL, fL, lL, q, fR, lR, n, prm, gp, gm);
#pragma unroll
                    for (int c = 0; c < NV; ++c) lds[(L::kFP + n * NV + c) * B + tid] = gp[c];
                    if constexpr (PDE::kNcp) {
#pragma unroll
                        for (int c = 0; c < NV; ++c) lds[(L::kFM + n * NV + c) * B + tid] = gm[c];
                    }
                }
            }
        }
        lds_barrier();

        if (active && pint) {
            // in-plane differences of this layer's volume: D_x (+ D_y)
            double din[NV];
#pragma unroll
            for (int c = 0; c < NV; ++c) din[c] = 0.0;
            if (inner) {
                constexpr int kRight = PDE::kNcp ? L::kFM : L::kFP;  // G- of the face to the right
#pragma unroll
                for (int n = 0; n < D - 1; ++n) {
                    const int nb = tid + ((n == 0) ? 1 : W);
#pragma unroll
                    for (int c = 0; c < NV; ++c) {
                        const double d = lds[(L::kFP + n * NV + c) * B + tid] - lds[(kRight + n * NV + c) * B + nb];
                        din[c] = (n == 0) ? d : din[c] + d;
                    }
                }
            }
            // marching-axis face between layers k-1 and k
            double gp[NV], gm[NV];
            if (k >= 1) face_terms<PDE>(qprev, fmprev, lmprev, q, fm, lm, D - 1, prm, gp, gm);
            // complete the volume of layer k-1
            if (k >= 2) {
                double qn[NQ], dsum[NV];
#pragma unroll
                for (int c = 0; c < NV; ++c) dsum[c] = dinprev[c] + (gpprev[c] - gm[c]);
                advance_pde<PDE>(qprev, dsum, r, dt, prm, qn);
                const int kk = k - 1;
                store_volume<NQ>(dst + kk * layer, qn);
                if (periodic) {
                    if (i == P) store_volume<NQ>(dst + kk * layer - (int64_t)P * NQ, qn);
                    if (i == 1) store_volume<NQ>(dst + kk * layer + (int64_t)P * NQ, qn);
                    if (D == 3) {
                        if (j == P) store_volume<NQ>(dst + kk * layer - (int64_t)P * W * NQ, qn);
                        if (j == 1) store_volume<NQ>(dst + kk * layer + (int64_t)P * W * NQ, qn);
                    }
                    if (kk == P) store_volume<NQ>(dst, qn);
                    if (kk == 1) store_volume<NQ>(dst + (int64_t)(P + 1) * layer, qn);
                }
                if (lambda_out) lmax = nanmax(lmax, PDE::template max_lambda<D>(qn, prm));
            }
#pragma unroll
            for (int c = 0; c < NQ; ++c) qprev[c] = q[c];
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                fmprev[c] = fm[c];
                gpprev[c] = gp[c];
                dinprev[c] = din[c];
            }
            lmprev = lm;
        }
    }

    if (lambda_out) {
        // per-patch maximum over the patch's lanes (NaN-propagating)
        lds[tid] = lmax;
        lds_barrier();
        if (active && l == 0) {
            double m = 0.0;
            for (int t = 0; t < S; ++t) m = nanmax(m, lds[tid + t]);
            lambda_out[ids ? ids[item] : item] = m;
        }
    }
}

template <int D, class PDE>
size_t pde_lds_bytes(int block) {
    return sizeof(double) * (size_t)Lds<D, PDE>::kWords * (size_t)block;
}

// Threads per block for the PDE's LDS footprint: the multiple of 64 that wastes the
// fewest lanes on partial patches while the block's LDS stays within 64 KiB.
template <int D, class PDE>
int pde_default_block(int p) {
    const int S = plane_lanes(p, D);
    int best = 0;
    double best_u = -1.0;
    for (int B = 64; B <= 1024; B += 64) {
        if (B < S) continue;
        if (pde_lds_bytes<D, PDE>(B) > 64 * 1024) break;
        const double u = (double)((B / S) * S) / B;
        if (u > best_u + 1e-9) { best_u = u; best = B; }
    }
    if (best == 0) best = ((S + 63) / 64) * 64;
    return best;
}

template <int D, class PDE>
hipError_t launch_typed(const UpdateLaunch &L, const typename PDE::Params &prm, hipStream_t stream) {
    const int S = plane_lanes(L.p, L.dim);
    const int B = L.block > 0 ? L.block
                              : (L.pde == 0 ? default_block(L.p, L.dim) : pde_default_block<D, PDE>(L.p));
    if (B % 64 != 0 || B > 1024 || B < S) return hipErrorInvalidConfiguration;
    const int ppb = B / S;
    const int64_t blocks = ((int64_t)L.num_items + ppb - 1) / ppb;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = pde_lds_bytes<D, PDE>(B);
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return hipErrorInvalidDevice;
    if (lds > (size_t)lds_max) return hipErrorInvalidConfiguration;
    if (lds > 64 * 1024) {
        const void *fn = B <= 256 ? reinterpret_cast<const void *>(&update_kernel<D, PDE, 256>)
                                  : reinterpret_cast<const void *>(&update_kernel<D, PDE, 1024>);
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (B <= 256)
        hipLaunchKernelGGL((update_kernel<D, PDE, 256>), dim3((unsigned)blocks), dim3(B), lds, stream,
                           L.in, L.out, L.offsets, L.out_offsets, L.ids, L.num_items, L.p, L.stride, L.r, L.r_dev,
                           prm, L.dt, L.flags, L.lambda_out);
    else
        hipLaunchKernelGGL((update_kernel<D, PDE, 1024>), dim3((unsigned)blocks), dim3(B), lds, stream,
                           L.in, L.out, L.offsets, L.out_offsets, L.ids, L.num_items, L.p, L.stride, L.r, L.r_dev,
                           prm, L.dt, L.flags, L.lambda_out);
    return hipGetLastError();
}

template <int D, int NQ>
hipError_t launch_euler(const UpdateLaunch &L, hipStream_t stream) {
    return launch_typed<D, EulerPDE<NQ>>(L, typename EulerPDE<NQ>::Params{L.gamma}, stream);
}

// The other built-in PDEs (FV_PDE_* of include/fvpatch.h): the 2D wave form and the 3D
// interior-mapped form where they are built, the plane-marching kernel otherwise.
hipError_t launch_pde(const UpdateLaunch &L, hipStream_t stream) {
    if (pde_wave_fits(L.pde, L.dim, L.p) && !L.r_dev) return launch_update2d_pde(L, stream);
    if (pde3d_fits(L.pde, L.dim, L.p) && !L.r_dev) return launch_update3d_pde(L, stream);
    const double *c = L.pde_prm;
    switch (L.pde) {
        case kPdeShallowWater:
            if (L.dim != 2) return hipErrorInvalidValue;
            return launch_typed<2, ShallowWaterPDE>(L, ShallowWaterPDE::Params{c[0], c[1]}, stream);
        case kPdeAdvection:
            if (L.dim == 2) return launch_typed<2, AdvectionPDE>(L, AdvectionPDE::Params{{c[0], c[1], c[2]}}, stream);
            return launch_typed<3, AdvectionPDE>(L, AdvectionPDE::Params{{c[0], c[1], c[2]}}, stream);
        case kPdeAcoustics:
            if (L.dim == 2)
                return launch_typed<2, AcousticsPDE<2, false>>(L, {c[0], c[1], c[2]}, stream);
            return launch_typed<3, AcousticsPDE<3, false>>(L, {c[0], c[1], c[2]}, stream);
        case kPdeAcousticsNcp:
            if (L.dim == 2)
                return launch_typed<2, AcousticsPDE<2, true>>(L, {c[0], c[1], c[2]}, stream);
            return launch_typed<3, AcousticsPDE<3, true>>(L, {c[0], c[1], c[2]}, stream);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace

int default_block(int p, int dim) {
    const int S = plane_lanes(p, dim);
    int best = 0;
    double best_u = -1.0;
    for (int B = 64; B <= 1024; B += 64) {
        if (B < S) continue;
        if (update_lds_bytes(dim, 5, B) > 64 * 1024) break;
        const double u = (double)((B / S) * S) / B;
        if (u > best_u + 1e-9) { best_u = u; best = B; }
    }
    if (best == 0) best = ((S + 63) / 64) * 64;
    return best;
}

size_t update_lds_bytes(int dim, int nq, int block) {
    const int words = (dim == 2) ? (nq == 5 ? Lds<2, EulerPDE<5>>::kWords : Lds<2, EulerPDE<4>>::kWords)
                                 : Lds<3, EulerPDE<5>>::kWords;
    return sizeof(double) * (size_t)words * (size_t)block;
}

size_t pde_min_lds_bytes(int pde, int dim, int p) {
    const int B = ((plane_lanes(p, dim) + 63) / 64) * 64;  // the smallest block holding one patch
    switch (pde) {
        case kPdeShallowWater: return pde_lds_bytes<2, ShallowWaterPDE>(B);
        case kPdeAdvection: return dim == 2 ? pde_lds_bytes<2, AdvectionPDE>(B) : pde_lds_bytes<3, AdvectionPDE>(B);
        case kPdeAcoustics:
            return dim == 2 ? pde_lds_bytes<2, AcousticsPDE<2, false>>(B) : pde_lds_bytes<3, AcousticsPDE<3, false>>(B);
        case kPdeAcousticsNcp:
            return dim == 2 ? pde_lds_bytes<2, AcousticsPDE<2, true>>(B) : pde_lds_bytes<3, AcousticsPDE<3, true>>(B);
        default: return update_lds_bytes(dim, 5, B);
    }
}

hipError_t launch_update(const UpdateLaunch &L, hipStream_t stream) {
    if (L.num_items <= 0) return hipSuccess;
    if (L.pde != kPdeEuler) return launch_pde(L, stream);
    // kernel: 0 default, 1 block, 2 wave, 3 tile, 4 fixed-size wave (2D and 3D)
    if (L.dim == 2 && L.kernel == 2) return wave2d_fits(L.p) ? launch_update2d(L, stream) : hipErrorInvalidConfiguration;
    if (L.dim == 2 && L.kernel == 3) return tile2d_fits(L.p) ? launch_update2d_tile(L, stream) : hipErrorInvalidConfiguration;
    if (L.dim == 2 && L.kernel == 4)
        return wave2d_fixed(L.p, L.nq) ? launch_update2d_fixed(L, stream) : hipErrorInvalidConfiguration;
    if (L.dim == 3 && L.kernel == 4)
        return wave3d_fixed(L.p, L.nq) ? launch_update3d_fixed(L, stream) : hipErrorInvalidConfiguration;
    if (L.dim == 2 && L.kernel == 0 && wave2d_fixed(L.p, L.nq)) return launch_update2d_fixed(L, stream);
    if (L.dim == 3 && L.kernel == 0 && wave3d_fixed(L.p, L.nq)) return launch_update3d_fixed(L, stream);
    if (L.dim == 2 && L.kernel == 0 && wave2d_fits(L.p)) return launch_update2d(L, stream);
    if (L.dim == 2 && L.nq == 5) return launch_euler<2, 5>(L, stream);
    if (L.dim == 2 && L.nq == 4) return launch_euler<2, 4>(L, stream);
    if (L.dim == 3 && L.nq == 5) return launch_euler<3, 5>(L, stream);
    return hipErrorInvalidValue;
}

}  // namespace fv
