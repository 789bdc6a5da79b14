// fv_update2d.hip -- 2D patch update with every patch row inside one wavefront.
//
// Same step as the generic kernel (conservative update of Sec. 2.2 with the
// Rusanov flux of Eq. 2, Euler user terms, per-patch eigenvalue of the new
// state), specialised for 2D patches whose padded row fits a wave64
// (p + 2 <= 64).  A wave holds floor(64 / (p+2)) patches side by side, one
// lane per column including the two halo columns, and marches up the rows:
//
//   layer k:  read row k (rows k+1 .. k+PF-1 already in flight)
//             user terms of every volume once: 1/rho, p, c, F_x, l_x, F_y, l_y
//             x face to the left of each lane from the lane to its left
//               (DPP wave shift: no LDS, no barrier)
//             D_x of each interior volume = its left face - the left face of
//               the lane to its right (second DPP shift)
//             y face between rows k-1 and k from registers
//             complete row k-1: Q + (dt/h) (D_x + D_y), store, fold l into the
//               patch maximum
//
// The waves of a block never synchronise with each other.  The per-patch
// maximum is a segmented tree reduction over the patch's lanes at the end.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_internal.h"
#include "fv_physics.h"

namespace fv {
namespace {

constexpr uint32_t kPeriodic = 0x2u;
constexpr int kDefaultPrefetch2d = 4;

// Cross-lane moves of a double through the DPP wave shifts.  They are issued
// in uniform control flow, so every source lane is enabled.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const int2 v = __builtin_bit_cast(int2, x);
    const int lo = __builtin_amdgcn_update_dpp(0, v.x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, v.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, make_int2(lo, hi));
}
__device__ __forceinline__ double from_left(double x) { return dpp_move<0x138>(x); }   // wave_shr:1
__device__ __forceinline__ double from_right(double x) { return dpp_move<0x130>(x); }  // wave_shl:1

template <int NQ, int PF>
__global__ void __launch_bounds__(256)
update2d_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                const int32_t *__restrict__ ids, int32_t num_items, int32_t P, int64_t stride, double r,
                double gamma, uint32_t flags, double *__restrict__ lambda_out) {
    const int W = P + 2;
    const int ppw = 64 / W;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int slot = lane / W;
    const int i = lane - slot * W;
    const int64_t item = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * ppw + slot;
    const bool active = slot < ppw && item < num_items;
    const bool xin = i >= 1 && i <= P;
    const bool writer = active && xin;

    const int64_t off = active ? (offsets ? offsets[item] : item * stride) : 0;
    const double *src = in + off + (int64_t)i * NQ;
    double *dst = out + off + (int64_t)i * NQ;
    const int64_t row = (int64_t)W * NQ;
    const bool periodic = (flags & kPeriodic) != 0;

    double qprev[NQ], fyprev[NQ], lyprev, fhprev[NQ], dxprev[NQ];
    rest_state<NQ>(qprev);
    rest_state<NQ>(fyprev);
    rest_state<NQ>(fhprev);
    rest_state<NQ>(dxprev);
    lyprev = 0.0;
    double lmax = 0.0;

    // Rows k .. k+PF-1 are in flight in registers while row k is processed.
    // Row 0 and row p+1 (y halo) are read in the interior columns only.
    double qbuf[PF][NQ];
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        if (m < W && active && (xin || (m >= 1 && m <= P))) load_volume<NQ>(src + m * row, qbuf[m]);
        else rest_state<NQ>(qbuf[m]);
    }

    for (int k = 0; k < W; ++k) {
        double q[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) q[c] = qbuf[0][c];
#pragma unroll
        for (int m = 0; m + 1 < PF; ++m)
#pragma unroll
            for (int c = 0; c < NQ; ++c) qbuf[m][c] = qbuf[m + 1][c];
        {
            const int kn = k + PF;
            if (kn < W && active && (xin || kn <= P)) load_volume<NQ>(src + kn * row, qbuf[PF - 1]);
            else rest_state<NQ>(qbuf[PF - 1]);
        }

        const Prim a = primitives<NQ>(q, gamma);
        double fx[NQ], lx, fy[NQ], ly;
        euler_flux<NQ>(q, a, 0, fx, lx);
        euler_flux<NQ>(q, a, 1, fy, ly);

        // x face at i - 1/2, formed once by the lane on its right
        double qL[NQ], fL[NQ], fhx[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            qL[c] = from_left(q[c]);
            fL[c] = from_left(fx[c]);
        }
        const double lL = from_left(lx);
        rusanov<NQ>(qL, fL, lL, q, fx, lx, fhx);
        double dx[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) dx[c] = fhx[c] - from_right(fhx[c]);

        // y face between rows k-1 and k
        double fh[NQ];
        rusanov<NQ>(qprev, fyprev, lyprev, q, fy, ly, fh);

        if (k >= 2 && writer) {
            double d[NQ], qn[NQ];
#pragma unroll
            for (int c = 0; c < NQ; ++c) d[c] = dxprev[c] + (fhprev[c] - fh[c]);
            advance<NQ>(qprev, d, r, qn);
            const int kk = k - 1;
            double *o = dst + kk * row;
            store_volume<NQ>(o, qn);
            if (periodic) {
                if (i == P) store_volume<NQ>(o - (int64_t)P * NQ, qn);
                if (i == 1) store_volume<NQ>(o + (int64_t)P * NQ, qn);
                if (kk == P) store_volume<NQ>(dst, qn);
                if (kk == 1) store_volume<NQ>(dst + (int64_t)(P + 1) * row, qn);
            }
            if (lambda_out) lmax = nanmax(lmax, volume_lambda<2, NQ>(qn, gamma));
        }
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            qprev[c] = q[c];
            fyprev[c] = fy[c];
            fhprev[c] = fh[c];
            dxprev[c] = dx[c];
        }
        lyprev = ly;
    }

    if (lambda_out) {
        // segmented maximum over the lanes of each patch: after the step with
        // offset o, lane i holds the maximum over columns [i, i + 2o - 1] of
        // its own patch
        for (int o = 1; o < W; o <<= 1) {
            const double other = __shfl_down(lmax, o, 64);
            if (i + o < W) lmax = nanmax(lmax, other);
        }
        if (active && i == 0) lambda_out[ids ? ids[item] : item] = lmax;
    }
}

template <int NQ, int PF>
hipError_t launch2d(const UpdateLaunch &L, hipStream_t stream) {
    const int W = L.p + 2;
    const int ppw = 64 / W;
    const int B = L.block > 0 ? L.block : 256;
    if (B % 64 != 0 || B > 256 || ppw < 1) return hipErrorInvalidConfiguration;
    const int per_block = (B / 64) * ppw;
    const int64_t blocks = ((int64_t)L.num_items + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((update2d_kernel<NQ, PF>), dim3((unsigned)blocks), dim3(B), 0, stream, L.in, L.out, L.offsets,
                       L.ids, L.num_items, L.p, L.stride, L.r, L.gamma, L.flags, L.lambda_out);
    return hipGetLastError();
}

}  // namespace

bool wave2d_fits(int p) { return p + 2 <= 64; }

template <int NQ>
hipError_t launch2d_pf(const UpdateLaunch &L, hipStream_t stream) {
    switch (L.prefetch > 0 ? L.prefetch : kDefaultPrefetch2d) {
        case 1: return launch2d<NQ, 1>(L, stream);
        case 2: return launch2d<NQ, 2>(L, stream);
        case 3: return launch2d<NQ, 3>(L, stream);
        case 4: return launch2d<NQ, 4>(L, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_update2d(const UpdateLaunch &L, hipStream_t stream) {
    if (L.nq == 5) return launch2d_pf<5>(L, stream);
    if (L.nq == 4) return launch2d_pf<4>(L, stream);
    return hipErrorInvalidValue;
}

}  // namespace fv
