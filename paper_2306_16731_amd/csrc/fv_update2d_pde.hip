// fv_update2d_pde.hip -- the 2D wave form for the other PDEs of Eq. 1.
//
// The fixed-size 2D wave kernel's design (every padded patch row inside one
// wavefront, one lane per column including the two halo columns, a march up
// the rows with the user terms of every volume evaluated once) instantiated
// on the PDE types of fv_pde.h instead of the Euler terms:
//
//   row k:  read row k (row k+1 already in flight)
//           user terms once: prepare, F_x and l_x, F_y and l_y
//           x face to the left of each lane from the lane to its left (DPP):
//             (G+, G-) = Fhat -/+ 1/2 B_x(Qbar) (Q_R - Q_L)
//           D_x = G+ of the left face - G- of the right face (the right
//             lane's left face, second DPP shift)
//           y face between rows k-1 and k from registers; complete row k-1:
//             Q + (dt/h) (D_x + D_y) (+ dt S(Q)), parameter unknowns kept,
//             into an LDS ring of R rows per patch
//           every R rows: write the ring out as contiguous chunks
//
// The faces are formed from the same states by the same face_terms /
// advance_pde as in the plane-marching kernel, in the same order, so both
// kernels give the same results bit for bit.  Built for p = 16 (18 lanes per
// patch, three patches per wave); other sizes take the plane-marching kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_internal.h"
#include "fv_pde.h"

namespace fv {
namespace {

constexpr uint32_t kPeriodicFlag = 0x2u;
constexpr int kPdeWaveP = 16;
constexpr int kPdeWaveBlock = 64;

// Cross-lane moves of a double through the DPP wave shifts, in uniform control
// flow; the lane at the wave's edge reads zero and no lane that receives it uses it.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double x) {
    const int2 v = __builtin_bit_cast(int2, x);
    const int lo = __builtin_amdgcn_mov_dpp(v.x, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(v.y, CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, make_int2(lo, hi));
}
__device__ __forceinline__ double left_lane(double x) { return dpp_shift<0x138>(x); }   // wave_shr:1
__device__ __forceinline__ double right_lane(double x) { return dpp_shift<0x130>(x); }  // wave_shl:1

__device__ __forceinline__ void lds_wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <class PDE, int P>
struct PdeWave {
    static constexpr int W = P + 2;
    static constexpr int ppw = 64 / W;             // patches per wave
    static constexpr int ROWD = W * PDE::NQ;       // doubles per padded row
    static constexpr int PF = 2;                   // rows in flight per lane
    static constexpr int R = P <= 12 ? P : 12;     // rows per burst
    static constexpr int ring_words = ppw * R * ROWD + ppw;
};

template <class PDE, int P, int VEC, bool PERIODIC>
__device__ __forceinline__ void wave_update_pde(const double *__restrict__ in, double *__restrict__ out,
                                                const int64_t *__restrict__ offsets,
                                                const int64_t *__restrict__ out_offsets,
                                                const int32_t *__restrict__ ids, int64_t item0, int64_t num_items,
                                                int64_t stride, double r, double dt,
                                                const typename PDE::Params &prm, double *__restrict__ lambda_out,
                                                double *ring) {
    using S = PdeWave<PDE, P>;
    constexpr int NQ = PDE::NQ, NV = PDE::NV;
    constexpr int W = S::W, ppw = S::ppw, ROWD = S::ROWD, PF = S::PF, R = S::R;
    static_assert(VEC == 1 || ROWD % 2 == 0, "16-byte bursts need whole 16-byte rows");
    typedef double dv2 __attribute__((ext_vector_type(2)));
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // lane-derived burst indices are formed at each burst, not kept
    const int slot = lane / W;
    const int i = lane - slot * W;
    const int64_t item = item0 + slot;
    const bool active = slot < ppw && item < num_items;
    const bool xin = i >= 1 && i <= P;
    const bool writer = active && xin;
    const int64_t self = active ? item : item0;
    const int64_t off = offsets ? offsets[self] : self * stride;
    const int64_t off_out = out_offsets ? out_offsets[self] : off;
    const double *src = in + off + (int64_t)i * NQ;

    int64_t *bases = reinterpret_cast<int64_t *>(ring + ppw * R * ROWD);
    lds_wave_fence();
    if (i == 0 && slot < ppw) bases[slot] = off_out;
    lds_wave_fence();

    double qprev[NQ], fyprev[NV], gpprev[NV], dxprev[NV];
    double lyprev = 0.0, lmax = 0.0;
#pragma unroll
    for (int c = 0; c < NQ; ++c) qprev[c] = 1.0;  // a finite state; the face it forms is never used
#pragma unroll
    for (int c = 0; c < NV; ++c) fyprev[c] = gpprev[c] = dxprev[c] = 0.0;

    double qbuf[PF][NQ];
#pragma unroll
    for (int m = 0; m < PF; ++m) load_volume<NQ>(src + (int64_t)(m < W ? m : W - 1) * ROWD, qbuf[m]);

#pragma unroll
    for (int k = 0; k < W; ++k) {
        double q[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) q[c] = qbuf[k % PF][c];
        load_volume<NQ>(src + (int64_t)(k + PF < W ? k + PF : W - 1) * ROWD, qbuf[k % PF]);

        const typename PDE::Cache a = PDE::prepare(q, prm);
        double fx[NV], lx, fy[NV], ly;
        PDE::flux(q, a, 0, fx, lx, prm);
        PDE::flux(q, a, 1, fy, ly, prm);
        double qL[NQ], fL[NV], gpx[NV], gmx[NV];
#pragma unroll
        for (int c = 0; c < NQ; ++c) qL[c] = left_lane(q[c]);
#pragma unroll
        for (int c = 0; c < NV; ++c) fL[c] = left_lane(fx[c]);
        const double lL = left_lane(lx);
        face_terms<PDE>(qL, fL, lL, q, fx, lx, 0, prm, gpx, gmx);
        double dx[NV], gpy[NV], gmy[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) dx[c] = gpx[c] - right_lane(gmx[c]);
        face_terms<PDE>(qprev, fyprev, lyprev, q, fy, ly, 1, prm, gpy, gmy);

        if (k >= 2) {
            const int kk = k - 1;         // output row completed at this row
            const int rr = (kk - 1) % R;  // its row in the ring
            if (writer) {
                double d[NV], qn[NQ];
#pragma unroll
                for (int c = 0; c < NV; ++c) d[c] = dxprev[c] + (gpprev[c] - gmy[c]);
                advance_pde<PDE>(qprev, d, r, dt, prm, qn);
                double *srow = ring + (slot * R + rr) * ROWD;
#pragma unroll
                for (int c = 0; c < NQ; ++c) srow[i * NQ + c] = qn[c];
                if (PERIODIC) {
                    if (i == P)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) srow[c] = qn[c];
                    if (i == 1)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) srow[(P + 1) * NQ + c] = qn[c];
                }
                if (lambda_out) lmax = nanmax(lmax, PDE::template max_lambda<2>(qn, prm));
            }
            if (rr == R - 1 || kk == P) {
                const int nrows = rr + 1;
                const int k0 = kk - rr;  // first output row in the ring
                int ln = lane;
                asm volatile("" : "+v"(ln));
                lds_wave_fence();
                if (PERIODIC) {
                    // whole rows (x-halo volumes hold their wrapped copies)
                    const int per = nrows * ROWD / VEC;
                    const int total = ppw * per;
#pragma unroll
                    for (int j = 0; j < (total + 63) / 64; ++j) {
                        const int c = ln + 64 * j < total ? ln + 64 * j : total - 1;
                        int sl = c / per;
                        const int rem = c - sl * per;
                        sl = item0 + sl < num_items ? sl : 0;
                        const int64_t base = bases[sl] + (int64_t)k0 * ROWD;
                        if constexpr (VEC == 2)
                            __builtin_nontemporal_store(reinterpret_cast<const dv2 *>(ring + sl * R * ROWD)[rem],
                                                        reinterpret_cast<dv2 *>(out + base) + rem);
                        else
                            __builtin_nontemporal_store(ring[sl * R * ROWD + rem], out + base + rem);
                    }
                    // y-halo rows: row P+1 takes row 1, row 0 takes row P (interior columns)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (h == 0 ? k0 != 1 : kk != P) continue;
                        const int from = h == 0 ? 0 : rr;
                        const int dest = h == 0 ? P + 1 : 0;
                        constexpr int iper = P * NQ;
                        constexpr int itotal = ppw * iper;
#pragma unroll
                        for (int j = 0; j < (itotal + 63) / 64; ++j) {
                            const int c = ln + 64 * j < itotal ? ln + 64 * j : itotal - 1;
                            int sl = c / iper;
                            const int d = c - sl * iper;
                            sl = item0 + sl < num_items ? sl : 0;
                            __builtin_nontemporal_store(ring[(sl * R + from) * ROWD + NQ + d],
                                                        out + bases[sl] + (int64_t)dest * ROWD + NQ + d);
                        }
                    }
                } else {
                    // interior volumes of each row
                    constexpr int inner = P * NQ;
                    const int per = nrows * inner;
                    const int total = ppw * per;
#pragma unroll
                    for (int j = 0; j < (total + 63) / 64; ++j) {
                        const int c = ln + 64 * j < total ? ln + 64 * j : total - 1;
                        int sl = c / per;
                        const int rem = c - sl * per;
                        const int rw = rem / inner, d = rem - rw * inner;
                        sl = item0 + sl < num_items ? sl : 0;
                        __builtin_nontemporal_store(ring[(sl * R + rw) * ROWD + NQ + d],
                                                    out + bases[sl] + (int64_t)(k0 + rw) * ROWD + NQ + d);
                    }
                }
                lds_wave_fence();
            }
        }
#pragma unroll
        for (int c = 0; c < NQ; ++c) qprev[c] = q[c];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            fyprev[c] = fy[c];
            gpprev[c] = gpy[c];
            dxprev[c] = dx[c];
        }
        lyprev = ly;
        __builtin_amdgcn_sched_barrier(0);
    }

    if (lambda_out) {
        for (int o = 1; o < W; o <<= 1) {
            const double other = __shfl_down(lmax, o, 64);
            if (i + o < W) lmax = nanmax(lmax, other);
        }
        if (active && i == 0) lambda_out[ids ? ids[item] : item] = lmax;
    }
}

template <class PDE, int P, int VEC, bool PERIODIC>
__global__ void __launch_bounds__(kPdeWaveBlock)
update2d_pde_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                    const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids, int32_t num_items,
                    int64_t stride, double r, double dt, typename PDE::Params prm, double *__restrict__ lambda_out) {
    extern __shared__ double lds[];
    constexpr int ppw = PdeWave<PDE, P>::ppw;
    const int64_t item0 = (int64_t)blockIdx.x * ppw;
    if (item0 >= num_items) return;
    wave_update_pde<PDE, P, VEC, PERIODIC>(in, out, offsets, out_offsets, ids, item0, num_items, stride, r, dt, prm,
                                           lambda_out, lds);
}

template <class PDE, int P, int VEC, bool PERIODIC>
void launch_pde_wave_form(const UpdateLaunch &L, const typename PDE::Params &prm, int64_t blocks, size_t lds,
                          hipStream_t stream) {
    hipLaunchKernelGGL((update2d_pde_kernel<PDE, P, VEC, PERIODIC>), dim3((unsigned)blocks), dim3(kPdeWaveBlock), lds,
                       stream, L.in, L.out, L.offsets, L.out_offsets, L.ids, L.num_items, L.stride, L.r, L.dt, prm,
                       L.lambda_out);
}

template <class PDE>
hipError_t launch_pde_wave(const UpdateLaunch &L, const typename PDE::Params &prm, hipStream_t stream) {
    constexpr int P = kPdeWaveP;
    using S = PdeWave<PDE, P>;
    const int64_t blocks = ((int64_t)L.num_items + S::ppw - 1) / S::ppw;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(double) * (size_t)S::ring_words;
    if ((L.flags & kPeriodicFlag) == 0) launch_pde_wave_form<PDE, P, 1, false>(L, prm, blocks, lds, stream);
    else if (L.vec2) launch_pde_wave_form<PDE, P, 2, true>(L, prm, blocks, lds, stream);
    else launch_pde_wave_form<PDE, P, 1, true>(L, prm, blocks, lds, stream);
    return hipGetLastError();
}

}  // namespace

bool pde_wave_fits(int pde, int dim, int p) {
    return dim == 2 && p == kPdeWaveP &&
           (pde == kPdeShallowWater || pde == kPdeAdvection || pde == kPdeAcoustics || pde == kPdeAcousticsNcp);
}

hipError_t launch_update2d_pde(const UpdateLaunch &L, hipStream_t stream) {
    if (!pde_wave_fits(L.pde, L.dim, L.p) || L.r_dev) return hipErrorInvalidValue;
    const double *c = L.pde_prm;
    switch (L.pde) {
        case kPdeShallowWater: return launch_pde_wave<ShallowWaterPDE>(L, {c[0], c[1]}, stream);
        case kPdeAdvection: return launch_pde_wave<AdvectionPDE>(L, AdvectionPDE::Params{{c[0], c[1], c[2]}}, stream);
        case kPdeAcoustics: return launch_pde_wave<AcousticsPDE<2, false>>(L, {c[0], c[1], c[2]}, stream);
        case kPdeAcousticsNcp: return launch_pde_wave<AcousticsPDE<2, true>>(L, {c[0], c[1], c[2]}, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace fv
