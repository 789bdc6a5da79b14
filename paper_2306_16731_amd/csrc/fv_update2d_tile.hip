// fv_update2d_tile.hip -- 2D patch update with a whole patch per tile.
//
// Same step as the other kernels (conservative update of Sec. 2.2 with the
// Rusanov flux of Eq. 2 and the Euler user terms; per-patch eigenvalue of the
// new state, end of Sec. 2.2).  A block holds G patches and one thread per
// interior volume.  Each patch is read from HBM in one coalesced burst into
// LDS and written back in one burst, so HBM sees few, large, nearby streams
// (a patch-row-at-a-time traversal keeps thousands of patches half-written
// and loses a quarter of the write bandwidth).
//
//   load      copy the padded patches into LDS (array of structures, as in HBM)
//   x phase   every volume that borders an x face evaluates F_x, l_x once
//             (interior volumes by their own thread, x-halo volumes in a
//             halo pass) and publishes them; each x face is formed once by
//             the volume on its right (the last one by the volume on its left)
//             and published; each volume takes D_x = left face - right face
//   y phase   the same along y
//   update    Q + (dt/h) (D_x + D_y), stored (and the periodic face halo);
//             the new volume's wave speed is folded into the patch maximum by
//             a segmented wave reduction and a 64-bit LDS max on the bit
//             pattern (exact for values >= 0, and NaN stays NaN)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fv_internal.h"
#include "fv_physics.h"

namespace fv {
namespace {

constexpr uint32_t kPeriodic = 0x2u;

__device__ __forceinline__ void block_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS words (doubles) per patch of a tile.
__host__ __device__ inline int tile_q_words(int P, int NQ) { return (P + 2) * (P + 2) * NQ; }
__host__ __device__ inline int tile_f_cells(int P) { return P * (P + 2); }  // volumes bordering faces of one axis
__host__ __device__ inline int tile_h_faces(int P) { return P * (P + 1); }  // faces of one axis
__host__ __device__ inline int tile_words(int P, int NQ) {
    return tile_q_words(P, NQ) + (NQ + 1) * tile_f_cells(P) + NQ * tile_h_faces(P);
}

// One axis phase of the tile kernel: publish the user terms along axis N of
// every volume bordering an N face, form every N face once, and return
// D_N = low face - high face of the calling thread's volume.
template <int NQ>
struct AxisTile {
    double *QS, *FB, *FH;
    const int64_t *POFF;
    const double *Qg;
    double *Fg, *Hg;
    int P, G, W, QW, FC, HF, B, tid, i, j;
    bool active;
    int hg, hn, hv, nh, stride_h;
    double gamma;

    // user-term slot of volume (a, b): x layout (b-1)(P+2) + a for a in [0, P+1];
    // y layout b P + (a-1) for b in [0, P+1]
    template <int N>
    __device__ __forceinline__ int slot(int a, int b) const { return N == 0 ? (b - 1) * W + a : b * P + (a - 1); }

    template <int N>
    __device__ __forceinline__ void phase(const double (&q)[NQ], const double (&f)[NQ], double l,
                                          const double (&hf)[NQ], double hl, double (&d)[NQ]) {
        if (active) {
            const int v = slot<N>(i, j);
#pragma unroll
            for (int k = 0; k < NQ; ++k) Fg[k * FC + v] = f[k];
            Fg[NQ * FC + v] = l;
        }
        if (hg >= 0 && hn == N) {
            double *F = FB + (size_t)hg * (NQ + 1) * FC;
#pragma unroll
            for (int k = 0; k < NQ; ++k) F[k * FC + hv] = hf[k];
            F[NQ * FC + hv] = hl;
        }
        // halo volumes beyond one per thread (only when 4 P G exceeds the block)
        for (int hh = tid + B * stride_h; hh < nh * stride_h; hh += B * stride_h) {
            const int hx = hh / stride_h;
            const int xg = hx / (4 * P);
            const int rem = hx - xg * 4 * P;
            const int side = rem / P;
            const int t = rem - side * P + 1;
            if ((side < 2 ? 0 : 1) != N || POFF[xg] < 0) continue;
            const int hi = side == 0 ? 0 : side == 1 ? P + 1 : t;
            const int hj = side == 2 ? 0 : side == 3 ? P + 1 : t;
            double hq[NQ], hf2[NQ], hl2;
            const double *src = QS + (size_t)xg * QW + (hj * W + hi) * NQ;
#pragma unroll
            for (int k = 0; k < NQ; ++k) hq[k] = src[k];
            const Prim a = primitives<NQ>(hq, gamma);
            euler_flux<NQ>(hq, a, N, hf2, hl2);
            double *F = FB + (size_t)xg * (NQ + 1) * FC;
            const int v = slot<N>(hi, hj);
#pragma unroll
            for (int k = 0; k < NQ; ++k) F[k * FC + v] = hf2[k];
            F[NQ * FC + v] = hl2;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");

        // faces: each volume forms its low face; the last volume along N also its high face
        //   x faces (i - 1/2, j): (j-1)(P+1) + (i-1);   y faces (i, j - 1/2): (j-1) P + (i-1)
        const int flo = N == 0 ? (j - 1) * (P + 1) + (i - 1) : (j - 1) * P + (i - 1);
        const int fhi = N == 0 ? flo + 1 : flo + P;
        if (active) {
            const int cn = N == 0 ? i : j;
            const int vlo = N == 0 ? slot<0>(i - 1, j) : slot<1>(i, j - 1);
            const int qlo = N == 0 ? (j * W + i - 1) * NQ : ((j - 1) * W + i) * NQ;
            double qo[NQ], fo[NQ], fh[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                qo[k] = Qg[qlo + k];
                fo[k] = Fg[k * FC + vlo];
            }
            rusanov<NQ>(qo, fo, Fg[NQ * FC + vlo], q, f, l, fh);
#pragma unroll
            for (int k = 0; k < NQ; ++k) Hg[k * HF + flo] = fh[k];
            if (cn == P) {
                const int vhi = N == 0 ? slot<0>(i + 1, j) : slot<1>(i, j + 1);
                const int qhi = N == 0 ? (j * W + i + 1) * NQ : ((j + 1) * W + i) * NQ;
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    qo[k] = Qg[qhi + k];
                    fo[k] = Fg[k * FC + vhi];
                }
                rusanov<NQ>(q, f, l, qo, fo, Fg[NQ * FC + vhi], fh);
#pragma unroll
                for (int k = 0; k < NQ; ++k) Hg[k * HF + fhi] = fh[k];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (active) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) d[k] = Hg[k * HF + flo] - Hg[k * HF + fhi];
        } else {
#pragma unroll
            for (int k = 0; k < NQ; ++k) d[k] = 0.0;
        }
    }
};

template <int NQ, int VEC>
__global__ void __launch_bounds__(1024)
update2d_tile_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                     const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids, int32_t num_items, int32_t P, int32_t G, int64_t stride,
                     double r_host, const double *__restrict__ r_dev, double gamma, uint32_t flags,
                     double *__restrict__ lambda_out) {
    extern __shared__ double lds[];
    const double r = r_dev ? *r_dev : r_host;
    const int B = blockDim.x;
    const int tid = threadIdx.x;
    const int C = P * P;
    const int W = P + 2;
    const int QW = tile_q_words(P, NQ);
    const int FC = tile_f_cells(P);
    const int HF = tile_h_faces(P);
    double *QS = lds;                              // [G][QW]
    double *FB = QS + (size_t)G * QW;              // [G][NQ+1][FC]  user terms F_n, l_n
    double *FH = FB + (size_t)G * (NQ + 1) * FC;   // [G][NQ][HF]    face fluxes
    int64_t *POFF = reinterpret_cast<int64_t *>(FH + (size_t)G * NQ * HF);  // [G] patch offsets
    int64_t *POUT = POFF + G;                                                       // [G] output offsets
    unsigned long long *PMAX = reinterpret_cast<unsigned long long *>(POUT + G);  // [G] lambda bits

    const int64_t item0 = (int64_t)blockIdx.x * G;
    if (tid < G) {
        const int64_t it = item0 + tid;
        POFF[tid] = it < num_items ? (offsets ? offsets[it] : it * stride) : -1;
        POUT[tid] = it < num_items ? (out_offsets ? out_offsets[it] : POFF[tid]) : -1;
        PMAX[tid] = 0ull;
    }
    block_lds_barrier();

    // ---- load: G padded patches into LDS.  Every lane keeps kBatch loads in
    // flight before it writes any of them (a load-then-store loop would pay
    // one HBM latency per element).  VEC = 2 moves 16 bytes per lane (all
    // patch offsets even), VEC = 1 moves 8 bytes.
    {
        constexpr int kBatch = 4;
        // native vector type: HIP's double2 is a union wrapper that keeps
        // arrays of it out of registers
        typedef double dvec2 __attribute__((ext_vector_type(2)));
        using vec_t = typename std::conditional<VEC == 2, dvec2, double>::type;
        const int nv = QW / VEC;                          // vectors per patch (QW is even for VEC = 2)
        const int total = G * nv;
        const float inv_nv = 1.0f / (float)nv;
        for (int base = 0; base < total; base += kBatch * B) {
            vec_t v[kBatch];
            int at[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int idx = base + u * B + tid;
                at[u] = -1;
                if (idx < total) {
                    int pg = (int)(((float)idx + 0.5f) * inv_nv);
                    const int d = idx - pg * nv;
                    const int64_t o = POFF[pg];
                    if (o >= 0) {
                        v[u] = reinterpret_cast<const vec_t *>(in + o)[d];
                        at[u] = idx;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u)
                if (at[u] >= 0) {
                    const int pg = (int)(((float)at[u] + 0.5f) * inv_nv);
                    reinterpret_cast<vec_t *>(QS + (size_t)pg * QW)[at[u] - pg * nv] = v[u];
                }
        }
    }
    block_lds_barrier();

    const int g = tid / C;
    const int c = tid - g * C;
    const int i = c % P + 1;
    const int j = c / P + 1;
    const bool active = g < G && POFF[g < G ? g : 0] >= 0;
    const int gg = active ? g : 0;
    double *Qg = QS + (size_t)gg * QW;
    double *Fg = FB + (size_t)gg * (NQ + 1) * FC;
    double *Hg = FH + (size_t)gg * NQ * HF;

    double q[NQ], fx[NQ], lx = 0.0, fy[NQ], ly = 0.0;
    if (active) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) q[k] = Qg[(j * W + i) * NQ + k];
        const Prim a = primitives<NQ>(q, gamma);
        euler_flux<NQ>(q, a, 0, fx, lx);
        euler_flux<NQ>(q, a, 1, fy, ly);
    } else {
        rest_state<NQ>(q);
        rest_state<NQ>(fx);
        rest_state<NQ>(fy);
    }
    // Face-halo volumes (4P per patch): halo h is owned by thread h * stride_h,
    // so the extra work is spread over every wave of the block.  Halo h of a
    // patch: side = h / P (0: i = 0, 1: i = P+1, 2: j = 0, 3: j = P+1), t = h % P + 1.
    const int nh = G * 4 * P;
    const int stride_h = nh > 0 && B / nh > 0 ? B / nh : 1;
    const int hidx = (tid % stride_h == 0) ? tid / stride_h : -1;
    int hg = -1, hn = 0, hv = 0;
    double hfl[NQ], hl = 0.0;
    if (hidx >= 0 && hidx < nh) {
        hg = hidx / (4 * P);
        const int rem = hidx - hg * 4 * P;
        const int side = rem / P;
        const int t = rem - side * P + 1;
        if (POFF[hg] >= 0) {
            hn = side < 2 ? 0 : 1;
            const int hi = side == 0 ? 0 : side == 1 ? P + 1 : t;
            const int hj = side == 2 ? 0 : side == 3 ? P + 1 : t;
            hv = hn == 0 ? (hj - 1) * W + hi : hj * P + (hi - 1);
            double hq[NQ];
            const double *src = QS + (size_t)hg * QW + (hj * W + hi) * NQ;
#pragma unroll
            for (int k = 0; k < NQ; ++k) hq[k] = src[k];
            const Prim a = primitives<NQ>(hq, gamma);
            euler_flux<NQ>(hq, a, hn, hfl, hl);
        } else {
            hg = -1;
        }
    }
    // halo volumes beyond one per thread (only when 4P G exceeds the block)
    double dx[NQ], dy[NQ];

    // ---- the two axis phases
    AxisTile<NQ> tile{QS, FB, FH, POFF, Qg, Fg, Hg, P, G, W, QW, FC, HF, B, tid, i, j, active,
                      hg, hn, hv, nh, stride_h, gamma};
    tile.template phase<0>(q, fx, lx, hfl, hl, dx);
    block_lds_barrier();  // x faces read before the y phase overwrites them
    tile.template phase<1>(q, fy, ly, hfl, hl, dy);

    // ---- update, store, eigenvalue of the new state
    double lam = 0.0;
    if (active) {
        double dsum[NQ], qn[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) dsum[k] = dx[k] + dy[k];
        advance<NQ>(q, dsum, r, qn);
        double *dst = out + POUT[g] + (j * W + i) * NQ;
        store_volume<NQ>(dst, qn);
        if (flags & kPeriodic) {
            if (i == P) store_volume<NQ>(dst - (int64_t)P * NQ, qn);
            if (i == 1) store_volume<NQ>(dst + (int64_t)P * NQ, qn);
            if (j == P) store_volume<NQ>(dst - (int64_t)P * W * NQ, qn);
            if (j == 1) store_volume<NQ>(dst + (int64_t)P * W * NQ, qn);
        }
        if (lambda_out) lam = volume_lambda<2, NQ>(qn, gamma);
    }
    if (lambda_out) {
        // segmented maximum within the wave over lanes of the same patch
        const int lane = tid & 63;
        unsigned long long bits = __builtin_bit_cast(unsigned long long, lam);
        const int myg = active ? g : -1;
        for (int o = 1; o < 64; o <<= 1) {
            const double other = __shfl_down(lam, o, 64);
            const int og = __shfl_down(myg, o, 64);
            if (lane + o < 64 && og == myg) lam = nanmax(lam, other);
        }
        bits = __builtin_bit_cast(unsigned long long, lam);
        const int prevg = __shfl_up(myg, 1, 64);
        const bool first = active && (lane == 0 || prevg != myg);
        if (first) atomicMax(&PMAX[g], bits);
        block_lds_barrier();
        if (tid < G && POFF[tid] >= 0) {
            const int64_t it = item0 + tid;
            lambda_out[ids ? ids[it] : it] = __builtin_bit_cast(double, PMAX[tid]);
        }
    }
}

}  // namespace

int tile2d_threads(int p) { return p * p; }

size_t tile2d_lds_bytes(int p, int nq, int G) {
    return sizeof(double) * (size_t)G * (size_t)tile_words(p, nq) + 24 * (size_t)G;
}

// Patches per block for a tile launch of `block` threads (0 when it does not fit).
int tile2d_patches_per_block(int p, int nq, int block, size_t lds_limit) {
    int G = block / (p * p);
    while (G > 0 && tile2d_lds_bytes(p, nq, G) > lds_limit) --G;
    return G;
}

int tile2d_default_block(int p) {
    const int C = p * p;
    if (C >= 128) return ((C + 63) / 64) * 64;
    int best = 64;
    double best_u = 0.0;
    for (int B = 64; B <= 256; B += 64) {
        const double u = (double)((B / C) * C) / B;
        if (u > best_u + 1e-9) { best_u = u; best = B; }
    }
    return best;
}

hipError_t launch_update2d_tile(const UpdateLaunch &L, hipStream_t stream) {
    const int p = L.p;
    const int B = L.block > 0 ? L.block : tile2d_default_block(p);
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return hipErrorInvalidDevice;
    if (B % 64 != 0 || B > 1024 || B < p * p) return hipErrorInvalidConfiguration;
    const int G = tile2d_patches_per_block(p, L.nq, B, (size_t)lds_max);
    if (G < 1) return hipErrorInvalidConfiguration;
    const size_t lds = tile2d_lds_bytes(p, L.nq, G);
    const int64_t blocks = ((int64_t)L.num_items + G - 1) / G;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const bool vec2 = L.vec2;
    const void *fn = L.nq == 5 ? (vec2 ? reinterpret_cast<const void *>(&update2d_tile_kernel<5, 2>)
                                       : reinterpret_cast<const void *>(&update2d_tile_kernel<5, 1>))
                               : (vec2 ? reinterpret_cast<const void *>(&update2d_tile_kernel<4, 2>)
                                       : reinterpret_cast<const void *>(&update2d_tile_kernel<4, 1>));
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
#define FV_TILE_LAUNCH(NQV, VV)                                                                                   \
    hipLaunchKernelGGL((update2d_tile_kernel<NQV, VV>), dim3((unsigned)blocks), dim3(B), lds, stream, L.in, L.out, \
                       L.offsets, L.out_offsets, L.ids, L.num_items, p, G, L.stride, L.r, L.r_dev, L.gamma, L.flags, \
                       L.lambda_out)
    if (L.nq == 5) {
        if (vec2) FV_TILE_LAUNCH(5, 2);
        else FV_TILE_LAUNCH(5, 1);
    } else if (L.nq == 4) {
        if (vec2) FV_TILE_LAUNCH(4, 2);
        else FV_TILE_LAUNCH(4, 1);
    } else {
        return hipErrorInvalidValue;
    }
#undef FV_TILE_LAUNCH
    return hipGetLastError();
}

}  // namespace fv
