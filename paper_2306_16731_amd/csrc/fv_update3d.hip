// fv_update3d.hip -- 3D patch update with a whole patch cross-section in one wavefront.
//
// Two lane mappings: the interior-mapped form (p = 4, 8; described at
// wave_update3d_i) and the pair-mapped form below (p = 6).
//
// The same step as the other kernels (conservative update of Sec. 2.2 with
// the Rusanov flux of Eq. 2 and the Euler user terms; per-patch eigenvalue
// of the new state), for small 3D patches: compile-time p with p + 2 even and
// (p + 2)^2 / 2 <= 64.  A lane owns two x-adjacent volumes (i = 2m, 2m + 1)
// of one row j of the cross-section, so a patch's (p + 2)^2 plane takes
// (p + 2)^2 / 2 lanes (50 for p = 8) and a wave holds floor(64 / that)
// patches.  The wave marches along z through the p + 2 layers:
//
//   layer k:  read layer k (layers k+1 .. k+PF-1 already in flight): each
//               lane reads its two volumes, 80 contiguous bytes, so the wave
//               reads the patch's 40 (p+2)^2-byte layer as one contiguous run
//             user terms of both volumes once: 1/rho, p, c, F and l per axis
//             x faces: the face between the lane's two volumes in registers,
//               the face to the left from the lane to the left (DPP shift),
//               the right face of the second volume from the lane to the
//               right (second DPP shift)
//             y faces: the lane p/2 + 1 positions down the wave holds row j-1
//               (ds_bpermute; no LDS allocation, no barrier)
//             z face between layers k-1 and k from registers
//             complete layer k-1 into an LDS ring of R layers, fold l into the
//               patch maximum
//             every R layers: write the ring in contiguous chunks
//
// As in the 2D fixed-size kernel, every loop has a static trip count and every
// global load and store is issued unconditionally (lanes without a patch read
// the wave's first patch, layers past the patch re-read its last layer, spare
// lanes of a burst repeat a chunk another lane writes with the same value), so
// the compiler counts outstanding memory operations exactly and the loads
// stay in flight across the bursts.  No block barriers: a wave is a block.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fv_internal.h"
#include "fv_pde.h"
#include "fv_physics.h"

namespace fv {
namespace {

constexpr uint32_t kPeriodic3 = 0x2u;
constexpr uint32_t kHaloFromIn3 = 0x4u;  // the output's halo volumes may take the input's values
constexpr int kBlock3 = 64;

template <int CTRL>
__device__ __forceinline__ double dpp3(double x) {
    const int2 v = __builtin_bit_cast(int2, x);
    const int lo = __builtin_amdgcn_mov_dpp(v.x, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(v.y, CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, make_int2(lo, hi));
}
__device__ __forceinline__ double lane_left(double x) { return dpp3<0x138>(x); }   // wave_shr:1
__device__ __forceinline__ double lane_right(double x) { return dpp3<0x130>(x); }  // wave_shl:1

// x from lane `src` (0 <= src < 64) through the LDS crossbar (ds_bpermute).
__device__ __forceinline__ double lane_from(double x, int src) {
    const int2 v = __builtin_bit_cast(int2, x);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, v.x);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, v.y);
    return __builtin_bit_cast(double, make_int2(lo, hi));
}

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <int P>
struct Shape3 {
    static constexpr int W = P + 2;
    static constexpr int H = W / 2;          // volume pairs per row
    static constexpr int LP = H * W;         // lanes per patch
    static constexpr int ppw = 64 / LP;      // patches per wave
    static constexpr int PLANE = W * W * 5;  // doubles per layer
    static constexpr int PF = 2;             // layers in flight per lane
    static constexpr int R = 2;              // layers per burst
    static constexpr int ring_words = ppw * R * PLANE + ppw;
    static_assert(W % 2 == 0 && ppw >= 1, "needs p + 2 even and (p + 2)^2 / 2 <= 64");
};

template <int NQ>
__device__ __forceinline__ void load_pair(const double *__restrict__ src, double (&q)[2][NQ]) {
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int c = 0; c < NQ; ++c) q[v][c] = src[v * NQ + c];
}

template <int NQ>
__device__ __forceinline__ void load_pair16(const double *__restrict__ src, double (&q)[2][NQ]) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    double t[2 * NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
        const dv2 x = reinterpret_cast<const dv2 *>(src)[c];
        t[2 * c] = x.x;
        t[2 * c + 1] = x.y;
    }
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int c = 0; c < NQ; ++c) q[v][c] = t[v * NQ + c];
}

// Copy `runs` runs of `len` doubles (run r starting at src_off(r) in the LDS
// layer and dst_off(r) in the patch) for every (slot, layer) of a burst.
// Spare lanes repeat the last chunk; chunks of slots without a patch repeat
// slot 0's.  VEC = 2 moves 16-byte chunks (len and both offsets even).
template <int VEC, int PPW, int NL, int RUNS, int LEN, class SrcOff, class DstOff>
__device__ __forceinline__ void burst(double *__restrict__ out, const double *ring, const int64_t *bases,
                                      int64_t item0, int64_t num_items, int lane, SrcOff src_off,
                                      DstOff dst_off) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    constexpr int per_run = LEN / VEC;
    constexpr int per_layer = RUNS * per_run;
    constexpr int per_slot = NL * per_layer;
    constexpr int total = PPW * per_slot;
#pragma unroll
    for (int jj = 0; jj < (total + 63) / 64; ++jj) {
        const int c = lane + 64 * jj < total ? lane + 64 * jj : total - 1;
        int sl = c / per_slot;
        int rem = c - sl * per_slot;
        const int ly = rem / per_layer;
        rem -= ly * per_layer;
        const int run = rem / per_run;
        const int e = (rem - run * per_run) * VEC;
        sl = item0 + sl < num_items ? sl : 0;
        const double *s = ring + src_off(sl, ly, run) + e;
        double *d = out + bases[sl] + dst_off(ly, run) + e;
        if constexpr (VEC == 2)
            __builtin_nontemporal_store(*reinterpret_cast<const dv2 *>(s), reinterpret_cast<dv2 *>(d));
        else
            __builtin_nontemporal_store(*s, d);
    }
}

// MESH: the face halos come from the neighbouring patches' interiors (a
// patch without a neighbour on a face keeps reading its own halo there), and
// patch t advances by dt[t] / h[t]; the output is the interior only.
template <int P, int VEC, bool PERIODIC, bool MESH = false>
__device__ __forceinline__ void wave_update3d(const double *__restrict__ in, double *__restrict__ out,
                                              const int64_t *__restrict__ offsets,
                                              const int64_t *__restrict__ out_offsets,
                                              const int32_t *__restrict__ ids, int64_t item0, int64_t num_items,
                                              int64_t stride, double r, double gamma,
                                              double *__restrict__ lambda_out, double *ring,
                                              MeshArgs mesh = MeshArgs{}) {
    static_assert(!(MESH && PERIODIC), "a mesh takes its halos from neighbours, not by self-wrap");
    using S = Shape3<P>;
    constexpr int NQ = 5;
    constexpr int W = S::W, H = S::H, LP = S::LP, ppw = S::ppw, PLANE = S::PLANE, PF = S::PF, R = S::R;
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int slot = lane / LP;
    const int l = lane - slot * LP;
    const int j = l / H;
    const int m = l - j * H;
    const int i0 = 2 * m;  // x index of the lane's first volume; the second is i0 + 1
    const int64_t item = item0 + slot;
    const bool active = slot < ppw && item < num_items;
    const bool yin = j >= 1 && j <= P;
    const bool int0 = active && yin && i0 >= 1;       // first volume in the plane interior
    const bool int1 = active && yin && i0 + 1 <= P;   // second volume in the plane interior
    const int64_t self = active ? item : item0;
    const int64_t off = offsets ? offsets[self] : self * stride;
    const int64_t off_out = out_offsets ? out_offsets[self] : off;
    const double *src = in + off + (int64_t)(j * W + i0) * NQ;
    // Mesh form: volume v of layer k is read at vbase[v][0] (k = 0), vbase[v][1] + k PLANE
    // (k = 1 .. p) or vbase[v][2] (k = p + 1): its own, or a neighbour's volume.
    const double *vbase[2][3];
    double ratio = r;  // dt / h of the lane's patch
    if constexpr (MESH) {
        const int32_t *nb = mesh.neighbors + 6 * self;
        auto base = [&](int32_t q) { return in + (offsets ? offsets[q >= 0 ? q : self] : (q >= 0 ? q : self) * stride); };
        const double *b[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) b[f] = base(nb[f]);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int i = i0 + v;
            const bool xi = i >= 1 && i <= P;
            const double *own = in + off + (int64_t)(j * W + i) * NQ;
            const double *mid = own;
            if (i == 0 && yin && nb[0] >= 0) mid = b[0] + (int64_t)(j * W + P) * NQ;
            if (i == W - 1 && yin && nb[1] >= 0) mid = b[1] + (int64_t)(j * W + 1) * NQ;
            if (j == 0 && xi && nb[2] >= 0) mid = b[2] + (int64_t)(P * W + i) * NQ;
            if (j == W - 1 && xi && nb[3] >= 0) mid = b[3] + (int64_t)(W + i) * NQ;
            vbase[v][1] = mid;
            vbase[v][0] = (xi && yin && nb[4] >= 0) ? b[4] + (int64_t)P * PLANE + (int64_t)(j * W + i) * NQ : own;
            vbase[v][2] = (xi && yin && nb[5] >= 0) ? b[5] + (int64_t)PLANE + (int64_t)(j * W + i) * NQ
                                                     : own + (int64_t)(W - 1) * PLANE;
        }
        ratio = mesh.dt[self] / mesh.h[self];
    }
    auto load_layer = [&](int k, double (&q)[2][NQ]) {
        if constexpr (MESH) {
#pragma unroll
            for (int v = 0; v < 2; ++v)
                load_volume<NQ>(k == 0 ? vbase[v][0] : (k == W - 1 ? vbase[v][2] : vbase[v][1] + (int64_t)k * PLANE),
                                q[v]);
        } else {
            const double *p = src + (int64_t)k * PLANE;
            if constexpr (VEC == 2) load_pair16<NQ>(p, q);
            else load_pair<NQ>(p, q);
        }
    };
    const int below = lane >= H ? lane - H : lane;    // row j - 1 of the same patch (j >= 1)
    const int above = lane + H < 64 ? lane + H : lane;  // row j + 1

    int64_t *bases = reinterpret_cast<int64_t *>(ring + ppw * R * PLANE);
    wave_fence();
    if (l == 0 && slot < ppw) bases[slot] = off_out;
    wave_fence();

    double qprev[2][NQ], fzprev[2][NQ], fhzprev[2][NQ], dprev[2][NQ], lzprev[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        rest_state<NQ>(qprev[v]);
        rest_state<NQ>(fzprev[v]);
        rest_state<NQ>(fhzprev[v]);
        rest_state<NQ>(dprev[v]);
        lzprev[v] = 0.0;
    }
    double lmax = 0.0;

    double qbuf[PF][2][NQ];
#pragma unroll
    for (int t = 0; t < PF; ++t) {
        load_layer(t < W ? t : W - 1, qbuf[t]);
    }

#pragma unroll
    for (int k = 0; k < W; ++k) {
        double q[2][NQ];
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int c = 0; c < NQ; ++c) q[v][c] = qbuf[k % PF][v][c];
        {
            load_layer(k + PF < W ? k + PF : W - 1, qbuf[k % PF]);
        }

        // Phases in this order keep few values alive at once: the primitives,
        // then the z face and the completion of layer k - 1 (its carried state
        // dies there), then the x and y differences of layer k.
        Prim a[2];
#pragma unroll
        for (int v = 0; v < 2; ++v) a[v] = primitives<NQ>(q[v], gamma);

        // z: the face between layers k - 1 and k
        double fz[2][NQ], lz[2], fhz[2][NQ];
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            euler_flux<NQ>(q[v], a[v], 2, fz[v], lz[v]);
            rusanov<NQ>(qprev[v], fzprev[v], lzprev[v], q[v], fz[v], lz[v], fhz[v]);
        }
        if (k >= 2) {
            const int kk = k - 1;         // layer completed now
            const int rr = (kk - 1) % R;  // its place in the ring
            double *lay = ring + (slot * R + rr) * PLANE;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                if (v == 0 ? int0 : int1) {
                    double dsum[NQ], qn[NQ];
#pragma unroll
                    for (int c = 0; c < NQ; ++c) dsum[c] = dprev[v][c] + (fhzprev[v][c] - fhz[v][c]);
                    advance<NQ>(qprev[v], dsum, ratio, qn);
                    const int i = i0 + v;
#pragma unroll
                    for (int c = 0; c < NQ; ++c) lay[(j * W + i) * NQ + c] = qn[c];
                    if (PERIODIC) {
                        // face-halo copies inside the layer (edges never)
                        if (i == P)
#pragma unroll
                            for (int c = 0; c < NQ; ++c) lay[(j * W) * NQ + c] = qn[c];
                        if (i == 1)
#pragma unroll
                            for (int c = 0; c < NQ; ++c) lay[(j * W + P + 1) * NQ + c] = qn[c];
                        if (j == P)
#pragma unroll
                            for (int c = 0; c < NQ; ++c) lay[i * NQ + c] = qn[c];
                        if (j == 1)
#pragma unroll
                            for (int c = 0; c < NQ; ++c) lay[((P + 1) * W + i) * NQ + c] = qn[c];
                    }
                    if (lambda_out) lmax = nanmax(lmax, volume_lambda<3, NQ>(qn, gamma));
                }
            }
            if (rr == R - 1 || kk == P) {
                const int nl = rr + 1;
                const int k0 = kk - rr;  // first layer in the ring
                int ln = lane;
                asm volatile("" : "+v"(ln));
                wave_fence();
                auto ring_layer = [&](int sl, int ly) { return (sl * R + ly) * PLANE; };
                if (PERIODIC) {
                    // rows 1 .. p whole (x face halos hold their copies), rows 0 and p+1 interior
                    auto body = [&](auto NLc) {
                        constexpr int NL = decltype(NLc)::value;
                        burst<VEC, ppw, NL, 1, P * W * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int ly, int) { return ring_layer(sl, ly) + W * NQ; },
                            [&](int ly, int) { return (int64_t)(k0 + ly) * PLANE + W * NQ; });
                        burst<1, ppw, NL, 2, P * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int ly, int run) { return ring_layer(sl, ly) + (run * (P + 1) * W + 1) * NQ; },
                            [&](int ly, int run) { return (int64_t)(k0 + ly) * PLANE + (run * (P + 1) * W + 1) * NQ; });
                    };
                    if (nl == R) body(std::integral_constant<int, R>{});
                    else body(std::integral_constant<int, 1>{});
                    // z face halos: layer p+1 takes layer 1, layer 0 takes layer p (plane interior)
#pragma unroll
                    for (int hz = 0; hz < 2; ++hz) {
                        if (hz == 0 ? k0 != 1 : kk != P) continue;
                        const int from = hz == 0 ? 0 : rr;
                        const int dest = hz == 0 ? P + 1 : 0;
                        burst<1, ppw, 1, P, P * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int, int run) { return ring_layer(sl, from) + ((run + 1) * W + 1) * NQ; },
                            [&](int, int run) { return (int64_t)dest * PLANE + ((run + 1) * W + 1) * NQ; });
                    }
                } else {
                    auto body = [&](auto NLc) {
                        constexpr int NL = decltype(NLc)::value;
                        burst<1, ppw, NL, P, P * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int ly, int run) { return ring_layer(sl, ly) + ((run + 1) * W + 1) * NQ; },
                            [&](int ly, int run) { return (int64_t)(k0 + ly) * PLANE + ((run + 1) * W + 1) * NQ; });
                    };
                    if (nl == R) body(std::integral_constant<int, R>{});
                    else body(std::integral_constant<int, 1>{});
                }
                wave_fence();
            }
        }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                qprev[v][c] = q[v][c];
                fzprev[v][c] = fz[v][c];
                fhzprev[v][c] = fhz[v][c];
            }
            lzprev[v] = lz[v];
        }
        __builtin_amdgcn_sched_barrier(0);

        // x: D_x = Fhat(i - 1/2) - Fhat(i + 1/2)
        double din[2][NQ];
        {
            double fx[2][NQ], lx[2], fmid[NQ], fleft[NQ], qL[NQ], fL[NQ];
#pragma unroll
            for (int v = 0; v < 2; ++v) euler_flux<NQ>(q[v], a[v], 0, fx[v], lx[v]);
            rusanov<NQ>(q[0], fx[0], lx[0], q[1], fx[1], lx[1], fmid);
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                qL[c] = lane_left(q[1][c]);
                fL[c] = lane_left(fx[1][c]);
            }
            rusanov<NQ>(qL, fL, lane_left(lx[1]), q[0], fx[0], lx[0], fleft);
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                din[0][c] = fleft[c] - fmid[c];
                din[1][c] = fmid[c] - lane_right(fleft[c]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // y: the face below each volume from row j - 1, the face above from row j + 1
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            double fy[NQ], ly, qS[NQ], fS[NQ], fbelow[NQ];
            euler_flux<NQ>(q[v], a[v], 1, fy, ly);
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                qS[c] = lane_from(q[v][c], below);
                fS[c] = lane_from(fy[c], below);
            }
            rusanov<NQ>(qS, fS, lane_from(ly, below), q[v], fy, ly, fbelow);
#pragma unroll
            for (int c = 0; c < NQ; ++c) dprev[v][c] = din[v][c] + (fbelow[c] - lane_from(fbelow[c], above));
        }
        __builtin_amdgcn_sched_barrier(0);
    }

    if (lambda_out) {
        // segmented maximum over the lanes of each patch
        for (int o = 1; o < LP; o <<= 1) {
            const double other = __shfl_down(lmax, o, 64);
            if (l + o < LP) lmax = nanmax(lmax, other);
        }
        if (active && l == 0) lambda_out[ids ? ids[item] : item] = lmax;
    }
}

// Interior-mapped form for p with p^2 dividing 64 (p = 4, 8): a lane owns ONE
// interior volume (i, j) of the cross-section, so a patch takes p^2 lanes
// (all 64 for p = 8, four patches per wave for p = 4) and no lane works on a
// halo or corner slot.  The face halos enter through the boundary lanes: a
// lane with i = 1 or i = p also reads the x face-halo volume beside it and
// forms that boundary face itself, likewise in y; z halos are the first and
// last layer of the march.  Per layer a lane evaluates its volume's user
// terms, its x face to the left (from the lane to the left by DPP, or from
// its halo volume) and its y face below (from the lane p positions down by
// ds_bpermute, or from its halo volume); the faces to the right and above
// come back from the neighbouring lanes, or from the boundary face.  Each
// face is the same Rusanov evaluation of the same two states as in the other
// kernels, so results are equal bit for bit.  The output goes through the
// same LDS ring and bursts as the pair-mapped form.
template <int P, int NQ = 5>
struct Shape3i {
    static constexpr int W = P + 2;
    static constexpr int LP = P * P;          // lanes per patch
    static constexpr int ppw = 64 / LP;       // patches per wave
    static constexpr int PLANE = W * W * NQ;  // doubles per layer
    static constexpr int PF = 1;             // layers in flight per lane (halos included: 15 doubles)
    static constexpr int R = 2;              // layers per burst
    static constexpr int ring_words = ppw * R * PLANE + ppw;
    // a burst of R interior layers without halos, in 8-byte chunks: per lane
    static constexpr int CHUNKS = ppw * R * P * P * NQ;
    static constexpr int ITERS = (CHUNKS + 63) / 64;
    static_assert(64 % LP == 0, "needs p^2 dividing 64");
    static_assert(P % R == 0, "bursts of whole rings");
};

template <class PDE, int P, int VEC, bool PERIODIC, bool MESH = false, bool WHOLE = false>
__device__ __forceinline__ void wave_update3d_i(const double *__restrict__ in, double *__restrict__ out,
                                                const int64_t *__restrict__ offsets,
                                                const int64_t *__restrict__ out_offsets,
                                                const int32_t *__restrict__ ids, int64_t item0, int64_t num_items,
                                                int64_t stride, double r, double dt,
                                                const typename PDE::Params &prm,
                                                double *__restrict__ lambda_out, double *ring,
                                                MeshArgs mesh = MeshArgs{}) {
    static_assert(!(MESH && PERIODIC), "a mesh takes its halos from neighbours, not by self-wrap");
    // WHOLE (without PERIODIC): the x-halo volumes of the interior rows of each interior layer go
    // out with their input values, so the rows 1 .. p of a layer are one contiguous run
    static_assert(!(WHOLE && (PERIODIC || MESH)), "whole rows are the non-periodic, non-mesh form");
    constexpr int NQ = PDE::NQ, NV = PDE::NV;
    using S = Shape3i<P, NQ>;
    constexpr int W = S::W, LP = S::LP, ppw = S::ppw, PLANE = S::PLANE, PF = S::PF, R = S::R;
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int slot = lane / LP;
    const int l = lane - slot * LP;
    const int j = 1 + l / P;
    const int i = 1 + (l - (j - 1) * P);
    const int64_t item = item0 + slot;
    const bool active = item < num_items;
    const int64_t self = active ? item : item0;
    const int64_t off = offsets ? offsets[self] : self * stride;
    const int64_t off_out = out_offsets ? out_offsets[self] : off;
    const bool xlo = i == 1, xhi = i == P, ylo = j == 1, yhi = j == P;
    // the lane's volume, its x and y face-halo volumes (its own volume where it has none), and
    // (mesh form) its volume's z neighbours in layers 0 and p + 1
    const double *own = in + off + (int64_t)(j * W + i) * NQ;
    const double *xh = in + off + (int64_t)(j * W + (xlo ? 0 : (xhi ? P + 1 : i))) * NQ;
    const double *yh = in + off + (int64_t)((ylo ? 0 : (yhi ? P + 1 : j)) * W + i) * NQ;
    const double *z0 = own, *zw = own + (int64_t)(W - 1) * PLANE;
    double ratio = r;  // dt / h of the lane's patch
    if constexpr (MESH) {
        const int32_t *nb = mesh.neighbors + 6 * self;
        auto base = [&](int32_t q) { return in + (offsets ? offsets[q >= 0 ? q : self] : (q >= 0 ? q : self) * stride); };
        if (xlo && nb[0] >= 0) xh = base(nb[0]) + (int64_t)(j * W + P) * NQ;
        if (xhi && nb[1] >= 0) xh = base(nb[1]) + (int64_t)(j * W + 1) * NQ;
        if (ylo && nb[2] >= 0) yh = base(nb[2]) + (int64_t)(P * W + i) * NQ;
        if (yhi && nb[3] >= 0) yh = base(nb[3]) + (int64_t)(W + i) * NQ;
        if (nb[4] >= 0) z0 = base(nb[4]) + (int64_t)P * PLANE + (int64_t)(j * W + i) * NQ;
        if (nb[5] >= 0) zw = base(nb[5]) + (int64_t)PLANE + (int64_t)(j * W + i) * NQ;
        ratio = mesh.dt[self] / mesh.h[self];
    }
    // layer k: the lane's volume (x = 0), its x halo (x = 1) and its y halo (x = 2); the halos
    // only for the interior layers 1 .. p
    auto load_layer = [&](int k, double (&q)[3][NQ]) {
        load_volume<NQ>(k == 0 ? z0 : (k == W - 1 ? zw : own + (int64_t)k * PLANE), q[0]);
        if (k >= 1 && k <= P) {
            load_volume<NQ>(xh + (int64_t)k * PLANE, q[1]);
            load_volume<NQ>(yh + (int64_t)k * PLANE, q[2]);
        }
    };
    const int below = lane >= P ? lane - P : lane;    // row j - 1 (used for j >= 2)
    const int above = lane + P < 64 ? lane + P : lane;  // row j + 1 (used for j <= p - 1)

    int64_t *bases = reinterpret_cast<int64_t *>(ring + ppw * R * PLANE);
    wave_fence();
    if (l == 0) bases[slot] = off_out;
    wave_fence();

    // Store table of the bursts without periodic halos: the ring holds layers in the patch's
    // own layout, so chunk c of a burst sits at the same offset q from the burst's first layer
    // in LDS and in the patch; entry jj = (slot << 12) | q for chunk lane + 64 jj (spare lanes
    // repeat the last chunk), two 16-bit entries per register.  Built once, it replaces the
    // per-burst index arithmetic.
    static_assert(2 * PLANE <= 4096 && ppw <= 16, "table entries take 12 + 4 bits");
    int tab[(S::ITERS + 1) / 2];
#pragma unroll
    for (int t = 0; t < (S::ITERS + 1) / 2; ++t) tab[t] = 0;
    if constexpr (!PERIODIC && !WHOLE) {
        constexpr int per_row = P * NQ, per_layer = P * per_row, per_slot = R * per_layer;
#pragma unroll
        for (int jj = 0; jj < S::ITERS; ++jj) {
            const int c = lane + 64 * jj < S::CHUNKS ? lane + 64 * jj : S::CHUNKS - 1;
            const int sl = c / per_slot;
            int rem = c - sl * per_slot;
            const int ly = rem / per_layer;
            rem -= ly * per_layer;
            const int row = rem / per_row;
            const int e = rem - row * per_row;
            tab[jj >> 1] |= ((sl << 12) | (ly * PLANE + ((row + 1) * W + 1) * NQ + e)) << (16 * (jj & 1));
        }
    }

    double qprev[NQ], fzprev[NV], gzprev[NV], dprev[NV], lzprev = 0.0;
    double qxprev[NQ];  // WHOLE: the lane's x-halo volume of the previous layer
#pragma unroll
    for (int c = 0; c < NQ; ++c) qprev[c] = qxprev[c] = 1.0;  // a finite state; the face it forms is never used
#pragma unroll
    for (int c = 0; c < NV; ++c) fzprev[c] = gzprev[c] = dprev[c] = 0.0;
    double lmax = 0.0;

    double qbuf[PF][3][NQ];
#pragma unroll
    for (int t = 0; t < PF; ++t) load_layer(t, qbuf[t]);

#pragma unroll
    for (int k = 0; k < W; ++k) {
        double q[NQ], qx[NQ], qy[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            q[c] = qbuf[k % PF][0][c];
            qx[c] = qbuf[k % PF][1][c];
            qy[c] = qbuf[k % PF][2][c];
        }
        if (k + PF < W) load_layer(k + PF, qbuf[k % PF]);

        const typename PDE::Cache a = PDE::prepare(q, prm);
        // z: the face between layers k - 1 and k (G+ for layer k, G- for layer k - 1)
        double fz[NV], lz, gpz[NV], gmz[NV];
        PDE::flux(q, a, 2, fz, lz, prm);
        face_terms<PDE>(qprev, fzprev, lzprev, q, fz, lz, 2, prm, gpz, gmz);
        if (k >= 2) {
            const int kk = k - 1;         // layer completed now
            const int rr = (kk - 1) % R;  // its place in the ring
            double *lay = ring + (slot * R + rr) * PLANE;
            if (active) {
                double dsum[NV], qn[NQ];
#pragma unroll
                for (int c = 0; c < NV; ++c) dsum[c] = dprev[c] + (gzprev[c] - gmz[c]);
                advance_pde<PDE>(qprev, dsum, ratio, dt, prm, qn);
#pragma unroll
                for (int c = 0; c < NQ; ++c) lay[(j * W + i) * NQ + c] = qn[c];
                if (PERIODIC) {
                    // face-halo copies inside the layer (edges never)
                    if (xhi)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) lay[(j * W) * NQ + c] = qn[c];
                    if (xlo)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) lay[(j * W + P + 1) * NQ + c] = qn[c];
                    if (yhi)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) lay[i * NQ + c] = qn[c];
                    if (ylo)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) lay[((P + 1) * W + i) * NQ + c] = qn[c];
                }
                if constexpr (WHOLE) {
                    // the x-halo volumes of this row, as read (left for xlo lanes, right for xhi)
                    if (xlo)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) lay[(j * W) * NQ + c] = qxprev[c];
                    if (xhi)
#pragma unroll
                        for (int c = 0; c < NQ; ++c) lay[(j * W + P + 1) * NQ + c] = qxprev[c];
                }
                if (lambda_out) lmax = nanmax(lmax, PDE::template max_lambda<3>(qn, prm));
            }
            if (rr == R - 1 || kk == P) {
                const int nl = rr + 1;
                const int k0 = kk - rr;  // first layer in the ring
                int ln = lane;
                asm volatile("" : "+v"(ln));
                wave_fence();
                auto ring_layer = [&](int sl, int ly) { return (sl * R + ly) * PLANE; };
                if constexpr (WHOLE) {
                    // rows 1 .. p of each layer, whole
                    auto body = [&](auto NLc) {
                        constexpr int NL = decltype(NLc)::value;
                        burst<VEC, ppw, NL, 1, P * W * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int ly, int) { return ring_layer(sl, ly) + W * NQ; },
                            [&](int ly, int) { return (int64_t)(k0 + ly) * PLANE + W * NQ; });
                    };
                    if (nl == R) body(std::integral_constant<int, R>{});
                    else body(std::integral_constant<int, 1>{});
                } else if (PERIODIC) {
                    auto body = [&](auto NLc) {
                        constexpr int NL = decltype(NLc)::value;
                        burst<VEC, ppw, NL, 1, P * W * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int ly, int) { return ring_layer(sl, ly) + W * NQ; },
                            [&](int ly, int) { return (int64_t)(k0 + ly) * PLANE + W * NQ; });
                        burst<1, ppw, NL, 2, P * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int ly, int run) { return ring_layer(sl, ly) + (run * (P + 1) * W + 1) * NQ; },
                            [&](int ly, int run) { return (int64_t)(k0 + ly) * PLANE + (run * (P + 1) * W + 1) * NQ; });
                    };
                    if (nl == R) body(std::integral_constant<int, R>{});
                    else body(std::integral_constant<int, 1>{});
#pragma unroll
                    for (int hz = 0; hz < 2; ++hz) {
                        if (hz == 0 ? k0 != 1 : kk != P) continue;
                        const int from = hz == 0 ? 0 : rr;
                        const int dest = hz == 0 ? P + 1 : 0;
                        burst<1, ppw, 1, P, P * NQ>(
                            out, ring, bases, item0, num_items, ln,
                            [&](int sl, int, int run) { return ring_layer(sl, from) + ((run + 1) * W + 1) * NQ; },
                            [&](int, int run) { return (int64_t)dest * PLANE + ((run + 1) * W + 1) * NQ; });
                    }
                } else {
                    // every burst holds R layers (p is a multiple of R): the table's chunks
                    (void)nl;
                    const int64_t layer0 = (int64_t)k0 * PLANE;
#pragma unroll
                    for (int jj = 0; jj < S::ITERS; ++jj) {
                        const int ent = (tab[jj >> 1] >> (16 * (jj & 1))) & 0xFFFF;
                        const int qoff = ent & 0xFFF;
                        int sl = ent >> 12;
                        sl = item0 + sl < num_items ? sl : 0;
                        const int64_t base = ppw == 1 ? off_out : bases[sl];
                        __builtin_nontemporal_store(ring[sl * R * PLANE + qoff], out + base + layer0 + qoff);
                    }
                }
                wave_fence();
            }
        }
#pragma unroll
        for (int c = 0; c < NQ; ++c) qprev[c] = q[c];
        if constexpr (WHOLE)
#pragma unroll
            for (int c = 0; c < NQ; ++c) qxprev[c] = qx[c];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            fzprev[c] = fz[c];
            gzprev[c] = gpz[c];
        }
        lzprev = lz;
        if (k == 0 || k == W - 1) continue;  // z halo layers: no in-plane faces
        __builtin_amdgcn_sched_barrier(0);

        // x: the face to the left from the lane to the left, or (i = 1) from the halo; the face
        // to the right from the lane to the right, or (i = p) the boundary face with the halo
        double din[NV];
        {
            double fx[NV], lx, fh[NV], lh, qL[NQ], fL[NV], gpl[NV], gml[NV], gpb[NV], gmb[NV];
            PDE::flux(q, a, 0, fx, lx, prm);
            const typename PDE::Cache ah = PDE::prepare(qx, prm);
            PDE::flux(qx, ah, 0, fh, lh, prm);
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                const double ql = lane_left(q[c]);
                qL[c] = xlo ? qx[c] : ql;
            }
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const double fl = lane_left(fx[c]);
                fL[c] = xlo ? fh[c] : fl;
            }
            const double ll = lane_left(lx);
            face_terms<PDE>(qL, fL, xlo ? lh : ll, q, fx, lx, 0, prm, gpl, gml);
            face_terms<PDE>(q, fx, lx, qx, fh, lh, 0, prm, gpb, gmb);
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const double fr = lane_right(gml[c]);
                din[c] = gpl[c] - (xhi ? gmb[c] : fr);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // y: the face below from row j - 1, or (j = 1) from the halo; the face above from
        // row j + 1, or (j = p) the boundary face with the halo
        {
            double fy[NV], ly, fh[NV], lh, qS[NQ], fS[NV], gpb_[NV], gmb_[NV], gpu[NV], gmu[NV];
            PDE::flux(q, a, 1, fy, ly, prm);
            const typename PDE::Cache ah = PDE::prepare(qy, prm);
            PDE::flux(qy, ah, 1, fh, lh, prm);
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                const double qs = lane_from(q[c], below);
                qS[c] = ylo ? qy[c] : qs;
            }
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const double fs = lane_from(fy[c], below);
                fS[c] = ylo ? fh[c] : fs;
            }
            const double ls = lane_from(ly, below);
            face_terms<PDE>(qS, fS, ylo ? lh : ls, q, fy, ly, 1, prm, gpb_, gmb_);   // the face below
            face_terms<PDE>(q, fy, ly, qy, fh, lh, 1, prm, gpu, gmu);                 // the boundary face above
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const double fa = lane_from(gmb_[c], above);
                dprev[c] = din[c] + (gpb_[c] - (yhi ? gmu[c] : fa));
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }

    if (lambda_out) {
        // segmented maximum over the lanes of each patch (LP a power of two, patches aligned)
        for (int o = LP / 2; o >= 1; o >>= 1) lmax = nanmax(lmax, __shfl_xor(lmax, o, 64));
        if (active && l == 0) lambda_out[ids ? ids[item] : item] = lmax;
    }
}

// p = 4 and 8 take the interior-mapped form, p = 6 (36 lanes: a wave would idle 28) the pair-mapped one.
template <int P>
constexpr bool kInteriorMapped = (P == 4 || P == 8);

template <int P>
constexpr int wave3d_ppw() {
    if constexpr (kInteriorMapped<P>) return Shape3i<P>::ppw;
    else return Shape3<P>::ppw;
}

template <int P>
constexpr int wave3d_ring_words() {
    if constexpr (kInteriorMapped<P>) return Shape3i<P>::ring_words;
    else return Shape3<P>::ring_words;
}

template <int P, int VEC, bool PERIODIC, bool MESH, bool WHOLE>
__global__ void __launch_bounds__(kBlock3)
update3d_fixed_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                      const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids, int32_t num_items,
                      int64_t stride, double r, const double *__restrict__ r_dev, double gamma,
                      double *__restrict__ lambda_out, MeshArgs mesh) {
    extern __shared__ double lds[];
    const double rr = r_dev ? *r_dev : r;
    if constexpr (kInteriorMapped<P>) {
        const int64_t item0 = (int64_t)blockIdx.x * Shape3i<P>::ppw;
        if (item0 >= num_items) return;
        wave_update3d_i<EulerPDE<5>, P, VEC, PERIODIC, MESH, WHOLE>(in, out, offsets, out_offsets, ids, item0,
                                                                    num_items, stride, rr, 0.0,
                                                                    typename EulerPDE<5>::Params{gamma}, lambda_out,
                                                                    lds, mesh);
    } else {
        const int64_t item0 = (int64_t)blockIdx.x * Shape3<P>::ppw;
        if (item0 >= num_items) return;
        wave_update3d<P, VEC, PERIODIC, MESH>(in, out, offsets, out_offsets, ids, item0, num_items, stride, rr, gamma,
                                              lambda_out, lds, mesh);
    }
}

template <int P, int VEC, bool PERIODIC, bool MESH = false, bool WHOLE = false>
hipError_t launch3d(const UpdateLaunch &L, hipStream_t stream) {
    constexpr int ppw = wave3d_ppw<P>();
    constexpr int words = wave3d_ring_words<P>();
    const int64_t blocks = ((int64_t)L.num_items + ppw - 1) / ppw;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(double) * (size_t)words;
    hipLaunchKernelGGL((update3d_fixed_kernel<P, VEC, PERIODIC, MESH, WHOLE>), dim3((unsigned)blocks), dim3(kBlock3), lds,
                       stream, L.in, L.out, L.offsets, L.out_offsets, L.ids, L.num_items, L.stride, L.r, L.r_dev,
                       L.gamma, L.lambda_out, L.mesh);
    return hipGetLastError();
}

template <int P>
hipError_t launch3d_p(const UpdateLaunch &L, hipStream_t stream) {
    const bool periodic = (L.flags & kPeriodic3) != 0;
    if (L.mesh.neighbors) {
        if (periodic) return hipErrorInvalidValue;
        return L.vec2 ? launch3d<P, 2, false, true>(L, stream) : launch3d<P, 1, false, true>(L, stream);
    }
    if constexpr (kInteriorMapped<P>) {
        // whole rows where the caller gave the output's halo volumes over
        if (!periodic && (L.flags & kHaloFromIn3))
            return L.vec2 ? launch3d<P, 2, false, false, true>(L, stream) : launch3d<P, 1, false, false, true>(L, stream);
    }
    if (L.vec2) return periodic ? launch3d<P, 2, true>(L, stream) : launch3d<P, 2, false>(L, stream);
    return periodic ? launch3d<P, 1, true>(L, stream) : launch3d<P, 1, false>(L, stream);
}

// The interior-mapped form for the other PDEs (fv_pde.h).
template <class PDE, int P, int VEC, bool PERIODIC>
__global__ void __launch_bounds__(kBlock3)
update3d_pde_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                    const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids, int32_t num_items,
                    int64_t stride, double r, double dt, typename PDE::Params prm, double *__restrict__ lambda_out) {
    extern __shared__ double lds[];
    const int64_t item0 = (int64_t)blockIdx.x * Shape3i<P, PDE::NQ>::ppw;
    if (item0 >= num_items) return;
    wave_update3d_i<PDE, P, VEC, PERIODIC>(in, out, offsets, out_offsets, ids, item0, num_items, stride, r, dt, prm,
                                           lambda_out, lds);
}

template <class PDE, int P, int VEC, bool PERIODIC>
void launch3d_pde_form(const UpdateLaunch &L, const typename PDE::Params &prm, int64_t blocks, size_t lds,
                       hipStream_t stream) {
    hipLaunchKernelGGL((update3d_pde_kernel<PDE, P, VEC, PERIODIC>), dim3((unsigned)blocks), dim3(kBlock3), lds,
                       stream, L.in, L.out, L.offsets, L.out_offsets, L.ids, L.num_items, L.stride, L.r, L.dt, prm,
                       L.lambda_out);
}

template <class PDE, int P>
hipError_t launch3d_pde(const UpdateLaunch &L, const typename PDE::Params &prm, hipStream_t stream) {
    using S = Shape3i<P, PDE::NQ>;
    const int64_t blocks = ((int64_t)L.num_items + S::ppw - 1) / S::ppw;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(double) * (size_t)S::ring_words;
    if ((L.flags & kPeriodic3) == 0) launch3d_pde_form<PDE, P, 1, false>(L, prm, blocks, lds, stream);
    else if (L.vec2) launch3d_pde_form<PDE, P, 2, true>(L, prm, blocks, lds, stream);
    else launch3d_pde_form<PDE, P, 1, true>(L, prm, blocks, lds, stream);
    return hipGetLastError();
}

template <class PDE>
hipError_t launch3d_pde_p(const UpdateLaunch &L, const typename PDE::Params &prm, hipStream_t stream) {
    return L.p == 4 ? launch3d_pde<PDE, 4>(L, prm, stream) : launch3d_pde<PDE, 8>(L, prm, stream);
}

}  // namespace

bool pde3d_fits(int pde, int dim, int p) {
    return dim == 3 && (p == 4 || p == 8) && (pde == kPdeAdvection || pde == kPdeAcoustics || pde == kPdeAcousticsNcp);
}

hipError_t launch_update3d_pde(const UpdateLaunch &L, hipStream_t stream) {
    if (!pde3d_fits(L.pde, L.dim, L.p) || L.r_dev) return hipErrorInvalidValue;
    const double *c = L.pde_prm;
    switch (L.pde) {
        case kPdeAdvection: return launch3d_pde_p<AdvectionPDE>(L, AdvectionPDE::Params{{c[0], c[1], c[2]}}, stream);
        case kPdeAcoustics: return launch3d_pde_p<AcousticsPDE<3, false>>(L, {c[0], c[1], c[2]}, stream);
        case kPdeAcousticsNcp: return launch3d_pde_p<AcousticsPDE<3, true>>(L, {c[0], c[1], c[2]}, stream);
    }
    return hipErrorInvalidValue;
}

bool wave3d_fixed(int p, int nq) { return nq == 5 && (p == 4 || p == 6 || p == 8); }

void wave3d_fixed_shape(int p, int *prefetch, int *rows) {
    *prefetch = 0;
    *rows = 0;
    if (!wave3d_fixed(p, 5)) return;
    *prefetch = Shape3<8>::PF;  // the same for every built size
    *rows = Shape3<8>::R;
}

hipError_t launch_update3d_fixed(const UpdateLaunch &L, hipStream_t stream) {
    if (L.nq != 5) return hipErrorInvalidValue;
    switch (L.p) {
        case 4: return launch3d_p<4>(L, stream);
        case 6: return launch3d_p<6>(L, stream);
        case 8: return launch3d_p<8>(L, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace fv
