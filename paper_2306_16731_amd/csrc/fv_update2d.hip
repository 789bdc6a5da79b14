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
//             complete row k-1: Q + (dt/h) (D_x + D_y) into an LDS ring of R
//               output rows per patch, fold l into the patch maximum
//             every R rows: flush the ring as contiguous 16- (or 8-) byte
//               chunks, R rows of a patch at a time
//
// Writing R consecutive rows of a patch in one burst keeps HBM write pages
// whole; storing each lane's 40-byte volume as it completes leaves every
// page to be reopened once per row and costs about a fifth of the write rate.
// The bursts are non-temporal stores: the output is not read again in this
// launch, and keeping it out of the L2 leaves that to the input rows.
// The waves of a block never synchronise with each other.  The per-patch
// maximum is a segmented tree reduction over the patch's lanes at the end.
//
// Two forms: the runtime-size kernel (any p + 2 <= 64, launch parameters
// from the tuning table) and the fixed-size kernel (compile-time p, see
// wave_update_fixed), which keeps its loads in flight across the bursts.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "fv_internal.h"
#include "fv_pde.h"
#include "fv_physics.h"

namespace fv {
namespace {

constexpr uint32_t kPeriodic = 0x2u;
constexpr uint32_t kHaloFromIn = 0x4u;  // the output's halo volumes may take the input's values
constexpr int kDefaultPrefetch2d = 4;
constexpr int kDefaultRows2d = 6;

// Cross-lane moves of a double through the DPP wave shifts.  They are issued
// in uniform control flow, so every source lane is enabled; the lane at the
// wave's edge (no source) reads zero, and no lane that receives it uses it.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const int2 v = __builtin_bit_cast(int2, x);
    const int lo = __builtin_amdgcn_mov_dpp(v.x, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(v.y, CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, make_int2(lo, hi));
}
__device__ __forceinline__ double from_left(double x) { return dpp_move<0x138>(x); }   // wave_shr:1
__device__ __forceinline__ double from_right(double x) { return dpp_move<0x130>(x); }  // wave_shl:1

// Exact quotient and remainder of small non-negative integers through a
// float reciprocal and one correction step.
__device__ __forceinline__ int small_div(int a, int b, float inv_b, int &rem) {
    int q = (int)((float)a * inv_b);
    int r = a - q * b;
    if (r < 0) { q -= 1; r += b; }
    else if (r >= b) { q += 1; r -= b; }
    rem = r;
    return q;
}

// Write rows [k0, k0 + nrows) of the wave's patches from the LDS ring: whole
// rows (the x-halo volumes hold their wrapped copies, or their input values),
// otherwise only the interior volumes of each row.
template <int NQ, int VEC>
__device__ __forceinline__ void flush_rows(double *__restrict__ out, const double *ring, const int64_t *bases,
                                           int ppw, int R, int W, int P, int k0, int nrows, bool whole_rows,
                                           int lane) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const int ROWD = W * NQ;
    const int64_t row = ROWD;
    if (whole_rows) {
        // rows are contiguous in HBM and in the ring: nrows * ROWD doubles per patch
        const int per = nrows * ROWD / VEC;
        const float inv = 1.0f / (float)per;
        for (int c = lane; c < ppw * per; c += 64) {
            int rem;
            const int sl = small_div(c, per, inv, rem);
            const int64_t base = bases[sl];
            if (base < 0) continue;
            if constexpr (VEC == 2) {
                const dv2 v = reinterpret_cast<const dv2 *>(ring + (size_t)sl * R * ROWD)[rem];
                __builtin_nontemporal_store(v, reinterpret_cast<dv2 *>(out + base + k0 * row) + rem);
            } else {
                __builtin_nontemporal_store(ring[(size_t)sl * R * ROWD + rem], out + base + k0 * row + rem);
            }
        }
    } else {
        const int inner = P * NQ;  // interior doubles of a row
        const int per = nrows * inner;
        const float inv = 1.0f / (float)per;
        const float inv_inner = 1.0f / (float)inner;
        for (int c = lane; c < ppw * per; c += 64) {
            int rem, d;
            const int sl = small_div(c, per, inv, rem);
            const int r = small_div(rem, inner, inv_inner, d);
            const int64_t base = bases[sl];
            if (base < 0) continue;
            __builtin_nontemporal_store(ring[((size_t)sl * R + r) * ROWD + NQ + d], out + base + (k0 + r) * row + NQ + d);
        }
    }
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// One wave advances patches item0 .. item0 + ppw - 1 (those below num_items)
// of size P.  Patch `item` starts at offsets[item] (or item * stride) in `in`
// and at out_offsets[item] (or the same offset) in `out`; its eigenvalue goes
// to lambda_out[ids[item]] (or [item]).  `ring` is the wave's
// LDS region: R output rows of each patch, then the patch bases.
template <int NQ, int PF, int VEC>
__device__ __forceinline__ void wave_update(const double *__restrict__ in, double *__restrict__ out,
                                            const int64_t *__restrict__ offsets,
                                            const int64_t *__restrict__ out_offsets,
                                            const int32_t *__restrict__ ids,
                                            int64_t item0, int64_t num_items, int P, int64_t stride, double r,
                                            double gamma, uint32_t flags, double *__restrict__ lambda_out, int R,
                                            double *ring) {
    const int W = P + 2;
    const int ppw = 64 / W;
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // lane-derived values stay inside the task (task-list kernel)
    const int slot = lane / W;
    const int i = lane - slot * W;
    const int64_t item = item0 + slot;
    const bool active = slot < ppw && item < num_items;
    const bool xin = i >= 1 && i <= P;
    const bool writer = active && xin;

    const int64_t off = active ? (offsets ? offsets[item] : item * stride) : 0;
    const int64_t off_out = active ? (out_offsets ? out_offsets[item] : off) : 0;
    const double *src = in + off + (int64_t)i * NQ;
    double *dst = out + off_out + (int64_t)i * NQ;
    const int64_t row = (int64_t)W * NQ;
    const bool periodic = (flags & kPeriodic) != 0;
    // the caller gave over the output's halo volumes: x-halo volumes of rows 1 .. p go out with
    // their input values, so each output row is written whole
    const bool whole = !periodic && (flags & kHaloFromIn) != 0;

    // LDS: the ring of R output rows of each of the wave's ppw patches, then their bases
    const int ring_words = ppw * R * W * NQ;
    int64_t *bases = reinterpret_cast<int64_t *>(ring + ring_words);
    wave_lds_fence();  // a previous patch group of this wave may still be reading the ring
    if (i == 0 && slot < ppw) bases[slot] = active ? off_out : -1;
    wave_lds_fence();
    int k0 = 1;  // first output row held in the ring

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
            double *srow = ring + ((size_t)slot * R + (kk - k0)) * row;
#pragma unroll
            for (int c = 0; c < NQ; ++c) srow[i * NQ + c] = qn[c];
            if (periodic) {
                // x-halo copies go into the ring row; y-halo rows are stored directly
                if (i == P)
#pragma unroll
                    for (int c = 0; c < NQ; ++c) srow[c] = qn[c];
                if (i == 1)
#pragma unroll
                    for (int c = 0; c < NQ; ++c) srow[(P + 1) * NQ + c] = qn[c];
                if (kk == P) store_volume<NQ>(dst, qn);
                if (kk == 1) store_volume<NQ>(dst + (int64_t)(P + 1) * row, qn);
            }
            if (lambda_out) lmax = nanmax(lmax, volume_lambda<2, NQ>(qn, gamma));
        }
        if (k >= 2 && whole && active && !xin) {
            double *srow = ring + ((size_t)slot * R + (k - 1 - k0)) * row;
#pragma unroll
            for (int c = 0; c < NQ; ++c) srow[i * NQ + c] = qprev[c];
        }
        if (k >= 2 && (k - k0 == R || k - 1 == P)) {
            wave_lds_fence();
            flush_rows<NQ, VEC>(out, ring, bases, ppw, R, W, P, k0, k - k0, periodic || whole, lane);
            wave_lds_fence();
            k0 = k;
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


// ---------------------------------------------------------------------------
// Fixed-size form.  The same step with the patch size a template parameter:
// the row loop unrolls completely and every loop has a static trip count.
// All global loads and stores are issued unconditionally -- lanes without a
// patch read the wave's first patch, rows past the patch re-read its last
// row, spare lanes of an output burst repeat a chunk another lane writes with
// the same value -- so the compiler can count the wave's outstanding memory
// operations exactly.  The PF rows in flight then stay in flight across the
// output bursts; in the runtime-size form the counts are unknown after any
// branch or loop with memory operations, and every row waits for all of them.
// Sizes: those of the benchmark batches (16) and the mixed-size batches
// (3, 5, 9, 17), Euler with five unknowns.

// Output rows per LDS burst.  Longer bursts write longer runs at once but take more LDS per wave and
// so leave fewer waves resident; the best depth depends on the launch:
//   Uniform       uniform launches writing whole rows (periodic, FV_HALO_FROM_IN), meshes, other PDEs;
//   Interior      uniform launches writing interior-only rows (their halo volumes stay untouched);
//   TaskWhole     the task-list launch of mixed sizes writing whole rows;
//   TaskInterior  the task-list launch writing interior-only rows.
// Every wave of a task-list launch reserves the ring of the batch's largest size class.  Measured on
// uniform batches of p = 16 and 17 and on the 200,000-patch mix of p = 3, 5, 9, 17 (caps 9 to 16
// tried): interior-only rows gain from long bursts, up to 14 rows in uniform launches (p = 16: 4%
// over 12, though five waves per CU stay resident instead of six) and 13 in the task-list launch,
// while whole rows in the task-list launch gain from short ones, up to 10 rows (6-7% over 12: seven
// waves per CU instead of five).  A patch of p rows up to the cap is written in one burst.
enum class RingUse { Uniform, Interior, TaskWhole, TaskInterior };

constexpr int burst_cap(RingUse u) {
    return u == RingUse::Interior ? 14 : u == RingUse::TaskWhole ? 10 : u == RingUse::TaskInterior ? 13 : 12;
}

template <int P, RingUse U = RingUse::Uniform>
struct FixedShape {
    static constexpr int PF = 2;                                   // rows in flight per lane
    static constexpr int R = P <= burst_cap(U) ? P : burst_cap(U);  // output rows per burst
};
constexpr int kFixedBlock = 64;                     // one wave per block: LDS, not registers, bounds residency
constexpr int kTaskBlock = 64;                      // the same for the task-list kernel

inline bool fixed_size(int p) { return p == 3 || p == 5 || p == 9 || p == 16 || p == 17; }

template <int P, RingUse U = RingUse::Uniform, int NQ = 5>
constexpr int fixed_ring_words() {
    return (64 / (P + 2)) * FixedShape<P, U>::R * (P + 2) * NQ + 64 / (P + 2);
}

// The ring use of a uniform launch of the fixed-size form, and of a body in the task-list launch.
template <bool PERIODIC, bool MESH, bool WHOLE>
constexpr RingUse uniform_use() {
    return (PERIODIC || MESH || WHOLE) ? RingUse::Uniform : RingUse::Interior;
}
template <bool PERIODIC, bool WHOLE>
constexpr RingUse task_use() {
    return (PERIODIC || WHOLE) ? RingUse::TaskWhole : RingUse::TaskInterior;
}

// MESH: the face halos come from the neighbouring patches' interiors (the
// halo volumes of a patch without a neighbour on that face are its own), and
// patch t advances by dt[t] / h[t]; the output is the interior only.
template <class PDE, int P, int VEC, bool PERIODIC, bool MESH = false, bool WHOLE = false,
          RingUse USE = RingUse::Uniform, int PFX = 0>
__device__ __forceinline__ void wave_update_fixed(const double *__restrict__ in, double *__restrict__ out,
                                                  const int64_t *__restrict__ offsets,
                                                  const int64_t *__restrict__ out_offsets,
                                                  const int32_t *__restrict__ ids, int64_t item0, int64_t num_items,
                                                  int64_t stride, double r, double dt,
                                                  const typename PDE::Params &prm,
                                                  double *__restrict__ lambda_out, double *ring,
                                                  MeshArgs mesh = MeshArgs{}) {
    static_assert(!(MESH && PERIODIC), "a mesh takes its halos from neighbours, not by self-wrap");
    // WHOLE (without PERIODIC): the x-halo volumes of rows 1 .. p are written with their input
    // values, so every output row is one contiguous run (partly written cache lines cost HBM time)
    static_assert(!(WHOLE && (PERIODIC || MESH)), "whole rows are the non-periodic, non-mesh form");
    constexpr bool kWholeRows = PERIODIC || WHOLE;
    constexpr int NQ = PDE::NQ, NV = PDE::NV;
    constexpr int W = P + 2;
    constexpr int ppw = 64 / W;
    constexpr int ROWD = W * NQ;
    constexpr int PF = PFX > 0 ? PFX : FixedShape<P, USE>::PF;  // PFX: the caller's prefetch depth
    constexpr int R = FixedShape<P, USE>::R;
    // VEC = 2: 16-byte burst stores.  Rows of an even number of doubles need every patch at an even
    // offset; rows of an odd number (odd p + 2 with N = 5) need only a 16-byte aligned output buffer:
    // each run of whole rows is written as the 16-byte pairs that start at its first even double,
    // plus its first and last double on their own.  The fixed sizes use that form for p = 17 only
    // (runs of 12 rows of 95 doubles): for the shorter runs of p = 3 and 5 the separate ends cost more
    // than the wider stores save, at p = 9 it is even, and interior-only runs stay in 8-byte chunks.
    typedef double dv2 __attribute__((ext_vector_type(2)));
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // lane-derived values stay inside the task (see the bursts below)
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
    // Row k is read at src_mid + k ROWD (k = 1 .. p), src_lo (k = 0) or src_hi
    // (k = p+1): the patch's own column, or in the mesh form the neighbour's
    // column (x halo lanes) / row (rows 0 and p+1).
    const double *src_mid = src, *src_lo = src, *src_hi = src + (int64_t)(W - 1) * ROWD;
    double ratio = r;  // dt / h of the lane's patch
    if constexpr (MESH) {
        const int32_t *nb = mesh.neighbors + 4 * self;
        const int32_t nl = nb[0], nr = nb[1], nd = nb[2], nu = nb[3];
        auto base = [&](int32_t q) { return in + (offsets ? offsets[q >= 0 ? q : self] : (q >= 0 ? q : self) * stride); };
        const double *bl = base(nl), *br = base(nr), *bd = base(nd), *bu = base(nu);
        src_mid = (i == 0 && nl >= 0) ? bl + P * NQ : ((i == P + 1 && nr >= 0) ? br + NQ : src);
        src_lo = (xin && nd >= 0) ? bd + (int64_t)P * ROWD + i * NQ : src;
        src_hi = (xin && nu >= 0) ? bu + (int64_t)ROWD + i * NQ : src_hi;
        ratio = mesh.dt[self] / mesh.h[self];
    }
    auto row_ptr = [&](int k) { return k == 0 ? src_lo : (k == W - 1 ? src_hi : src_mid + (int64_t)k * ROWD); };

    int64_t *bases = reinterpret_cast<int64_t *>(ring + ppw * R * ROWD);
    wave_lds_fence();  // a previous patch group of this wave may still be reading the ring
    if (i == 0 && slot < ppw) bases[slot] = off_out;
    wave_lds_fence();

    double qprev[NQ], fyprev[NV], fhprev[NV], dxprev[NV];
    double lyprev = 0.0, lmax = 0.0;
#pragma unroll
    for (int c = 0; c < NQ; ++c) qprev[c] = 1.0;  // a finite state; the face it forms is never used
#pragma unroll
    for (int c = 0; c < NV; ++c) fyprev[c] = fhprev[c] = dxprev[c] = 0.0;

    double qbuf[PF][NQ];
#pragma unroll
    for (int m = 0; m < PF; ++m) load_volume<NQ>(row_ptr(m < W ? m : W - 1), qbuf[m]);

#pragma unroll
    for (int k = 0; k < W; ++k) {
        double q[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) q[c] = qbuf[k % PF][c];
        load_volume<NQ>(row_ptr(k + PF < W ? k + PF : W - 1), qbuf[k % PF]);

        // the faces of the row: x to the lane's left (G+ for this lane, G- for the lane to the left)
        // and y below (G+ for this row, G- for the row below); G+ = G- = Fhat without a
        // non-conservative product
        const typename PDE::Cache a = PDE::prepare(q, prm);
        double fx[NV], lx, fy[NV], ly;
        PDE::flux(q, a, 0, fx, lx, prm);
        PDE::flux(q, a, 1, fy, ly, prm);
        double qL[NQ], fL[NV], gpx[NV], gmx[NV];
#pragma unroll
        for (int c = 0; c < NQ; ++c) qL[c] = from_left(q[c]);
#pragma unroll
        for (int c = 0; c < NV; ++c) fL[c] = from_left(fx[c]);
        const double lL = from_left(lx);
        face_terms<PDE>(qL, fL, lL, q, fx, lx, 0, prm, gpx, gmx);
        double dx[NV], fh[NV], gmy[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) dx[c] = gpx[c] - from_right(gmx[c]);
        face_terms<PDE>(qprev, fyprev, lyprev, q, fy, ly, 1, prm, fh, gmy);

        if (k >= 2) {
            const int kk = k - 1;          // output row completed at this layer
            const int rr = (kk - 1) % R;   // its row in the ring
            if (writer) {
                double d[NV], qn[NQ];
#pragma unroll
                for (int c = 0; c < NV; ++c) d[c] = dxprev[c] + (fhprev[c] - gmy[c]);
                advance_pde<PDE>(qprev, d, ratio, dt, prm, qn);
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
            if constexpr (WHOLE) {
                if (active && !xin) {
                    double *hrow = ring + (slot * R + rr) * ROWD;
#pragma unroll
                    for (int c = 0; c < NQ; ++c) hrow[i * NQ + c] = qprev[c];
                }
            }
            if (rr == R - 1 || kk == P) {
                const int nrows = rr + 1;
                const int k0 = kk - rr;    // first output row in the ring
                // The burst's per-lane indices are formed here from a lane id
                // the optimiser cannot see through: otherwise it computes the
                // indices of every burst up front and keeps them in registers
                // across all layers (and, in the task-list kernel, across all
                // tasks).
                int ln = lane;
                asm volatile("" : "+v"(ln));
                wave_lds_fence();
                if constexpr (kWholeRows && VEC == 2 && ROWD % 2 == 1) {
                    // whole rows of an odd number of doubles: per slot one run of len doubles at a
                    // parity of its own; pair m starts at double par + 2 m of the run (the pairs a slot
                    // has fewer of repeat its last one), then the run's first and last double
                    const int len = nrows * ROWD;
                    const int per = len / 2;
                    const int total = ppw * per;
#pragma unroll
                    for (int j = 0; j < (total + 63) / 64; ++j) {
                        const int c = ln + 64 * j < total ? ln + 64 * j : total - 1;
                        int sl = c / per;
                        int m = c - sl * per;
                        sl = item0 + sl < num_items ? sl : 0;
                        const int64_t base = bases[sl] + (int64_t)k0 * ROWD;
                        const int par = (int)(base & 1);
                        m = m < (len - par) / 2 ? m : (len - par) / 2 - 1;
                        const double *src = ring + sl * R * ROWD + par + 2 * m;
                        dv2 v;
                        v.x = src[0];
                        v.y = src[1];
                        __builtin_nontemporal_store(v, reinterpret_cast<dv2 *>(out + base + par) + m);
                    }
                    constexpr int ends = 2 * ppw;
#pragma unroll
                    for (int j = 0; j < (ends + 63) / 64; ++j) {
                        const int c = ln + 64 * j < ends ? ln + 64 * j : ends - 1;
                        int sl = c >> 1;
                        const int e = (c & 1) ? len - 1 : 0;
                        sl = item0 + sl < num_items ? sl : 0;
                        __builtin_nontemporal_store(ring[sl * R * ROWD + e], out + bases[sl] + (int64_t)k0 * ROWD + e);
                    }
                    // y-halo rows: row P+1 takes row 1, row 0 takes row P (interior columns)
                    if (PERIODIC && (k0 == 1 || kk == P)) {
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            if (h == 0 ? k0 != 1 : kk != P) continue;
                            const int from = h == 0 ? 0 : rr;
                            const int dest = h == 0 ? P + 1 : 0;
                            constexpr int iper = P * NQ;
                            constexpr int itotal = ppw * iper;
#pragma unroll
                            for (int jj = 0; jj < (itotal + 63) / 64; ++jj) {
                                const int c = ln + 64 * jj < itotal ? ln + 64 * jj : itotal - 1;
                                int sl = c / iper;
                                const int d = c - sl * iper;
                                sl = item0 + sl < num_items ? sl : 0;
                                __builtin_nontemporal_store(ring[(sl * R + from) * ROWD + NQ + d],
                                                            out + bases[sl] + (int64_t)dest * ROWD + NQ + d);
                            }
                        }
                    }
                } else if (kWholeRows) {
                    // whole rows (x-halo volumes hold their wrapped copies, or their input values)
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
                    if (PERIODIC && (k0 == 1 || kk == P)) {
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
                wave_lds_fence();
            }
        }
#pragma unroll
        for (int c = 0; c < NQ; ++c) qprev[c] = q[c];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            fyprev[c] = fy[c];
            fhprev[c] = fh[c];
            dxprev[c] = dx[c];
        }
        lyprev = ly;
        // keep the layers apart: interleaving them buys no latency (the loads
        // already run PF layers ahead) and costs registers, hence occupancy
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

// Rows in flight of a fixed-size body in a task-list launch with one wave per task: deeper than in
// the uniform launches (config 3's mix: 6 rows for interior-only rows, 3% faster than 2; 4 for whole
// rows, 1%).  A persistent grid, whose waves run many tasks each, was 3% slower with them, so its
// bodies keep the uniform depth.
constexpr int task_prefetch(RingUse u) { return u == RingUse::TaskInterior ? 6 : 4; }

// One task of the fixed-size form; DEEP: the launch runs one wave per task.
template <int P, int VEC, bool PERIODIC, bool WHOLE, bool DEEP>
__device__ __forceinline__ void fixed_task_body(const double *__restrict__ in, double *__restrict__ out,
                                             const int64_t *__restrict__ offsets,
                                             const int64_t *__restrict__ out_offsets,
                                             const int32_t *__restrict__ ids, int64_t count, double r, double gamma,
                                             double *__restrict__ lambda_out, double *ring) {
    constexpr RingUse U = task_use<PERIODIC, WHOLE>();
    wave_update_fixed<EulerPDE<5>, P, VEC, PERIODIC, false, WHOLE, U, DEEP ? task_prefetch(U) : 0>(
        in, out, offsets, out_offsets, ids, 0, count, 0, r, 0.0, typename EulerPDE<5>::Params{gamma}, lambda_out, ring);
}

// Task-list body for a fixed size: false when p has no fixed-size build.
template <int NQ, int VEC, bool PERIODIC, bool WHOLE, bool DEEP>
__device__ __forceinline__ bool fixed_task_depth(int p, const double *__restrict__ in, double *__restrict__ out,
                                                 const int64_t *__restrict__ offsets,
                                                 const int64_t *__restrict__ out_offsets,
                                                 const int32_t *__restrict__ ids, int64_t count, double r,
                                                 double gamma, double *__restrict__ lambda_out, double *ring) {
    switch (p) {
        case 3: fixed_task_body<3, 1, PERIODIC, WHOLE, DEEP>(in, out, offsets, out_offsets, ids, count, r, gamma, lambda_out, ring); return true;
        case 5: fixed_task_body<5, 1, PERIODIC, WHOLE, DEEP>(in, out, offsets, out_offsets, ids, count, r, gamma, lambda_out, ring); return true;
        case 9: fixed_task_body<9, 1, PERIODIC, WHOLE, DEEP>(in, out, offsets, out_offsets, ids, count, r, gamma, lambda_out, ring); return true;
        case 16: fixed_task_body<16, VEC, PERIODIC, WHOLE, DEEP>(in, out, offsets, out_offsets, ids, count, r, gamma, lambda_out, ring); return true;
        case 17: fixed_task_body<17, VEC, PERIODIC, WHOLE, DEEP>(in, out, offsets, out_offsets, ids, count, r, gamma, lambda_out, ring); return true;
    }
    return false;
}

// deep: the launch runs one wave per task (uniform across the launch).
template <int NQ, int VEC, bool PERIODIC, bool WHOLE>
__device__ __forceinline__ bool fixed_task(int p, bool deep, const double *__restrict__ in, double *__restrict__ out,
                                           const int64_t *__restrict__ offsets,
                                           const int64_t *__restrict__ out_offsets,
                                           const int32_t *__restrict__ ids, int64_t count, double r, double gamma,
                                           double *__restrict__ lambda_out, double *ring) {
    if constexpr (NQ != 5) {
        return false;
    } else {
        return deep ? fixed_task_depth<NQ, VEC, PERIODIC, WHOLE, true>(p, in, out, offsets, out_offsets, ids, count, r,
                                                                       gamma, lambda_out, ring)
                    : fixed_task_depth<NQ, VEC, PERIODIC, WHOLE, false>(p, in, out, offsets, out_offsets, ids, count,
                                                                        r, gamma, lambda_out, ring);
    }
}


// Uniform launch: every wave takes the next ppw patches of one size.
template <int NQ, int PF, int VEC>
__global__ void __launch_bounds__(256)
update2d_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids, int32_t num_items,
                int32_t P, int64_t stride, double r,
                const double *__restrict__ r_dev, double gamma, uint32_t flags, double *__restrict__ lambda_out,
                int32_t R) {
    extern __shared__ double lds[];
    const int wave = threadIdx.x >> 6;
    const int ppw = 64 / (P + 2);
    const int64_t item0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * ppw;
    const double rr = r_dev ? *r_dev : r;
    wave_update<NQ, PF, VEC>(in, out, offsets, out_offsets, ids, item0, num_items, P, stride, rr, gamma, flags,
                             lambda_out, R,
                             lds + (size_t)wave * (ppw * R * (P + 2) * NQ + ppw));
}

// Uniform launch of the fixed-size form.
template <int P, int VEC, bool PERIODIC, bool MESH, bool WHOLE>
__global__ void __launch_bounds__(kFixedBlock)
update2d_fixed_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                      const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids, int32_t num_items,
                      int64_t stride, double r, const double *__restrict__ r_dev, double gamma,
                      double *__restrict__ lambda_out, MeshArgs mesh) {
    extern __shared__ double lds[];
    constexpr int ppw = 64 / (P + 2);
    const int wave = threadIdx.x >> 6;
    const int64_t item0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * ppw;
    if (item0 >= num_items) return;
    const double rr = r_dev ? *r_dev : r;
    constexpr RingUse U = uniform_use<PERIODIC, MESH, WHOLE>();
    wave_update_fixed<EulerPDE<5>, P, VEC, PERIODIC, MESH, WHOLE, U>(
        in, out, offsets, out_offsets, ids, item0, num_items, stride, rr, 0.0, typename EulerPDE<5>::Params{gamma},
        lambda_out, lds + (size_t)wave * fixed_ring_words<P, U>(), mesh);
}

// The wave form for the other PDEs of Eq. 1 (fv_pde.h) at the fixed sizes: the
// same march as the Euler instance above on the PDE's user terms.
template <class PDE, int P, int VEC, bool PERIODIC>
__global__ void __launch_bounds__(kFixedBlock)
update2d_pde_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                    const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids, int32_t num_items,
                    int64_t stride, double r, double dt, typename PDE::Params prm, double *__restrict__ lambda_out) {
    extern __shared__ double lds[];
    constexpr int ppw = 64 / (P + 2);
    const int64_t item0 = (int64_t)blockIdx.x * ppw;
    if (item0 >= num_items) return;
    wave_update_fixed<PDE, P, VEC, PERIODIC>(in, out, offsets, out_offsets, ids, item0, num_items, stride, r, dt, prm,
                                             lambda_out, lds);
}

// Task-list launch over mixed patch sizes: task t holds `count` patches of
// size `p` at offsets[first ..] (ids[first ..]); rows == 0 selects the
// fixed-size form.  Each wave takes tasks gw, gw + nw, ... (nw = waves in
// the grid), so a grid smaller than the task list is persistent; tasks sorted
// largest first balance the tail.
template <int NQ, int PF, int VEC, bool PERIODIC, bool WHOLE>
__global__ void __launch_bounds__(kTaskBlock)
update2d_tasks_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets,
                      const int64_t *__restrict__ out_offsets, const int32_t *__restrict__ ids,
                      const WaveTask *__restrict__ tasks, int32_t num_tasks,
                      double r, const double *__restrict__ r_dev, double gamma,
                      double *__restrict__ lambda_out, int32_t ring_words) {
    extern __shared__ double lds[];
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * waves + wave;
    const int64_t nw = (int64_t)gridDim.x * waves;
    const double rr = r_dev ? *r_dev : r;
    double *ring = lds + (size_t)wave * ring_words;
    const bool one_per_task = nw >= num_tasks;
    for (int64_t t = gw; t < num_tasks; t += nw) {
        const WaveTask tk = tasks[t];
        const int64_t *to = out_offsets ? out_offsets + tk.first : nullptr;
        if (tk.rows == 0 && fixed_task<NQ, VEC, PERIODIC, WHOLE>(tk.p, one_per_task, in, out, offsets + tk.first, to,
                                                                 ids + tk.first, tk.count, rr, gamma, lambda_out,
                                                                 ring))
            continue;
        wave_update<NQ, PF, VEC>(in, out, offsets + tk.first, to, ids + tk.first, 0, tk.count, tk.p, 0, rr, gamma,
                                 (PERIODIC ? kPeriodic : 0u) | (WHOLE ? kHaloFromIn : 0u), lambda_out,
                                 tk.rows > 0 ? tk.rows : kDefaultRows2d,
                                 ring);
    }
}

size_t wave2d_lds_bytes_(int p, int nq, int block, int R) {
    const int W = p + 2, ppw = 64 / W;
    return sizeof(double) * (size_t)(block / 64) * (size_t)(ppw * R * W * nq + ppw);
}

template <int NQ, int PF, int VEC>
hipError_t launch2d(const UpdateLaunch &L, hipStream_t stream) {
    const int W = L.p + 2;
    const int ppw = 64 / W;
    const int B = L.block > 0 ? L.block : 256;
    const int R = L.rows > 0 ? L.rows : kDefaultRows2d;
    if (B % 64 != 0 || B > 256 || ppw < 1 || R < 1 || R > 16) return hipErrorInvalidConfiguration;
    const int per_block = (B / 64) * ppw;
    const int64_t blocks = ((int64_t)L.num_items + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = wave2d_lds_bytes_(L.p, NQ, B, R);
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return hipErrorInvalidDevice;
    if (lds > (size_t)lds_max) return hipErrorInvalidConfiguration;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&update2d_kernel<NQ, PF, VEC>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((update2d_kernel<NQ, PF, VEC>), dim3((unsigned)blocks), dim3(B), lds, stream, L.in, L.out,
                       L.offsets, L.out_offsets, L.ids, L.num_items, L.p, L.stride, L.r, L.r_dev, L.gamma, L.flags,
                       L.lambda_out, R);
    return hipGetLastError();
}

template <int NQ, int PF, int VEC, bool PERIODIC, bool WHOLE>
hipError_t launch2d_tasks(const TaskLaunch &T, hipStream_t stream) {
    const int B = kTaskBlock;
    const size_t lds = sizeof(double) * (size_t)(B / 64) * (size_t)T.ring_words;
    int dev = 0, lds_max = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return hipErrorInvalidDevice;
    if (lds > (size_t)lds_max) return hipErrorInvalidConfiguration;
    const void *fn = reinterpret_cast<const void *>(&update2d_tasks_kernel<NQ, PF, VEC, PERIODIC, WHOLE>);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int64_t blocks = ((int64_t)T.num_tasks + B / 64 - 1) / (B / 64);
    if (T.persistent) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, B, lds) != hipSuccess || per_cu < 1) per_cu = 1;
        blocks = std::min<int64_t>(blocks, (int64_t)per_cu * cus);
    }
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL((update2d_tasks_kernel<NQ, PF, VEC, PERIODIC, WHOLE>), dim3((unsigned)blocks), dim3(B), lds, stream,
                       T.in, T.out, T.offsets, T.out_offsets, T.ids, T.tasks, T.num_tasks, T.r, T.r_dev, T.gamma,
                       T.lambda_out, T.ring_words);
    return hipGetLastError();
}

}  // namespace

bool wave2d_fits(int p) { return p + 2 <= 64; }

template <int NQ, int VEC>
hipError_t launch2d_pf(const UpdateLaunch &L, hipStream_t stream) {
    switch (L.prefetch > 0 ? L.prefetch : kDefaultPrefetch2d) {
        case 1: return launch2d<NQ, 1, VEC>(L, stream);
        case 2: return launch2d<NQ, 2, VEC>(L, stream);
        case 3: return launch2d<NQ, 3, VEC>(L, stream);
        case 4: return launch2d<NQ, 4, VEC>(L, stream);
    }
    return hipErrorInvalidValue;
}

size_t wave2d_lds_bytes(int p, int nq, int block, int rows) { return wave2d_lds_bytes_(p, nq, block, rows); }

int wave2d_ring_words(int p, int nq, int rows) {
    const int W = p + 2, ppw = 64 / W;
    return ppw * rows * W * nq + ppw;
}

template <int NQ, int VEC, bool PERIODIC, bool WHOLE>
static hipError_t tasks_pf(const TaskLaunch &T, hipStream_t stream) {
    switch (T.prefetch > 0 ? T.prefetch : kDefaultPrefetch2d) {
        case 1: return launch2d_tasks<NQ, 1, VEC, PERIODIC, WHOLE>(T, stream);
        case 2: return launch2d_tasks<NQ, 2, VEC, PERIODIC, WHOLE>(T, stream);
        case 3: return launch2d_tasks<NQ, 3, VEC, PERIODIC, WHOLE>(T, stream);
        case 4: return launch2d_tasks<NQ, 4, VEC, PERIODIC, WHOLE>(T, stream);
    }
    return hipErrorInvalidValue;
}

template <int NQ, int VEC>
static hipError_t tasks_periodic(const TaskLaunch &T, hipStream_t stream) {
    if (T.flags & kPeriodic) return tasks_pf<NQ, VEC, true, false>(T, stream);
    // whole output rows for the fixed-size bodies (N = 5) where the caller allows it
    if constexpr (NQ == 5)
        if (T.flags & kHaloFromIn) return tasks_pf<NQ, VEC, false, true>(T, stream);
    return tasks_pf<NQ, VEC, false, false>(T, stream);
}

hipError_t launch_update2d_tasks(const TaskLaunch &T, hipStream_t stream) {
    if (T.num_tasks <= 0) return hipSuccess;
    if (T.nq == 5) return T.vec2 ? tasks_periodic<5, 2>(T, stream) : tasks_periodic<5, 1>(T, stream);
    if (T.nq == 4) return T.vec2 ? tasks_periodic<4, 2>(T, stream) : tasks_periodic<4, 1>(T, stream);
    return hipErrorInvalidValue;
}

// Uniform launch of the fixed-size form over patches of one size.
template <int P, int VEC, bool PERIODIC, bool MESH = false, bool WHOLE = false>
static hipError_t launch_fixed(const UpdateLaunch &L, hipStream_t stream) {
    constexpr int ppw = 64 / (P + 2);
    const int B = kFixedBlock;
    const int per_block = (B / 64) * ppw;
    const int64_t blocks = ((int64_t)L.num_items + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(double) * (size_t)(B / 64) * (size_t)fixed_ring_words<P, uniform_use<PERIODIC, MESH, WHOLE>()>();
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return hipErrorInvalidDevice;
    if (lds > (size_t)lds_max) return hipErrorInvalidConfiguration;
    const void *fn = reinterpret_cast<const void *>(&update2d_fixed_kernel<P, VEC, PERIODIC, MESH, WHOLE>);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((update2d_fixed_kernel<P, VEC, PERIODIC, MESH, WHOLE>), dim3((unsigned)blocks), dim3(B), lds, stream,
                       L.in, L.out, L.offsets, L.out_offsets, L.ids, L.num_items, L.stride, L.r, L.r_dev, L.gamma,
                       L.lambda_out, L.mesh);
    return hipGetLastError();
}

template <int P, int VEC>
static hipError_t fixed_periodic(const UpdateLaunch &L, hipStream_t stream) {
    if (L.mesh.neighbors) return (L.flags & kPeriodic) ? hipErrorInvalidValue : launch_fixed<P, VEC, false, true>(L, stream);
    if (L.flags & kPeriodic) return launch_fixed<P, VEC, true>(L, stream);
    if (L.flags & kHaloFromIn) return launch_fixed<P, VEC, false, false, true>(L, stream);
    return launch_fixed<P, VEC, false>(L, stream);
}

bool wave2d_fixed(int p, int nq) { return nq == 5 && fixed_size(p); }

void wave2d_fixed_shape(int p, int *prefetch, int *rows) {
    switch (p) {
        case 3: *prefetch = FixedShape<3>::PF; *rows = FixedShape<3>::R; return;
        case 5: *prefetch = FixedShape<5>::PF; *rows = FixedShape<5>::R; return;
        case 9: *prefetch = FixedShape<9>::PF; *rows = FixedShape<9>::R; return;
        case 16: *prefetch = FixedShape<16>::PF; *rows = FixedShape<16>::R; return;
        case 17: *prefetch = FixedShape<17>::PF; *rows = FixedShape<17>::R; return;
    }
    *prefetch = 0;
    *rows = 0;
}

int wave2d_fixed_block() { return kFixedBlock; }

template <RingUse U>
static int task_ring_words(int p) {
    switch (p) {
        case 3: return fixed_ring_words<3, U>();
        case 5: return fixed_ring_words<5, U>();
        case 9: return fixed_ring_words<9, U>();
        case 16: return fixed_ring_words<16, U>();
        case 17: return fixed_ring_words<17, U>();
    }
    return 0;
}

int wave2d_fixed_ring_words(int p, bool whole_rows) {
    return whole_rows ? task_ring_words<RingUse::TaskWhole>(p) : task_ring_words<RingUse::TaskInterior>(p);
}

hipError_t launch_update2d_fixed(const UpdateLaunch &L, hipStream_t stream) {
    if (L.nq != 5) return hipErrorInvalidValue;
    switch (L.p) {
        case 3: return fixed_periodic<3, 1>(L, stream);
        case 5: return fixed_periodic<5, 1>(L, stream);
        case 9: return fixed_periodic<9, 1>(L, stream);
        case 16: return L.vec2 ? fixed_periodic<16, 2>(L, stream) : fixed_periodic<16, 1>(L, stream);
        case 17: return L.vec2 ? fixed_periodic<17, 2>(L, stream) : fixed_periodic<17, 1>(L, stream);
    }
    return hipErrorInvalidValue;
}

namespace {

template <class PDE, int P, int VEC, bool PERIODIC>
void launch_pde_wave_form(const UpdateLaunch &L, const typename PDE::Params &prm, int64_t blocks, size_t lds,
                          hipStream_t stream) {
    hipLaunchKernelGGL((update2d_pde_kernel<PDE, P, VEC, PERIODIC>), dim3((unsigned)blocks), dim3(kFixedBlock), lds,
                       stream, L.in, L.out, L.offsets, L.out_offsets, L.ids, L.num_items, L.stride, L.r, L.dt, prm,
                       L.lambda_out);
}

template <class PDE, int P>
hipError_t launch_pde_wave(const UpdateLaunch &L, const typename PDE::Params &prm, hipStream_t stream) {
    constexpr int ppw = 64 / (P + 2);
    const int64_t blocks = ((int64_t)L.num_items + ppw - 1) / ppw;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(double) * (size_t)fixed_ring_words<P, RingUse::Uniform, PDE::NQ>();
    // 16-byte row bursts where the rows are an even number of doubles (p = 16)
    if ((L.flags & kPeriodic) == 0) launch_pde_wave_form<PDE, P, 1, false>(L, prm, blocks, lds, stream);
    else if (P == 16 && L.vec2) launch_pde_wave_form<PDE, P, P == 16 ? 2 : 1, true>(L, prm, blocks, lds, stream);
    else launch_pde_wave_form<PDE, P, 1, true>(L, prm, blocks, lds, stream);
    return hipGetLastError();
}

template <class PDE>
hipError_t launch_pde_wave_p(const UpdateLaunch &L, const typename PDE::Params &prm, hipStream_t stream) {
    switch (L.p) {
        case 3: return launch_pde_wave<PDE, 3>(L, prm, stream);
        case 5: return launch_pde_wave<PDE, 5>(L, prm, stream);
        case 9: return launch_pde_wave<PDE, 9>(L, prm, stream);
        case 16: return launch_pde_wave<PDE, 16>(L, prm, stream);
        case 17: return launch_pde_wave<PDE, 17>(L, prm, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool pde_wave_fits(int pde, int dim, int p) {
    return dim == 2 && fixed_size(p) &&
           (pde == kPdeShallowWater || pde == kPdeAdvection || pde == kPdeAcoustics || pde == kPdeAcousticsNcp);
}

hipError_t launch_update2d_pde(const UpdateLaunch &L, hipStream_t stream) {
    if (!pde_wave_fits(L.pde, L.dim, L.p) || L.r_dev) return hipErrorInvalidValue;
    const double *c = L.pde_prm;
    switch (L.pde) {
        case kPdeShallowWater: return launch_pde_wave_p<ShallowWaterPDE>(L, {c[0], c[1]}, stream);
        case kPdeAdvection: return launch_pde_wave_p<AdvectionPDE>(L, AdvectionPDE::Params{{c[0], c[1], c[2]}}, stream);
        case kPdeAcoustics: return launch_pde_wave_p<AcousticsPDE<2, false>>(L, {c[0], c[1], c[2]}, stream);
        case kPdeAcousticsNcp: return launch_pde_wave_p<AcousticsPDE<2, true>>(L, {c[0], c[1], c[2]}, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_update2d(const UpdateLaunch &L, hipStream_t stream) {
    // 16-byte flush chunks need 16-byte aligned patches and an even row length
    const bool v2 = L.vec2 && ((L.p + 2) * L.nq) % 2 == 0;
    if (L.nq == 5) return v2 ? launch2d_pf<5, 2>(L, stream) : launch2d_pf<5, 1>(L, stream);
    if (L.nq == 4) return v2 ? launch2d_pf<4, 2>(L, stream) : launch2d_pf<4, 1>(L, stream);
    return hipErrorInvalidValue;
}

}  // namespace fv
