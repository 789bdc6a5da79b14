// fv_flavours.hip -- the paper's three kernel realisations (Sec. 3) as MI355X
// comparison variants of the fused update.
//
// They compute the same step as the fused kernels, with the same microkernels
// (fv_physics.h) in the same order per volume, so their results agree with
// the fused kernels bit for bit; they differ in how the steps of Alg. 1 are
// mapped onto launches:
//
//   batched     one launch per algorithmic step over all volumes of all
//               patches, with HBM temporaries between the steps: user terms
//               F_n, l_n of every volume; face fluxes; the update; the
//               per-patch eigenvalue reduction (Sec. 3, "batched").
//   patch-wise  one work-group per patch; the steps run one after another
//               inside it with a barrier between them (x faces, y faces, z
//               faces, update, reduction), patch state and face fluxes in LDS,
//               threads masked to the patch's volumes (Sec. 3, "patch-wise").
//   task graph  a task per (patch, microkernel type): the d face-flux tasks
//               of a patch are independent, its update task depends on them
//               (Sec. 3, "task graph"); the tasks are submitted from the host
//               every call, as the paper's realisation submits its tasks every
//               time step: flux tasks on one library stream per axis, the
//               update on the caller's stream after events from its flux
//               tasks.
//
// All three take batches of one patch size and five unknowns.  The batched
// and task-graph forms keep their temporaries in a grow-only device workspace
// owned by the library (one per device, kept until the process ends).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "fv_host.h"
#include "fv_internal.h"
#include "fv_physics.h"

namespace fv {
namespace {

constexpr int NQ = 5;
constexpr uint32_t kPeriodicF = 0x2u;

struct Geo {
    int p, W, V;         // interior size, padded size, padded volumes
    int NF;              // faces per axis: (p+1) p^(d-1)
};

__host__ __device__ inline Geo geo(int p, int D) {
    Geo g;
    g.p = p;
    g.W = p + 2;
    g.V = D == 2 ? g.W * g.W : g.W * g.W * g.W;
    g.NF = D == 2 ? (p + 1) * p : (p + 1) * p * p;
    return g;
}

// padded index of (i, j, k)
__device__ inline int vidx(const Geo &g, int i, int j, int k) { return (k * g.W + j) * g.W + i; }

// face f of axis n -> the left volume (i, j, k); the right one is one step along n.
// The face index runs over m = 0..p along n (the face between m and m+1) and
// 1..p along the other axes, the first other axis fastest.
template <int D>
__device__ inline void face_left(const Geo &g, int n, int f, int &i, int &j, int &k) {
    const int m = f % (g.p + 1);
    const int o = f / (g.p + 1);
    const int a = 1 + o % g.p, b = D == 3 ? 1 + o / g.p : 0;
    if (n == 0) { i = m; j = a; k = b; }
    else if (n == 1) { i = a; j = m; k = b; }
    else { i = a; j = b; k = m; }
}

// face index of the face on the low side of volume (i, j, k) along n (c_n - 1/2)
template <int D>
__device__ inline int face_of(const Geo &g, int n, int i, int j, int k) {
    int m, a, b;
    if (n == 0) { m = i - 1; a = j; b = k; }
    else if (n == 1) { m = j - 1; a = i; b = k; }
    else { m = k - 1; a = i; b = j; }
    const int o = (a - 1) + (D == 3 ? (b - 1) * g.p : 0);
    return o * (g.p + 1) + m;
}

template <int D>
__device__ inline void interior_coords(const Geo &g, int c, int &i, int &j, int &k) {
    i = 1 + c % g.p;
    j = 1 + (c / g.p) % g.p;
    k = D == 3 ? 1 + c / (g.p * g.p) : 0;
}

__device__ inline void load_q(const double *src, double (&q)[NQ]) {
#pragma unroll
    for (int c = 0; c < NQ; ++c) q[c] = src[c];
}

// the update of one interior volume from its face fluxes (difference first,
// axes in order), plus the periodic face-halo copies
template <int D>
__device__ inline void finish_volume(const Geo &g, const double (&q)[NQ], const double (&dsum)[NQ], double r,
                                     double *patch_out, int i, int j, int k, bool periodic, double (&qn)[NQ]) {
    advance<NQ>(q, dsum, r, qn);
    store_volume<NQ>(patch_out + (int64_t)vidx(g, i, j, k) * NQ, qn);
    if (periodic) {
        const int p = g.p;
        if (i == p) store_volume<NQ>(patch_out + (int64_t)vidx(g, 0, j, k) * NQ, qn);
        if (i == 1) store_volume<NQ>(patch_out + (int64_t)vidx(g, p + 1, j, k) * NQ, qn);
        if (j == p) store_volume<NQ>(patch_out + (int64_t)vidx(g, i, 0, k) * NQ, qn);
        if (j == 1) store_volume<NQ>(patch_out + (int64_t)vidx(g, i, p + 1, k) * NQ, qn);
        if (D == 3) {
            if (k == p) store_volume<NQ>(patch_out + (int64_t)vidx(g, i, j, 0) * NQ, qn);
            if (k == 1) store_volume<NQ>(patch_out + (int64_t)vidx(g, i, j, p + 1) * NQ, qn);
        }
    }
}

__device__ inline int64_t patch_off(const int64_t *offsets, int64_t stride, int64_t t) {
    return offsets ? offsets[t] : t * stride;
}

// ------------------------------------------------------------------ batched
// step 1: user terms of every volume the faces of axis n need
template <int D>
__global__ void __launch_bounds__(256)
bt_terms(const double *__restrict__ in, const int64_t *__restrict__ offsets, int64_t stride, int32_t T, int p,
         double gamma, double *__restrict__ tf, double *__restrict__ tl) {
    const Geo g = geo(p, D);
    const int64_t total = (int64_t)T * D * g.V;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / ((int64_t)D * g.V);
        const int rem = (int)(e - t * D * g.V);
        const int n = rem / g.V, v = rem - n * g.V;
        const int i = v % g.W, j = (v / g.W) % g.W, k = D == 3 ? v / (g.W * g.W) : 0;
        const int c[3] = {i, j, k};
        bool need = true;  // coordinate n anywhere, the others interior
        for (int a = 0; a < D; ++a)
            if (a != n && (c[a] < 1 || c[a] > p)) need = false;
        if (!need) continue;
        double q[NQ], f[NQ], l;
        load_q(in + patch_off(offsets, stride, t) + (int64_t)v * NQ, q);
        const Prim pr = primitives<NQ>(q, gamma);
        euler_flux<NQ>(q, pr, n, f, l);
        const int64_t base = (t * D + n) * g.V + v;
#pragma unroll
        for (int cc = 0; cc < NQ; ++cc) tf[base * NQ + cc] = f[cc];
        tl[base] = l;
    }
}

// step 2: face fluxes from the temporaries
template <int D>
__global__ void __launch_bounds__(256)
bt_faces(const double *__restrict__ in, const int64_t *__restrict__ offsets, int64_t stride, int32_t T, int p,
         const double *__restrict__ tf, const double *__restrict__ tl, double *__restrict__ fh) {
    const Geo g = geo(p, D);
    const int64_t total = (int64_t)T * D * g.NF;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / ((int64_t)D * g.NF);
        const int rem = (int)(e - t * D * g.NF);
        const int n = rem / g.NF, f = rem - n * g.NF;
        int i, j, k;
        face_left<D>(g, n, f, i, j, k);
        const int vl = vidx(g, i, j, k);
        const int vr = vl + (n == 0 ? 1 : (n == 1 ? g.W : g.W * g.W));
        const double *P = in + patch_off(offsets, stride, t);
        double qL[NQ], qR[NQ], fL[NQ], fR[NQ], out[NQ];
        load_q(P + (int64_t)vl * NQ, qL);
        load_q(P + (int64_t)vr * NQ, qR);
        const int64_t bl = (t * D + n) * g.V + vl, br = (t * D + n) * g.V + vr;
#pragma unroll
        for (int cc = 0; cc < NQ; ++cc) {
            fL[cc] = tf[bl * NQ + cc];
            fR[cc] = tf[br * NQ + cc];
        }
        rusanov<NQ>(qL, fL, tl[bl], qR, fR, tl[br], out);
#pragma unroll
        for (int cc = 0; cc < NQ; ++cc) fh[((t * D + n) * g.NF + f) * NQ + cc] = out[cc];
    }
}

// step 3: the update of every interior volume
template <int D>
__global__ void __launch_bounds__(256)
bt_update(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets, int64_t stride,
          int32_t T, int p, double r, uint32_t flags, const double *__restrict__ fh) {
    const Geo g = geo(p, D);
    const int inner = D == 2 ? p * p : p * p * p;
    const int64_t total = (int64_t)T * inner;
    const bool periodic = (flags & kPeriodicF) != 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / inner;
        const int c = (int)(e - t * inner);
        int i, j, k;
        interior_coords<D>(g, c, i, j, k);
        double dsum[NQ];
        for (int n = 0; n < D; ++n) {
            const int flo = face_of<D>(g, n, i, j, k);
            const int fhi = flo + 1;  // the face on the high side: next m along n
            const double *a = fh + ((t * D + n) * g.NF + flo) * NQ;
            const double *b = fh + ((t * D + n) * g.NF + fhi) * NQ;
#pragma unroll
            for (int cc = 0; cc < NQ; ++cc) {
                const double d = a[cc] - b[cc];
                dsum[cc] = n == 0 ? d : dsum[cc] + d;
            }
        }
        const int64_t off = patch_off(offsets, stride, t);
        double q[NQ], qn[NQ];
        load_q(in + off + (int64_t)vidx(g, i, j, k) * NQ, q);
        finish_volume<D>(g, q, dsum, r, out + off, i, j, k, periodic, qn);
    }
}

// step 4: per-patch maximum wave speed of the new interior (one block per patch)
template <int D>
__global__ void __launch_bounds__(256)
bt_lambda(const double *__restrict__ out, const int64_t *__restrict__ offsets, int64_t stride, int p, double gamma,
          double *__restrict__ lambda_out) {
    __shared__ double red[256];
    const Geo g = geo(p, D);
    const int64_t t = blockIdx.x;
    const int inner = D == 2 ? p * p : p * p * p;
    const double *P = out + patch_off(offsets, stride, t);
    double m = 0.0;
    for (int c = threadIdx.x; c < inner; c += blockDim.x) {
        int i, j, k;
        interior_coords<D>(g, c, i, j, k);
        double q[NQ];
        load_q(P + (int64_t)vidx(g, i, j, k) * NQ, q);
        m = nanmax(m, volume_lambda<D, NQ>(q, gamma));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) lambda_out[t] = red[0];
}

// ------------------------------------------------------------------ patch-wise
// One work-group per patch: the padded patch state in LDS, then per axis the
// face fluxes of the patch into LDS (barrier) and their differences into the
// threads' accumulators (barrier), then the update and the reduction.
constexpr int kPwBlock = 256;
constexpr int kPwMaxPerThread = 2;  // interior volumes per thread: p^d <= 512

template <int D>
__global__ void __launch_bounds__(kPwBlock)
pw_kernel(const double *__restrict__ in, double *__restrict__ out, const int64_t *__restrict__ offsets, int64_t stride,
          int p, double r, double gamma, uint32_t flags, double *__restrict__ lambda_out) {
    extern __shared__ double lds[];
    const Geo g = geo(p, D);
    double *Q = lds;                            // V * NQ
    double *FH = lds + (size_t)g.V * NQ;        // NF * NQ
    double *red = FH + (size_t)g.NF * NQ;       // kPwBlock
    const int64_t t = blockIdx.x;
    const int64_t off = patch_off(offsets, stride, t);
    const int tid = threadIdx.x;
    const int inner = D == 2 ? p * p : p * p * p;
    const bool periodic = (flags & kPeriodicF) != 0;
    for (int e = tid; e < g.V * NQ; e += kPwBlock) Q[e] = in[off + e];
    __syncthreads();
    double dacc[kPwMaxPerThread][NQ];
    for (int n = 0; n < D; ++n) {
        for (int f = tid; f < g.NF; f += kPwBlock) {
            int i, j, k;
            face_left<D>(g, n, f, i, j, k);
            const int vl = vidx(g, i, j, k);
            const int vr = vl + (n == 0 ? 1 : (n == 1 ? g.W : g.W * g.W));
            double qL[NQ], qR[NQ], fL[NQ], fR[NQ], lL, lR, o[NQ];
            load_q(Q + vl * NQ, qL);
            load_q(Q + vr * NQ, qR);
            const Prim aL = primitives<NQ>(qL, gamma), aR = primitives<NQ>(qR, gamma);
            euler_flux<NQ>(qL, aL, n, fL, lL);
            euler_flux<NQ>(qR, aR, n, fR, lR);
            rusanov<NQ>(qL, fL, lL, qR, fR, lR, o);
#pragma unroll
            for (int cc = 0; cc < NQ; ++cc) FH[f * NQ + cc] = o[cc];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kPwMaxPerThread; ++s) {
            const int c = tid + s * kPwBlock;
            if (c >= inner) continue;
            int i, j, k;
            interior_coords<D>(g, c, i, j, k);
            const int flo = face_of<D>(g, n, i, j, k);
#pragma unroll
            for (int cc = 0; cc < NQ; ++cc) {
                const double d = FH[flo * NQ + cc] - FH[(flo + 1) * NQ + cc];
                dacc[s][cc] = n == 0 ? d : dacc[s][cc] + d;
            }
        }
        __syncthreads();
    }
    double m = 0.0;
#pragma unroll
    for (int s = 0; s < kPwMaxPerThread; ++s) {
        const int c = tid + s * kPwBlock;
        if (c >= inner) continue;
        int i, j, k;
        interior_coords<D>(g, c, i, j, k);
        double q[NQ], qn[NQ];
        load_q(Q + vidx(g, i, j, k) * NQ, q);
        finish_volume<D>(g, q, dacc[s], r, out + off, i, j, k, periodic, qn);
        if (lambda_out) m = nanmax(m, volume_lambda<D, NQ>(qn, gamma));
    }
    if (lambda_out) {
        red[tid] = m;
        __syncthreads();
        for (int s = kPwBlock / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] = nanmax(red[tid], red[tid + s]);
            __syncthreads();
        }
        if (tid == 0) lambda_out[t] = red[0];
    }
}

size_t pw_lds_bytes(int p, int D) {
    const Geo g = geo(p, D);
    return sizeof(double) * ((size_t)g.V * NQ + (size_t)g.NF * NQ + kPwBlock);
}

// ------------------------------------------------------------------ task graph
// node kernels: the face fluxes of one axis of one patch, the update (+ reduction) of one patch
template <int D>
__global__ void __launch_bounds__(256)
tg_flux(const double *__restrict__ patch_in, int p, int n, double gamma, double *__restrict__ fh_patch) {
    const Geo g = geo(p, D);
    for (int f = threadIdx.x; f < g.NF; f += blockDim.x) {
        int i, j, k;
        face_left<D>(g, n, f, i, j, k);
        const int vl = vidx(g, i, j, k);
        const int vr = vl + (n == 0 ? 1 : (n == 1 ? g.W : g.W * g.W));
        double qL[NQ], qR[NQ], fL[NQ], fR[NQ], lL, lR, o[NQ];
        load_q(patch_in + (int64_t)vl * NQ, qL);
        load_q(patch_in + (int64_t)vr * NQ, qR);
        const Prim aL = primitives<NQ>(qL, gamma), aR = primitives<NQ>(qR, gamma);
        euler_flux<NQ>(qL, aL, n, fL, lL);
        euler_flux<NQ>(qR, aR, n, fR, lR);
        rusanov<NQ>(qL, fL, lL, qR, fR, lR, o);
#pragma unroll
        for (int cc = 0; cc < NQ; ++cc) fh_patch[((int64_t)n * g.NF + f) * NQ + cc] = o[cc];
    }
}

template <int D>
__global__ void __launch_bounds__(256)
tg_update(const double *__restrict__ patch_in, double *__restrict__ patch_out, int p, double r, double gamma,
          uint32_t flags, const double *__restrict__ fh_patch, double *__restrict__ lambda_slot) {
    __shared__ double red[256];
    const Geo g = geo(p, D);
    const int inner = D == 2 ? p * p : p * p * p;
    const bool periodic = (flags & kPeriodicF) != 0;
    double m = 0.0;
    for (int c = threadIdx.x; c < inner; c += blockDim.x) {
        int i, j, k;
        interior_coords<D>(g, c, i, j, k);
        double dsum[NQ];
        for (int n = 0; n < D; ++n) {
            const int flo = face_of<D>(g, n, i, j, k);
            const double *a = fh_patch + ((int64_t)n * g.NF + flo) * NQ;
#pragma unroll
            for (int cc = 0; cc < NQ; ++cc) {
                const double d = a[cc] - a[NQ + cc];
                dsum[cc] = n == 0 ? d : dsum[cc] + d;
            }
        }
        double q[NQ], qn[NQ];
        load_q(patch_in + (int64_t)vidx(g, i, j, k) * NQ, q);
        finish_volume<D>(g, q, dsum, r, patch_out, i, j, k, periodic, qn);
        if (lambda_slot) m = nanmax(m, volume_lambda<D, NQ>(qn, gamma));
    }
    if (lambda_slot) {
        red[threadIdx.x] = m;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) *lambda_slot = red[0];
    }
}

// ------------------------------------------------------------------ workspace
struct Workspace {
    void *ptr = nullptr;
    size_t cap = 0;
};
std::mutex g_ws_mu;

// One workspace per device, kept until the process ends (the registry is never destroyed).
Workspace &workspace(int dev) {
    static auto *ws = new std::vector<Workspace>();
    if ((int)ws->size() <= dev) ws->resize(dev + 1);
    return (*ws)[dev];
}

fv_status ensure(Workspace &w, size_t bytes) {
    if (w.cap >= bytes) return FV_OK;
    if (hipDeviceSynchronize() != hipSuccess) return fail(FV_ERR_LAUNCH, "device synchronisation failed");
    if (w.ptr) (void)hipFree(w.ptr);
    w.ptr = nullptr;
    w.cap = 0;
    if (hipMalloc(&w.ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FV_ERR_OOM, "workspace of %zu bytes", bytes);
    }
    w.cap = bytes;
    return FV_OK;
}

template <int D>
fv_status run_batched(const double *in, double *out, const int64_t *d_off, int64_t stride, int32_t T, int p, double r,
                      double gamma, uint32_t flags, double *lambda_out, hipStream_t s, Workspace &w) {
    const Geo g = geo(p, D);
    const size_t tf_n = (size_t)T * D * g.V * NQ, tl_n = (size_t)T * D * g.V, fh_n = (size_t)T * D * g.NF * NQ;
    fv_status st = ensure(w, sizeof(double) * (tf_n + tl_n + fh_n));
    if (st != FV_OK) return st;
    double *tf = static_cast<double *>(w.ptr), *tl = tf + tf_n, *fh = tl + tl_n;
    auto grid = [](int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20); };
    hipLaunchKernelGGL((bt_terms<D>), dim3(grid((int64_t)T * D * g.V)), dim3(256), 0, s, in, d_off, stride, T, p, gamma,
                       tf, tl);
    hipLaunchKernelGGL((bt_faces<D>), dim3(grid((int64_t)T * D * g.NF)), dim3(256), 0, s, in, d_off, stride, T, p, tf,
                       tl, fh);
    const int inner = D == 2 ? p * p : p * p * p;
    hipLaunchKernelGGL((bt_update<D>), dim3(grid((int64_t)T * inner)), dim3(256), 0, s, in, out, d_off, stride, T, p, r,
                       flags, fh);
    if (lambda_out)
        hipLaunchKernelGGL((bt_lambda<D>), dim3(T), dim3(256), 0, s, out, d_off, stride, p, gamma, lambda_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FV_OK : fail(FV_ERR_LAUNCH, "batched launch failed: %s", hipGetErrorString(e));
}

template <int D>
fv_status run_patch_wise(const double *in, double *out, const int64_t *d_off, int64_t stride, int32_t T, int p,
                         double r, double gamma, uint32_t flags, double *lambda_out, hipStream_t s) {
    const size_t lds = pw_lds_bytes(p, D);
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return fail(FV_ERR_NO_DEVICE, "device query failed");
    if (lds > (size_t)lds_max) return fail(FV_ERR_UNSUPPORTED, "a patch of p=%d does not fit the LDS of one work-group", p);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&pw_kernel<D>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((pw_kernel<D>), dim3(T), dim3(kPwBlock), lds, s, in, out, d_off, stride, p, r, gamma, flags,
                       lambda_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FV_OK : fail(FV_ERR_LAUNCH, "patch-wise launch failed: %s", hipGetErrorString(e));
}

// The task graph as dependent command submission: per patch, one face-flux task per axis on
// that axis's library stream and the update task on the caller's stream after events from the
// flux tasks, the way a SYCL runtime executes the task graph its command groups define.  Flux
// tasks of later patches run while earlier patches update.  Nothing outlives the call but work
// queued on streams (no graph objects).  Streams and events are the device's, created once.
struct TaskStreams {
    bool ready = false;
    hipStream_t flux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t start = nullptr;     // the caller's stream reached the call
    hipEvent_t finished = nullptr;  // the previous call's last update (guards the flux workspace)
    hipEvent_t flux_done[3] = {nullptr, nullptr, nullptr};
};

fv_status task_streams(int dev, TaskStreams **out) {
    static auto *all = new std::vector<TaskStreams>();
    if ((int)all->size() <= dev) all->resize(dev + 1);
    TaskStreams &ts = (*all)[dev];
    if (!ts.ready) {
        bool ok = true;
        for (int n = 0; n < 3 && ok; ++n)
            ok = hipStreamCreateWithFlags(&ts.flux[n], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&ts.flux_done[n], hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&ts.start, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&ts.finished, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            return fail(FV_ERR_LAUNCH, "task streams or events could not be created");
        }
        // `finished` starts out complete, so the first call's flux tasks need not wait for it
        if (hipEventRecord(ts.finished, ts.flux[0]) != hipSuccess)
            return fail(FV_ERR_LAUNCH, "hipEventRecord failed");
        ts.ready = true;
    }
    *out = &ts;
    return FV_OK;
}

template <int D>
fv_status run_task_graph(const double *in, double *out, const int64_t *h_off, int64_t stride, int32_t T, int p,
                         double r, double gamma, uint32_t flags, double *lambda_out, hipStream_t s, Workspace &w,
                         int dev) {
    const Geo g = geo(p, D);
    const size_t per_patch = (size_t)D * g.NF * NQ;
    fv_status st = ensure(w, sizeof(double) * per_patch * T);
    if (st != FV_OK) return st;
    TaskStreams *ts = nullptr;
    st = task_streams(dev, &ts);
    if (st != FV_OK) return st;
    double *fh = static_cast<double *>(w.ptr);
    bool ok = hipEventRecord(ts->start, s) == hipSuccess;
    for (int n = 0; n < D && ok; ++n)
        ok = hipStreamWaitEvent(ts->flux[n], ts->start, 0) == hipSuccess &&
             hipStreamWaitEvent(ts->flux[n], ts->finished, 0) == hipSuccess;
    for (int32_t t = 0; t < T && ok; ++t) {
        const double *pin = in + (h_off ? h_off[t] : t * stride);
        double *pout = out + (h_off ? h_off[t] : t * stride);
        double *fht = fh + per_patch * t;
        for (int n = 0; n < D; ++n)
            hipLaunchKernelGGL((tg_flux<D>), dim3(1), dim3(256), 0, ts->flux[n], pin, p, n, gamma, fht);
        // the update waits for this patch's flux tasks (each wait binds to the record just made)
        for (int n = 0; n < D && ok; ++n)
            ok = hipEventRecord(ts->flux_done[n], ts->flux[n]) == hipSuccess &&
                 hipStreamWaitEvent(s, ts->flux_done[n], 0) == hipSuccess;
        hipLaunchKernelGGL((tg_update<D>), dim3(1), dim3(256), 0, s, pin, pout, p, r, gamma, flags,
                           static_cast<const double *>(fht), lambda_out ? lambda_out + t : nullptr);
    }
    ok = ok && hipEventRecord(ts->finished, s) == hipSuccess;
    const hipError_t e = hipGetLastError();
    if (!ok || e != hipSuccess) return fail(FV_ERR_LAUNCH, "task submission failed: %s", hipGetErrorString(e));
    return FV_OK;
}

}  // namespace
}  // namespace fv

using namespace fv;

extern "C" fv_status fv_flavour_update(int32_t flavour, const double *patches_in, double *patches_out,
                                       const int32_t *sizes, const int64_t *offsets, int32_t num_patches, int32_t dim,
                                       int32_t unknowns, double dt, double h, double gamma, uint32_t flags,
                                       double *lambda_out, void *stream) {
    clear_error();
    if (flavour < FV_FLAVOUR_BATCHED || flavour > FV_FLAVOUR_TASK_GRAPH)
        return fail(FV_ERR_INVALID_ARG, "unknown flavour %d", flavour);
    fv_status st = check_scalars(dim, unknowns, dt, h, gamma, flags);
    if (st != FV_OK) return st;
    if (unknowns != 5) return fail(FV_ERR_UNSUPPORTED, "the comparison flavours take five unknowns");
    if (num_patches < 0) return fail(FV_ERR_INVALID_ARG, "num_patches must be >= 0");
    if (num_patches == 0) return FV_OK;
    BatchShape shape;
    st = check_batch(patches_in, patches_out, sizes, offsets, num_patches, dim, unknowns, lambda_out, &shape);
    if (st != FV_OK) return st;
    if (shape.uniform_p < 0) return fail(FV_ERR_UNSUPPORTED, "the comparison flavours take patches of one size");
    const int p = shape.uniform_p;
    if (p * p * (dim == 3 ? p : 1) > kPwBlock * kPwMaxPerThread)
        return fail(FV_ERR_UNSUPPORTED, "the comparison flavours take at most %d interior volumes per patch",
                    kPwBlock * kPwMaxPerThread);
    DeviceContext *ctx = nullptr;
    st = current_context(&ctx);
    if (st != FV_OK) return st;
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t stride = patch_doubles(p, dim, unknowns);
    const double r = dt / h;
    std::lock_guard<std::mutex> g(g_ws_mu);
    Workspace &w = workspace(dev);
    // device copy of the offsets for the batched and patch-wise launches
    int64_t *d_off = nullptr;
    if (offsets && flavour != FV_FLAVOUR_TASK_GRAPH) {
        const size_t need = sizeof(int64_t) * num_patches;
        // offsets sit after the temporaries: grow the workspace to hold both
        const Geo gg = geo(p, dim);
        const size_t tmp = flavour == FV_FLAVOUR_BATCHED
                               ? sizeof(double) * ((size_t)num_patches * dim * gg.V * (NQ + 1) +
                                                   (size_t)num_patches * dim * gg.NF * NQ)
                               : 0;
        st = ensure(w, tmp + need);
        if (st != FV_OK) return st;
        d_off = reinterpret_cast<int64_t *>(static_cast<char *>(w.ptr) + tmp);
        if (hipMemcpyAsync(d_off, offsets, need, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(FV_ERR_LAUNCH, "offset upload failed");
    }
    if (flavour == FV_FLAVOUR_BATCHED)
        return dim == 2 ? run_batched<2>(patches_in, patches_out, d_off, stride, num_patches, p, r, gamma, flags,
                                         lambda_out, s, w)
                        : run_batched<3>(patches_in, patches_out, d_off, stride, num_patches, p, r, gamma, flags,
                                         lambda_out, s, w);
    if (flavour == FV_FLAVOUR_PATCH_WISE)
        return dim == 2 ? run_patch_wise<2>(patches_in, patches_out, d_off, stride, num_patches, p, r, gamma, flags,
                                            lambda_out, s)
                        : run_patch_wise<3>(patches_in, patches_out, d_off, stride, num_patches, p, r, gamma, flags,
                                            lambda_out, s);
    return dim == 2 ? run_task_graph<2>(patches_in, patches_out, offsets, stride, num_patches, p, r, gamma, flags,
                                        lambda_out, s, w, dev)
                    : run_task_graph<3>(patches_in, patches_out, offsets, stride, num_patches, p, r, gamma, flags,
                                        lambda_out, s, w, dev);
}
