// fv_mesh.hip -- the mesh steps either side of the patch update (Sec. 2.2):
// face halos from neighbouring patches, per-patch step sizes (local time
// stepping), and the fused mesh step.
//
// A mesh is a fixed set of equal-size patches with a face-neighbour table,
// validated and uploaded once.  fv_mesh_step runs the fixed-size kernels in
// their mesh form: a patch's face-halo volumes are read straight from the
// neighbours' interiors while the patch is updated, so no halo is ever copied
// (the halo layer costs no HBM traffic beyond what the update reads anyway),
// and patch t advances by its own dt[t] with its own h[t].  fv_mesh_halo_fill
// materialises the halos (any patch size) for callers that want them in
// memory; fv_local_dt forms dt[t] = cfl h[t] / (d lambda[t]) on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "fv_host.h"
#include "fv_internal.h"

struct fv_mesh {
    int device = -1;
    int32_t dim = 2, nq = 5, p = 0, num_patches = 0;
    bool contiguous = true;      // offsets == NULL: patch t at t * stride
    bool even = true;            // every patch starts at an even double (16-byte chunks possible)
    int64_t stride = 0;
    int64_t lo = 0, hi = 0;      // extent of the patches in doubles
    int64_t *d_offsets = nullptr;
    int32_t *d_neighbors = nullptr;
};

namespace fv {
namespace {

// One thread per (patch, face, volume of the face, unknown): the halo volume
// of patch t on face (axis a, side s) takes the neighbour's interior volume
// next to their common face.
__global__ void __launch_bounds__(256)
halo_fill_kernel(double *__restrict__ state, const int64_t *__restrict__ offsets, int64_t stride,
                 const int32_t *__restrict__ neighbors, int32_t T, int32_t dim, int32_t nq, int32_t p) {
    const int W = p + 2;
    const int64_t face_vols = dim == 2 ? p : (int64_t)p * p;
    const int64_t per_patch = 2 * dim * face_vols * nq;
    const int64_t total = (int64_t)T * per_patch;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = g / per_patch;
        int64_t rem = g - t * per_patch;
        const int f = (int)(rem / (face_vols * nq));
        rem -= (int64_t)f * face_vols * nq;
        const int64_t v = rem / nq;
        const int q = (int)(rem - v * nq);
        const int32_t nb = neighbors[t * 2 * dim + f];
        if (nb < 0) continue;
        const int a = f >> 1, s = f & 1;
        // the two coordinates along the other axes, each in 1..p (the second is 0 in 2D)
        const int u = 1 + (int)(v % p);
        const int w = dim == 3 ? 1 + (int)(v / p) : 0;
        int h[3], src[3];
        int m = 0;
        for (int ax = 0; ax < 3; ++ax) {
            if (ax == a) continue;
            h[ax] = src[ax] = (m++ == 0) ? u : w;
        }
        h[a] = s == 0 ? 0 : p + 1;
        src[a] = s == 0 ? p : 1;
        const int64_t ho = ((int64_t)(h[2] * W + h[1]) * W + h[0]) * nq + q;
        const int64_t so = ((int64_t)(src[2] * W + src[1]) * W + src[0]) * nq + q;
        const int64_t ot = offsets ? offsets[t] : t * stride;
        const int64_t on = offsets ? offsets[nb] : (int64_t)nb * stride;
        state[ot + ho] = state[on + so];
    }
}

__global__ void __launch_bounds__(256)
local_dt_kernel(const double *__restrict__ lambda, const double *__restrict__ h, int32_t T, int32_t dim, double cfl,
                double *__restrict__ dt) {
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) dt[t] = cfl * h[t] / (dim * lambda[t]);
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

}  // namespace
}  // namespace fv

using namespace fv;

extern "C" {

fv_status fv_mesh_create(fv_mesh **mesh, const int32_t *sizes, const int64_t *offsets, const int32_t *neighbors,
                         int32_t num_patches, int32_t dim, int32_t unknowns) {
    clear_error();
    if (!mesh) return fail(FV_ERR_INVALID_ARG, "mesh must be non-null");
    *mesh = nullptr;
    if (dim != 2 && dim != 3) return fail(FV_ERR_INVALID_ARG, "dim must be 2 or 3 (got %d)", dim);
    if (!(unknowns == 5 || (dim == 2 && unknowns == 4)))
        return fail(FV_ERR_INVALID_ARG, "unsupported unknowns=%d for %dD", unknowns, dim);
    if (num_patches <= 0) return fail(FV_ERR_INVALID_ARG, "a mesh needs at least one patch");
    if (!sizes || !neighbors) return fail(FV_ERR_INVALID_ARG, "sizes and neighbors must be non-null");
    BatchShape shape;
    fv_status st = check_layout(sizes, offsets, num_patches, dim, unknowns, &shape);
    if (st != FV_OK) return st;
    if (shape.uniform_p < 0) return fail(FV_ERR_UNSUPPORTED, "the patches of a mesh must all have the same size");
    const int64_t nn = (int64_t)num_patches * 2 * dim;
    for (int64_t e = 0; e < nn; ++e)
        if (neighbors[e] < -1 || neighbors[e] >= num_patches)
            return fail(FV_ERR_INVALID_ARG, "neighbors[%lld]=%d is neither -1 nor a patch index", (long long)e,
                        neighbors[e]);
    DeviceContext *ctx = nullptr;
    st = current_context(&ctx);
    if (st != FV_OK) return st;

    auto *m = new fv_mesh();
    (void)hipGetDevice(&m->device);
    m->dim = dim;
    m->nq = unknowns;
    m->p = shape.uniform_p;
    m->num_patches = num_patches;
    m->contiguous = offsets == nullptr;
    m->stride = patch_doubles(m->p, dim, unknowns);
    m->lo = shape.lo;
    m->hi = shape.hi;
    m->even = m->stride % 2 == 0;
    if (offsets)
        for (int32_t t = 0; t < num_patches; ++t)
            if (offsets[t] & 1) m->even = false;
    bool ok = hipMalloc(&m->d_neighbors, sizeof(int32_t) * nn) == hipSuccess &&
              hipMemcpy(m->d_neighbors, neighbors, sizeof(int32_t) * nn, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && offsets)
        ok = hipMalloc(&m->d_offsets, sizeof(int64_t) * num_patches) == hipSuccess &&
             hipMemcpy(m->d_offsets, offsets, sizeof(int64_t) * num_patches, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        if (m->d_neighbors) (void)hipFree(m->d_neighbors);
        if (m->d_offsets) (void)hipFree(m->d_offsets);
        delete m;
        return fail(FV_ERR_OOM, "device memory for the mesh tables");
    }
    *mesh = m;
    return FV_OK;
}

fv_status fv_mesh_halo_fill(fv_mesh *mesh, double *patches, void *stream) {
    clear_error();
    if (!mesh) return fail(FV_ERR_INVALID_ARG, "mesh must be non-null");
    if (!patches || !aligned(patches, 8))
        return fail(FV_ERR_INVALID_ARG, "patches must be a non-null 8-byte aligned device pointer");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != mesh->device)
        return fail(FV_ERR_INVALID_ARG, "the mesh belongs to device %d", mesh->device);
    const int64_t face_vols = mesh->dim == 2 ? mesh->p : (int64_t)mesh->p * mesh->p;
    const int64_t total = (int64_t)mesh->num_patches * 2 * mesh->dim * face_vols * mesh->nq;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(halo_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       patches, mesh->d_offsets, mesh->stride, mesh->d_neighbors, mesh->num_patches, mesh->dim,
                       mesh->nq, mesh->p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "halo fill launch failed: %s", hipGetErrorString(e));
    return FV_OK;
}

fv_status fv_mesh_step(fv_mesh *mesh, const double *patches_in, double *patches_out, const double *dt,
                       const double *h, double gamma, double *lambda_out, void *stream) {
    clear_error();
    if (!mesh) return fail(FV_ERR_INVALID_ARG, "mesh must be non-null");
    if (!dt || !h || !aligned(dt, 8) || !aligned(h, 8))
        return fail(FV_ERR_INVALID_ARG, "dt and h must be non-null 8-byte aligned device arrays");
    if (!std::isfinite(gamma) || !(gamma > 1.0)) return fail(FV_ERR_INVALID_ARG, "gamma must be finite and > 1");
    const bool fixed = mesh->dim == 2 ? wave2d_fixed(mesh->p, mesh->nq) : wave3d_fixed(mesh->p, mesh->nq);
    if (!fixed)
        return fail(FV_ERR_UNSUPPORTED,
                    "the mesh step is built for 2D p in {3, 5, 9, 16, 17} and 3D p in {4, 6, 8} with 5 unknowns "
                    "(p=%d, %dD, N=%d): fill the halos with fv_mesh_halo_fill and use fv_patch_batch_update",
                    mesh->p, mesh->dim, mesh->nq);
    fv_status st = check_buffers(patches_in, patches_out, lambda_out, mesh->num_patches, mesh->lo, mesh->hi);
    if (st != FV_OK) return st;
    const uintptr_t d0 = reinterpret_cast<uintptr_t>(dt), d1 = d0 + sizeof(double) * mesh->num_patches;
    const uintptr_t h0 = reinterpret_cast<uintptr_t>(h), h1 = h0 + sizeof(double) * mesh->num_patches;
    const uintptr_t o0 = reinterpret_cast<uintptr_t>(patches_out + mesh->lo);
    const uintptr_t o1 = reinterpret_cast<uintptr_t>(patches_out + mesh->hi);
    if ((d0 < o1 && o0 < d1) || (h0 < o1 && o0 < h1))
        return fail(FV_ERR_OVERLAP, "dt / h overlap the output patches");
    if (lambda_out) {
        const uintptr_t l0 = reinterpret_cast<uintptr_t>(lambda_out), l1 = l0 + sizeof(double) * mesh->num_patches;
        if ((d0 < l1 && l0 < d1) || (h0 < l1 && l0 < h1)) return fail(FV_ERR_OVERLAP, "dt / h overlap lambda_out");
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != mesh->device)
        return fail(FV_ERR_INVALID_ARG, "the mesh belongs to device %d", mesh->device);
    UpdateLaunch L;
    L.in = patches_in;
    L.out = patches_out;
    L.offsets = mesh->d_offsets;
    L.num_items = mesh->num_patches;
    L.p = mesh->p;
    L.dim = mesh->dim;
    L.nq = mesh->nq;
    L.stride = mesh->stride;
    L.gamma = gamma;
    L.flags = 0;
    L.lambda_out = lambda_out;
    L.kernel = FV_KERNEL_FIXED;
    L.vec2 = mesh->even && aligned(patches_in, 16) && aligned(patches_out, 16);
    L.mesh.neighbors = mesh->d_neighbors;
    L.mesh.dt = dt;
    L.mesh.h = h;
    hipError_t e = launch_update(L, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "mesh step launch failed: %s", hipGetErrorString(e));
    return FV_OK;
}

fv_status fv_local_dt(const double *lambda, const double *h, int32_t num_patches, int32_t dim, double cfl,
                      double *dt_out, void *stream) {
    clear_error();
    if (num_patches < 0) return fail(FV_ERR_INVALID_ARG, "num_patches must be >= 0");
    if (num_patches == 0) return FV_OK;
    if (dim != 2 && dim != 3) return fail(FV_ERR_INVALID_ARG, "dim must be 2 or 3 (got %d)", dim);
    if (!std::isfinite(cfl) || !(cfl > 0.0)) return fail(FV_ERR_INVALID_ARG, "cfl must be finite and > 0");
    if (!lambda || !h || !dt_out || !aligned(lambda, 8) || !aligned(h, 8) || !aligned(dt_out, 8))
        return fail(FV_ERR_INVALID_ARG, "lambda, h and dt_out must be non-null 8-byte aligned device arrays");
    DeviceContext *ctx = nullptr;
    fv_status st = current_context(&ctx);
    if (st != FV_OK) return st;
    const int blocks = (num_patches + 255) / 256;
    hipLaunchKernelGGL(local_dt_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), lambda, h,
                       num_patches, dim, cfl, dt_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "local dt launch failed: %s", hipGetErrorString(e));
    return FV_OK;
}

fv_status fv_mesh_destroy(fv_mesh *mesh) {
    clear_error();
    if (!mesh) return FV_OK;
    (void)hipDeviceSynchronize();  // no step of this mesh may still be running
    if (mesh->d_neighbors) (void)hipFree(mesh->d_neighbors);
    if (mesh->d_offsets) (void)hipFree(mesh->d_offsets);
    delete mesh;
    return FV_OK;
}

}  // extern "C"
