// fv_abi.hip -- host side of the C ABI declared in include/fvpatch.h:
// argument validation, status strings, per-device context, and the plain
// per-batch launch of the patch-update kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fvpatch.h"
#include "fv_internal.h"
#include "fv_host.h"

namespace fv {

// Thread-local, fixed-size: recording an error allocates nothing.
static thread_local char g_last_error[512];

fv_status fail(fv_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return s;
}

void clear_error() { g_last_error[0] = '\0'; }

int max_p(int dim) { return dim == 2 ? FV_MAX_P_2D : FV_MAX_P_3D; }

int64_t patch_doubles(int p, int dim, int nq) {
    int64_t w = p + 2;
    return (dim == 2 ? w * w : w * w * w) * nq;
}

fv_status check_scalars(int32_t dim, int32_t nq, double dt, double h, double gamma, uint32_t flags) {
    if (dim != 2 && dim != 3) return fail(FV_ERR_INVALID_ARG, "dim must be 2 or 3 (got %d)", dim);
    if (!(nq == 5 || (dim == 2 && nq == 4))) {
        if (nq == 4 || nq == 5) return fail(FV_ERR_UNSUPPORTED, "unknowns=%d is not supported in %dD", nq, dim);
        return fail(FV_ERR_INVALID_ARG, "unknowns must be 5 (2D/3D) or 4 (2D) (got %d)", nq);
    }
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(FV_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (!std::isfinite(h) || !(h > 0.0)) return fail(FV_ERR_INVALID_ARG, "h must be finite and > 0");
    if (!std::isfinite(gamma) || !(gamma > 1.0)) return fail(FV_ERR_INVALID_ARG, "gamma must be finite and > 1");
    const uint32_t known = FV_HALO_PERIODIC | FV_HALO_FROM_IN;
    if (flags & ~known) return fail(FV_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags & ~known);
    return FV_OK;
}

static bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

static bool ranges_overlap(uintptr_t a0, uintptr_t a1, uintptr_t b0, uintptr_t b1) {
    return a0 < b1 && b0 < a1;
}

fv_status check_layout(const int32_t *sizes, const int64_t *offsets, int32_t num_patches, int32_t dim, int32_t nq,
                       BatchShape *shape, std::pair<int64_t, int64_t> *sort_buf, int64_t sort_cap) {
    if (!sizes) return fail(FV_ERR_INVALID_ARG, "sizes must be non-null");
    if (num_patches <= 0) return fail(FV_ERR_INVALID_ARG, "num_patches must be > 0");
    const int pmax = max_p(dim);
    shape->contiguous = offsets == nullptr;
    int64_t lo = INT64_MAX, hi = 0;
    // Branch-free min / max over the sizes (the compiler vectorises it: this
    // runs once per call over up to millions of entries); the offending entry
    // is looked up only when the range check fails.
    int32_t smin = INT32_MAX, smax = INT32_MIN;
    for (int32_t t = 0; t < num_patches; ++t) {
        smin = std::min(smin, sizes[t]);
        smax = std::max(smax, sizes[t]);
    }
    if (smin < 1 || smax > pmax) {
        for (int32_t t = 0; t < num_patches; ++t)
            if (sizes[t] < 1 || sizes[t] > pmax)
                return fail(FV_ERR_INVALID_ARG, "sizes[%d]=%d outside [1, %d] for %dD", t, sizes[t], pmax, dim);
    }
    shape->uniform_p = smin == smax ? smin : -1;
    if (offsets == nullptr) {
        if (shape->uniform_p < 0) return fail(FV_ERR_INVALID_ARG, "offsets == NULL requires equal sizes");
        lo = 0;
        hi = patch_doubles(shape->uniform_p, dim, nq) * (int64_t)num_patches;
    } else {
        bool sorted = true;
        int64_t prev_end = -1;
        for (int32_t t = 0; t < num_patches; ++t) {
            const int64_t o = offsets[t];
            const int64_t e = o + patch_doubles(sizes[t], dim, nq);  // no overflow: o < 2^48 is checked first
            if (o < 0 || o >= FV_MAX_OFFSET || e > FV_MAX_OFFSET)
                return fail(FV_ERR_INVALID_ARG, "patch %d at offset %lld does not lie in [0, 2^48)", t, (long long)o);
            lo = std::min(lo, o);
            hi = std::max(hi, e);
            if (o < prev_end) sorted = false;
            prev_end = std::max(prev_end, e);
        }
        if (!sorted) {
            std::vector<std::pair<int64_t, int64_t>> own;
            std::pair<int64_t, int64_t> *r = sort_buf;
            if (!r) {
                own.resize(num_patches);
                r = own.data();
            } else if (num_patches > sort_cap) {
                return fail(FV_ERR_INVALID_ARG, "%d patches at unsorted offsets exceed the %lld this call can check",
                            num_patches, (long long)sort_cap);
            }
            for (int32_t t = 0; t < num_patches; ++t) r[t] = {offsets[t], offsets[t] + patch_doubles(sizes[t], dim, nq)};
            std::sort(r, r + num_patches);
            for (int32_t t = 1; t < num_patches; ++t)
                if (r[t].first < r[t - 1].second) return fail(FV_ERR_OVERLAP, "patch ranges overlap");
        }
    }
    shape->lo = lo;
    shape->hi = hi;
    return FV_OK;
}

fv_status check_buffers(const double *in, const double *out, const double *lambda_out, int32_t num_patches,
                        int64_t lo, int64_t hi) {
    if (!in || !out) return fail(FV_ERR_INVALID_ARG, "patches_in and patches_out must be non-null");
    if (!aligned8(in) || !aligned8(out) || (lambda_out && !aligned8(lambda_out)))
        return fail(FV_ERR_INVALID_ARG, "device pointers must be 8-byte aligned");
    const uintptr_t in0 = reinterpret_cast<uintptr_t>(in + lo), in1 = reinterpret_cast<uintptr_t>(in + hi);
    const uintptr_t o0 = reinterpret_cast<uintptr_t>(out + lo), o1 = reinterpret_cast<uintptr_t>(out + hi);
    if (ranges_overlap(in0, in1, o0, o1)) return fail(FV_ERR_OVERLAP, "patches_in and patches_out overlap");
    if (lambda_out) {
        const uintptr_t l0 = reinterpret_cast<uintptr_t>(lambda_out), l1 = reinterpret_cast<uintptr_t>(lambda_out + num_patches);
        if (ranges_overlap(l0, l1, o0, o1) || ranges_overlap(l0, l1, in0, in1))
            return fail(FV_ERR_OVERLAP, "lambda_out overlaps the patch buffers");
    }
    return FV_OK;
}

fv_status check_batch(const double *in, const double *out, const int32_t *sizes, const int64_t *offsets,
                      int32_t num_patches, int32_t dim, int32_t nq, const double *lambda_out,
                      BatchShape *shape, std::pair<int64_t, int64_t> *sort_buf, int64_t sort_cap) {
    if (!in || !out || !sizes) return fail(FV_ERR_INVALID_ARG, "patches_in, patches_out and sizes must be non-null");
    if (!aligned8(in) || !aligned8(out) || (lambda_out && !aligned8(lambda_out)))
        return fail(FV_ERR_INVALID_ARG, "device pointers must be 8-byte aligned");
    fv_status st = check_layout(sizes, offsets, num_patches, dim, nq, shape, sort_buf, sort_cap);
    if (st != FV_OK) return st;
    return check_buffers(in, out, lambda_out, num_patches, shape->lo, shape->hi);
}

// ---------------------------------------------------------------- device context
struct DescSlot {
    std::mutex busy;         // held by the call that fills the slot, from acquire_slot to release_slot
    void *host = nullptr;    // pinned staging, which the kernels read in place
    void *dev = nullptr;     // the device's address of `host`
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};

struct DeviceContext {
    int device = -1;
    bool ok = false;
    std::string arch;
    std::mutex mu;
    static constexpr int kSlots = 4;
    DescSlot slots[kSlots];
    int next = 0;
};

static std::mutex g_ctx_mu;
// Per-device contexts live until the process ends: the registry is never destroyed, so
// no static destructor runs while another thread may still be inside the library.
static std::vector<DeviceContext *> &contexts() {
    static auto *v = new std::vector<DeviceContext *>();
    return *v;
}

fv_status current_context(DeviceContext **out) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(FV_ERR_NO_DEVICE, "no HIP device visible");
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FV_ERR_NO_DEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> g(g_ctx_mu);
    std::vector<DeviceContext *> &g_ctx = contexts();
    if ((int)g_ctx.size() < n) g_ctx.resize(n, nullptr);
    if (!g_ctx[dev]) {
        auto *c = new DeviceContext();
        c->device = dev;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            c->arch = prop.gcnArchName;
            c->ok = c->arch.rfind("gfx950", 0) == 0;
        }
        g_ctx[dev] = c;
    }
    DeviceContext *c = g_ctx[dev];
    if (!c->ok) return fail(FV_ERR_UNSUPPORTED, "device %d is '%s'; this library is built for gfx950 only", dev, c->arch.c_str());
    *out = c;
    return FV_OK;
}

// Take a descriptor slot with at least `bytes` of pinned and device memory,
// waiting for the last launch that used it.
fv_status acquire_slot(DeviceContext *c, size_t bytes, DescSlot **out) {
    DescSlot *sp = nullptr;
    {
        std::lock_guard<std::mutex> g(c->mu);
        sp = &c->slots[c->next];
        c->next = (c->next + 1) % DeviceContext::kSlots;
    }
    DescSlot &s = *sp;
    // With more concurrent callers than slots, a call on another thread may still be filling this
    // slot: wait for it to release the slot, then for the launches that read it.
    std::unique_lock<std::mutex> hold(s.busy);
    if (s.used && hipEventSynchronize(s.done) != hipSuccess) return fail(FV_ERR_LAUNCH, "descriptor event wait failed");
    if (!s.done && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
        return fail(FV_ERR_LAUNCH, "hipEventCreate failed");
    if (s.cap < bytes) {
        if (s.host) (void)hipHostFree(s.host);
        s.host = s.dev = nullptr;
        s.cap = 0;
        s.used = false;
        size_t cap = std::max<size_t>(bytes, 1 << 16);
        if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess) return fail(FV_ERR_OOM, "pinned allocation of %zu bytes failed", cap);
        if (hipHostGetDevicePointer(&s.dev, s.host, 0) != hipSuccess || !s.dev)
            return fail(FV_ERR_LAUNCH, "no device address for the pinned descriptor staging");
        s.cap = cap;
    }
    hold.release();  // unlocked by release_slot
    *out = &s;
    return FV_OK;
}

// Marks the slot's contents as read by the work enqueued on `stream` so far and hands it back.
fv_status release_slot(DescSlot *s, hipStream_t stream) {
    const hipError_t e = hipEventRecord(s->done, stream);
    if (e == hipSuccess) {
        s->used = true;
    } else {
        (void)hipStreamSynchronize(stream);  // no event to wait on later: let the readers finish now
        s->used = false;
    }
    s->busy.unlock();
    return e == hipSuccess ? FV_OK : fail(FV_ERR_LAUNCH, "hipEventRecord failed");
}

// ---------------------------------------------------------------- tuning table
static std::mutex g_tune_mu;
static fv_tuning g_tune[2][2][FV_MAX_P_2D + 1];  // [dim-2][nq-4][p], kernel = -1 when unset
static bool g_tune_init = false;

static fv_tuning *tune_slot(int dim, int nq, int p) {
    if (!g_tune_init) {
        for (auto &a : g_tune)
            for (auto &b : a)
                for (auto &c : b) c = fv_tuning{-1, 0, 0, 0};
        g_tune_init = true;
    }
    return &g_tune[dim - 2][nq - 4][p];
}

static int default_block_for(int kernel, int p, int dim) {
    if (kernel == FV_KERNEL_WAVE) return 256;
    if (kernel == FV_KERNEL_FIXED) return wave2d_fixed_block();
    if (kernel == FV_KERNEL_TILE) return tile2d_default_block(p);
    return default_block(p, dim);
}

static void fixed_shape(int dim, int p, int *prefetch, int *rows) {
    if (dim == 2) wave2d_fixed_shape(p, prefetch, rows);
    else wave3d_fixed_shape(p, prefetch, rows);
}

fv_tuning default_tuning(int dim, int nq, int p) {
    fv_tuning t{FV_KERNEL_AUTO, 0, 0, 0};
    t.kernel = (dim == 2 && wave2d_fits(p)) ? FV_KERNEL_WAVE : FV_KERNEL_BLOCK;
    if ((dim == 2 && wave2d_fixed(p, nq)) || (dim == 3 && wave3d_fixed(p, nq))) t.kernel = FV_KERNEL_FIXED;
    t.block = default_block_for(t.kernel, p, dim);
    t.prefetch = t.kernel == FV_KERNEL_WAVE ? 4 : 1;
    t.rows = t.kernel == FV_KERNEL_WAVE ? 6 : 1;
    if (t.kernel == FV_KERNEL_FIXED) fixed_shape(dim, p, &t.prefetch, &t.rows);
    return t;
}

fv_tuning tuning_for(int dim, int nq, int p) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    const fv_tuning *t = tune_slot(dim, nq, p);
    return t->kernel < 0 ? default_tuning(dim, nq, p) : *t;
}

void apply_tuning(UpdateLaunch &L) { apply_tuning(L, tuning_for(L.dim, L.nq, L.p)); }

void apply_tuning(UpdateLaunch &L, const fv_tuning &t) {
    L.kernel = t.kernel;
    L.block = t.block;
    L.prefetch = t.prefetch;
    L.rows = t.rows;
}

// Launch parameters shared by every launch of one plain call (everything but the patch
// selection): the PDE, the step, the flags, lambda.
UpdateLaunch launch_template(const double *in, double *out, int32_t dim, int32_t nq, double dt, double h,
                             double gamma, uint32_t flags, double *lambda_out, const PdeArgs *pde) {
    UpdateLaunch L;
    if (pde) {
        L.pde = pde->pde;
        for (int k = 0; k < 4; ++k) L.pde_prm[k] = pde->prm[k];
    }
    L.dt = dt;
    L.in = in;
    L.out = out;
    L.dim = dim;
    L.nq = nq;
    L.r = dt / h;
    L.gamma = gamma;
    L.flags = flags;
    L.lambda_out = lambda_out;
    return L;
}

// Euler classes take their tuned kernel; the other PDEs their built wave form, else the
// generic block kernel (launch_pde picks).
static void tune_launch(UpdateLaunch &X) {
    if (X.pde == kPdeEuler) {
        apply_tuning(X);
    } else {
        X.kernel = FV_KERNEL_BLOCK;
        X.block = 0;
    }
}

bool regular_batch(const int64_t *offsets, int32_t T, int32_t dim, int32_t nq, const BatchShape &shape,
                   int64_t *base, int64_t *stride) {
    // Equal sizes at evenly spaced offsets (offsets[t] = offsets[0] + t s, s at least one patch):
    // the launch of a contiguous batch from offsets[0] with stride s, no descriptors to upload.
    *base = 0;
    *stride = shape.uniform_p > 0 ? patch_doubles(shape.uniform_p, dim, nq) : 0;
    bool regular = shape.contiguous;
    if (!shape.contiguous && shape.uniform_p > 0) {
        *base = offsets[0];
        if (T > 1) *stride = offsets[1] - offsets[0];
        regular = *stride >= patch_doubles(shape.uniform_p, dim, nq);
        for (int32_t t = 2; t < T && regular; ++t) regular = offsets[t] - offsets[t - 1] == *stride;
    }
    return regular;
}

fv_status regular_launch(const UpdateLaunch &tmpl, const int64_t *offsets, int32_t T, const BatchShape &shape,
                         hipStream_t stream, bool *taken) {
    *taken = false;
    const int32_t dim = tmpl.dim, nq = tmpl.nq;
    int64_t base = 0, stride = 0;
    if (!regular_batch(offsets, T, dim, nq, shape, &base, &stride)) return FV_OK;
    *taken = true;
    UpdateLaunch L = tmpl;
    L.in = tmpl.in + base;
    L.out = tmpl.out + base;
    L.num_items = T;
    L.p = shape.uniform_p;
    L.stride = stride;
    // 16-byte accesses need every patch to start on a 16-byte boundary and span an even number
    // of doubles (the row loaders of the runtime-size kernels assume it), as on the descriptor path
    L.vec2 = (L.stride % 2 == 0) && patch_doubles(shape.uniform_p, dim, nq) % 2 == 0 && aligned16(L.in) &&
             aligned16(L.out);
    tune_launch(L);
    if (L.pde == kPdeEuler && L.kernel == FV_KERNEL_FIXED && fixed_odd_rows(dim, L.p, nq)) L.vec2 = aligned16(L.out);
    hipError_t e = launch_update(L, stream);
    if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "kernel launch failed: %s", hipGetErrorString(e));
    return FV_OK;
}

size_t descriptor_bytes(int32_t T, bool with_out_offsets) {
    return (size_t)T * (sizeof(int64_t) + sizeof(int32_t)) + (with_out_offsets ? (size_t)T * sizeof(int64_t) : 0);
}

void build_descriptors(const int32_t *sizes, const int64_t *offsets, const int64_t *out_offsets, int32_t T,
                       int32_t dim, int32_t nq, void *host, DescriptorGroups *g) {
    const int pmax = max_p(dim);
    for (int p = 0; p <= pmax + 1; ++p) {
        g->count[p] = 0;
        g->odd[p] = 0;
    }
    for (int32_t t = 0; t < T; ++t) g->count[sizes[t]]++;
    g->start[0] = 0;
    for (int p = 1; p <= pmax + 1; ++p) g->start[p] = g->start[p - 1] + g->count[p - 1];
    g->num = T;
    g->with_out = out_offsets != nullptr;
    int32_t fill[FV_MAX_P_2D + 2];
    for (int p = 0; p <= pmax + 1; ++p) fill[p] = g->start[p];
    const int64_t nout = out_offsets ? T : 0;
    int64_t *hoff = static_cast<int64_t *>(host);
    int64_t *hout = hoff + T;
    int32_t *hid = reinterpret_cast<int32_t *>(hout + nout);
    for (int32_t t = 0; t < T; ++t) {
        const int32_t k = fill[sizes[t]]++;
        const int64_t o = offsets ? offsets[t] : (int64_t)t * patch_doubles(sizes[t], dim, nq);
        hoff[k] = o;
        hid[k] = t;
        g->odd[sizes[t]] |= (char)(o & 1);
        if (out_offsets) {
            hout[k] = out_offsets[t];
            g->odd[sizes[t]] |= (char)(out_offsets[t] & 1);
        }
    }
}

fv_status launch_descriptor_groups(const UpdateLaunch &tmpl, const void *dev, const DescriptorGroups &g,
                                   hipStream_t stream) {
    const int32_t T = g.num;
    const int64_t nout = g.with_out ? T : 0;
    const int64_t *doff = static_cast<const int64_t *>(dev);
    const int64_t *dout = g.with_out ? doff + T : nullptr;
    const int32_t *did = reinterpret_cast<const int32_t *>(doff + T + nout);
    const bool bufs16 = aligned16(tmpl.in) && aligned16(tmpl.out);
    for (int p = max_p(tmpl.dim); p >= 1; --p) {  // largest patches first
        if (!g.count[p]) continue;
        UpdateLaunch L = tmpl;
        L.num_items = g.count[p];
        L.p = p;
        L.offsets = doff + g.start[p];
        L.out_offsets = dout ? dout + g.start[p] : nullptr;
        L.ids = did + g.start[p];
        L.vec2 = bufs16 && !g.odd[p] && patch_doubles(p, tmpl.dim, tmpl.nq) % 2 == 0;
        tune_launch(L);
        if (L.pde == kPdeEuler && L.kernel == FV_KERNEL_FIXED && fixed_odd_rows(tmpl.dim, p, tmpl.nq))
            L.vec2 = aligned16(tmpl.out);
        hipError_t e = launch_update(L, stream);
        if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "kernel launch failed (p=%d): %s", p, hipGetErrorString(e));
    }
    return FV_OK;
}

// Plain per-batch launch; arguments already validated.  out_offsets (host,
// optional) places patch t's output at out + out_offsets[t] instead of at its
// input offset (used by the serving loop, whose patches ping-pong between two
// slots individually).
fv_status plain_update(const double *in, double *out, const int32_t *sizes, const int64_t *offsets,
                       int32_t T, int32_t dim, int32_t nq, double dt, double h, double gamma, uint32_t flags,
                       double *lambda_out, hipStream_t stream, const BatchShape &shape,
                       const int64_t *out_offsets, const PdeArgs *pde) {
    DeviceContext *ctx = nullptr;
    fv_status st = current_context(&ctx);
    if (st != FV_OK) return st;
    const UpdateLaunch L = launch_template(in, out, dim, nq, dt, h, gamma, flags, lambda_out, pde);
    if (!out_offsets) {
        bool taken = false;
        st = regular_launch(L, offsets, T, shape, stream, &taken);
        if (st != FV_OK || taken) return st;
    }
    // Group the patches by size (counting sort) into (offset, id) lists in a pinned slot, which the
    // kernels read in place (the slot is reused only after the launches that read it have run).
    const size_t bytes = descriptor_bytes(T, out_offsets != nullptr);
    DescSlot *slot = nullptr;
    st = acquire_slot(ctx, bytes, &slot);
    if (st != FV_OK) return st;
    DescriptorGroups g;
    build_descriptors(sizes, offsets, out_offsets, T, dim, nq, slot->host, &g);
    st = launch_descriptor_groups(L, slot->dev, g, stream);
    const fv_status rs = release_slot(slot, stream);
    return st != FV_OK ? st : rs;
}

// ---------------------------------------------------------------- no-allocation launch
// Descriptor memory of fv_patch_batch_update_noalloc: (offset, id) per patch, 12 bytes, in
// a fixed array of the device image.  Each GPU holds its own copy at its own address until
// the process ends.  In host code `scratch` is only a host-side stand-in: kernels and copies
// take the device address resolved once per device (NoallocDevice::ptr).
constexpr size_t kNoallocBytes = (size_t)FV_NOALLOC_MAX_PATCHES * (sizeof(int64_t) + sizeof(int32_t));
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kNoallocDevices = 64;
struct NoallocDevice {
    bool ready = false;
    void *ptr = nullptr;          // this GPU's copy of `scratch`
    hipEvent_t staged = nullptr;  // recorded after each upload from the host staging array
};
// All state below is guarded by g_noalloc_mu: calls are serialised on the host.
static std::mutex g_noalloc_mu;
static NoallocDevice g_noalloc_dev[kNoallocDevices];
static hipEvent_t g_noalloc_last_upload = nullptr;  // the upload that last read the staging array
alignas(64) static unsigned char g_noalloc_host[kNoallocBytes];
static std::pair<int64_t, int64_t> g_noalloc_sort[FV_NOALLOC_MAX_PATCHES];

// Set-up on the first call on a device (that device current): the device address of
// `scratch` and the upload event.
static fv_status noalloc_device(int device, NoallocDevice **out) {
    if (device < 0 || device >= kNoallocDevices)
        return fail(FV_ERR_UNSUPPORTED, "device %d: the no-allocation entry point serves devices 0..%d", device,
                    kNoallocDevices - 1);
    NoallocDevice &d = g_noalloc_dev[device];
    if (!d.ready) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FV_ERR_LAUNCH, "device address of the descriptor array unavailable: %s", hipGetErrorString(e));
        if (!d.staged && hipEventCreateWithFlags(&d.staged, hipEventDisableTiming) != hipSuccess)
            return fail(FV_ERR_LAUNCH, "hipEventCreate failed");
        d.ptr = ptr;
        d.ready = true;
    }
    *out = &d;
    return FV_OK;
}

static fv_status noalloc_update(const double *in, double *out, const int32_t *sizes, const int64_t *offsets,
                                int32_t T, int32_t dim, int32_t nq, double dt, double h, double gamma,
                                uint32_t flags, double *lambda_out, hipStream_t stream) {
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    BatchShape shape;
    fv_status st = check_batch(in, out, sizes, offsets, T, dim, nq, lambda_out, &shape, g_noalloc_sort,
                               FV_NOALLOC_MAX_PATCHES);
    if (st != FV_OK) return st;
    DeviceContext *ctx = nullptr;
    st = current_context(&ctx);
    if (st != FV_OK) return st;
    NoallocDevice *nd = nullptr;
    st = noalloc_device(ctx->device, &nd);
    if (st != FV_OK) return st;
    const UpdateLaunch L = launch_template(in, out, dim, nq, dt, h, gamma, flags, lambda_out, nullptr);
    bool taken = false;
    st = regular_launch(L, offsets, T, shape, stream, &taken);  // no descriptors at all
    if (st != FV_OK || taken) return st;
    // the staging array may still feed the previous upload
    if (g_noalloc_last_upload && hipEventSynchronize(g_noalloc_last_upload) != hipSuccess)
        return fail(FV_ERR_LAUNCH, "wait for the previous descriptor upload failed");
    DescriptorGroups grp;
    build_descriptors(sizes, offsets, nullptr, T, dim, nq, g_noalloc_host, &grp);
    if (hipMemcpyAsync(nd->ptr, g_noalloc_host, descriptor_bytes(T, false), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return fail(FV_ERR_LAUNCH, "descriptor upload failed");
    if (hipEventRecord(nd->staged, stream) != hipSuccess) return fail(FV_ERR_LAUNCH, "hipEventRecord failed");
    g_noalloc_last_upload = nd->staged;
    return launch_descriptor_groups(L, nd->ptr, grp, stream);
}

// Unknowns and parameters of a built-in PDE in dim dimensions.
fv_status pde_shape(int32_t pde, int32_t dim, int32_t *nq, int32_t *nprm) {
    if (dim != 2 && dim != 3) return fail(FV_ERR_INVALID_ARG, "dim must be 2 or 3 (got %d)", dim);
    switch (pde) {
        case FV_PDE_EULER: *nq = 5; *nprm = 1; return FV_OK;
        case FV_PDE_SHALLOW_WATER:
            if (dim != 2) return fail(FV_ERR_UNSUPPORTED, "the shallow water equations are 2D");
            *nq = 4; *nprm = 2; return FV_OK;
        case FV_PDE_ADVECTION: *nq = 1; *nprm = 3; return FV_OK;
        case FV_PDE_ACOUSTICS:
        case FV_PDE_ACOUSTICS_NCP: *nq = 1 + dim; *nprm = 2; return FV_OK;
        default: return fail(FV_ERR_INVALID_ARG, "unknown PDE %d", pde);
    }
}

fv_status check_class(int32_t dim, int32_t nq, int32_t p) {
    if (dim != 2 && dim != 3) return fail(FV_ERR_INVALID_ARG, "dim must be 2 or 3 (got %d)", dim);
    if (!(nq == 5 || (dim == 2 && nq == 4))) return fail(FV_ERR_INVALID_ARG, "unsupported unknowns=%d for %dD", nq, dim);
    if (p < 1 || p > max_p(dim)) return fail(FV_ERR_INVALID_ARG, "p=%d outside [1, %d]", p, max_p(dim));
    return FV_OK;
}

// Validate launch parameters for a class and fill in their defaults (the rules of
// fv_set_tuning; also used for a plan's own table).
fv_status resolve_tuning(int32_t dim, int32_t unknowns, int32_t p, const fv_tuning &in, fv_tuning *out) {
    fv_status st = check_class(dim, unknowns, p);
    if (st != FV_OK) return st;
    const fv_tuning *t = &in;
    if (t->kernel < FV_KERNEL_AUTO || t->kernel > FV_KERNEL_FIXED) return fail(FV_ERR_INVALID_ARG, "unknown kernel %d", t->kernel);
    if (t->block < 0 || t->block > 1024 || t->block % 64 != 0) return fail(FV_ERR_INVALID_ARG, "block must be a multiple of 64 in [0, 1024]");
    if (t->prefetch < 0 || t->prefetch > 4) return fail(FV_ERR_INVALID_ARG, "prefetch must be in [0, 4]");
    if (t->rows < 0 || t->rows > 16) return fail(FV_ERR_INVALID_ARG, "rows must be in [0, 16]");
    fv_tuning v = *t;
    const fv_tuning d = default_tuning(dim, unknowns, p);
    if (v.kernel == FV_KERNEL_AUTO) {
        v.kernel = d.kernel;
        // explicit prefetch / rows other than the fixed-size build's: the runtime-size wave kernel
        if (v.kernel == FV_KERNEL_FIXED && ((v.prefetch != 0 && v.prefetch != d.prefetch) ||
                                            (v.rows != 0 && v.rows != d.rows)))
            v.kernel = FV_KERNEL_WAVE;
    }
    if (v.kernel == FV_KERNEL_WAVE && !(dim == 2 && wave2d_fits(p)))
        return fail(FV_ERR_UNSUPPORTED, "the wave kernel needs 2D and p + 2 <= 64");
    if (v.kernel == FV_KERNEL_TILE && !(dim == 2 && tile2d_fits(p)))
        return fail(FV_ERR_UNSUPPORTED, "the tile kernel needs 2D and p*p <= 1024");
    if (v.kernel == FV_KERNEL_FIXED) {
        if (!((dim == 2 && wave2d_fixed(p, unknowns)) || (dim == 3 && wave3d_fixed(p, unknowns))))
            return fail(FV_ERR_UNSUPPORTED, "no fixed-size kernel for dim=%d unknowns=%d p=%d", dim, unknowns, p);
        int pf = 0, rows = 0;
        fixed_shape(dim, p, &pf, &rows);
        const int fb = wave2d_fixed_block();
        if (v.block != 0 && v.block != fb) return fail(FV_ERR_INVALID_ARG, "the fixed-size kernel takes %d threads", fb);
        if ((v.prefetch != 0 && v.prefetch != pf) || (v.rows != 0 && v.rows != rows))
            return fail(FV_ERR_INVALID_ARG, "the fixed-size kernel for p=%d is built with prefetch %d and rows %d", p,
                        pf, rows);
        *out = fv_tuning{FV_KERNEL_FIXED, fb, pf, rows};
        return FV_OK;
    }
    if (v.block == 0) v.block = v.kernel == d.kernel ? d.block : default_block_for(v.kernel, p, dim);
    if (v.kernel == FV_KERNEL_WAVE && v.block > 256) return fail(FV_ERR_INVALID_ARG, "the wave kernel takes at most 256 threads");
    if (v.kernel == FV_KERNEL_TILE) {
        if (v.block < p * p) return fail(FV_ERR_INVALID_ARG, "the tile kernel needs at least p*p = %d threads", p * p);
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            tile2d_patches_per_block(p, unknowns, v.block, (size_t)lds_max) < 1)
            return fail(FV_ERR_INVALID_ARG, "a tile of p=%d needs more LDS than the device offers", p);
        (void)hipGetLastError();
    }
    if (v.kernel == FV_KERNEL_BLOCK) {
        if (v.block < plane_lanes(p, dim)) return fail(FV_ERR_INVALID_ARG, "block %d smaller than the %d lanes of a patch", v.block, plane_lanes(p, dim));
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            update_lds_bytes(dim, unknowns, v.block) > (size_t)lds_max)
            return fail(FV_ERR_INVALID_ARG, "block %d needs more LDS than the device offers", v.block);
        (void)hipGetLastError();
    }
    if (v.prefetch == 0) v.prefetch = v.kernel == FV_KERNEL_WAVE ? 4 : 1;
    if (v.rows == 0) v.rows = v.kernel == FV_KERNEL_WAVE ? 6 : 1;
    if (v.kernel == FV_KERNEL_WAVE) {
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            wave2d_lds_bytes(p, unknowns, v.block, v.rows) > (size_t)lds_max)
            return fail(FV_ERR_INVALID_ARG, "block %d with %d staged rows needs more LDS than the device offers", v.block, v.rows);
        (void)hipGetLastError();
    }
    *out = v;
    return FV_OK;
}


}  // namespace fv

using namespace fv;

extern "C" {

fv_status fv_patch_batch_update(const double *patches_in, double *patches_out, const int32_t *sizes,
                                const int64_t *offsets, int32_t num_patches, int32_t dim, int32_t unknowns,
                                double dt, double h, double gamma, uint32_t flags, double *lambda_out,
                                void *stream) {
    clear_error();
    fv_status st = check_scalars(dim, unknowns, dt, h, gamma, flags);
    if (st != FV_OK) return st;
    if (num_patches < 0) return fail(FV_ERR_INVALID_ARG, "num_patches must be >= 0");
    if (num_patches == 0) return FV_OK;
    BatchShape shape;
    st = check_batch(patches_in, patches_out, sizes, offsets, num_patches, dim, unknowns, lambda_out, &shape);
    if (st != FV_OK) return st;
    return plain_update(patches_in, patches_out, sizes, offsets, num_patches, dim, unknowns, dt, h, gamma, flags,
                        lambda_out, static_cast<hipStream_t>(stream), shape, nullptr);
}

fv_status fv_patch_batch_update_noalloc(const double *patches_in, double *patches_out, const int32_t *sizes,
                                        const int64_t *offsets, int32_t num_patches, int32_t dim, int32_t unknowns,
                                        double dt, double h, double gamma, uint32_t flags, double *lambda_out,
                                        void *stream) {
    clear_error();
    fv_status st = check_scalars(dim, unknowns, dt, h, gamma, flags);
    if (st != FV_OK) return st;
    if (num_patches < 0) return fail(FV_ERR_INVALID_ARG, "num_patches must be >= 0");
    if (num_patches > FV_NOALLOC_MAX_PATCHES)
        return fail(FV_ERR_INVALID_ARG, "%d patches exceed the %d the no-allocation entry point's descriptor array holds",
                    num_patches, FV_NOALLOC_MAX_PATCHES);
    if (num_patches == 0) return FV_OK;
    return noalloc_update(patches_in, patches_out, sizes, offsets, num_patches, dim, unknowns, dt, h, gamma, flags,
                          lambda_out, static_cast<hipStream_t>(stream));
}

fv_status fv_pde_unknowns(int32_t pde, int32_t dim, int32_t *unknowns, int32_t *num_params) {
    clear_error();
    if (!unknowns || !num_params) return fail(FV_ERR_INVALID_ARG, "unknowns and num_params must be non-null");
    return pde_shape(pde, dim, unknowns, num_params);
}

fv_status fv_pde_batch_update(int32_t pde, const double *params, int32_t num_params, const double *patches_in,
                              double *patches_out, const int32_t *sizes, const int64_t *offsets,
                              int32_t num_patches, int32_t dim, double dt, double h, uint32_t flags,
                              double *lambda_out, void *stream) {
    clear_error();
    int32_t nq = 0, nprm = 0;
    fv_status st = pde_shape(pde, dim, &nq, &nprm);
    if (st != FV_OK) return st;
    if (num_params != nprm) return fail(FV_ERR_INVALID_ARG, "PDE %d takes %d parameters (got %d)", pde, nprm, num_params);
    if (!params) return fail(FV_ERR_INVALID_ARG, "params must be non-null");
    for (int k = 0; k < nprm; ++k)
        if (!std::isfinite(params[k])) return fail(FV_ERR_INVALID_ARG, "params[%d] is not finite", k);
    if (pde == FV_PDE_EULER)
        return fv_patch_batch_update(patches_in, patches_out, sizes, offsets, num_patches, dim, 5, dt, h, params[0],
                                     flags, lambda_out, stream);
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(FV_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (!std::isfinite(h) || !(h > 0.0)) return fail(FV_ERR_INVALID_ARG, "h must be finite and > 0");
    if (flags & ~(FV_HALO_PERIODIC | FV_HALO_FROM_IN))
        return fail(FV_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags & ~(FV_HALO_PERIODIC | FV_HALO_FROM_IN));
    PdeArgs args;
    args.pde = pde;
    for (int k = 0; k < nprm; ++k) args.prm[k] = params[k];
    if (pde == FV_PDE_SHALLOW_WATER && !(params[0] > 0.0)) return fail(FV_ERR_INVALID_ARG, "g must be > 0");
    if (pde == FV_PDE_ACOUSTICS || pde == FV_PDE_ACOUSTICS_NCP) {
        if (!(params[0] > 0.0) || !(params[1] > 0.0)) return fail(FV_ERR_INVALID_ARG, "rho0 and K0 must be > 0");
        args.prm[2] = std::sqrt(params[1] / params[0]);  // the sound speed, a kernel parameter
    }
    if (num_patches < 0) return fail(FV_ERR_INVALID_ARG, "num_patches must be >= 0");
    if (num_patches == 0) return FV_OK;
    BatchShape shape;
    st = check_batch(patches_in, patches_out, sizes, offsets, num_patches, dim, nq, lambda_out, &shape);
    if (st != FV_OK) return st;
    DeviceContext *ctx = nullptr;
    st = current_context(&ctx);
    if (st != FV_OK) return st;
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return fail(FV_ERR_NO_DEVICE, "device attributes unavailable");
    const int32_t pmax = *std::max_element(sizes, sizes + num_patches);  // LDS grows with p
    if (pde_min_lds_bytes(pde, dim, pmax) > (size_t)lds_max)
        return fail(FV_ERR_UNSUPPORTED, "a patch of size %d needs more LDS than a block has for PDE %d in %dD", pmax,
                    pde, dim);
    return plain_update(patches_in, patches_out, sizes, offsets, num_patches, dim, nq, dt, h, 0.0, flags, lambda_out,
                        static_cast<hipStream_t>(stream), shape, nullptr, &args);
}


fv_status fv_set_tuning(int32_t dim, int32_t unknowns, int32_t p, const fv_tuning *t) {
    clear_error();
    if (!t) {
        fv_status st = check_class(dim, unknowns, p);
        if (st != FV_OK) return st;
        std::lock_guard<std::mutex> g(g_tune_mu);
        *tune_slot(dim, unknowns, p) = fv_tuning{-1, 0, 0, 0};
        return FV_OK;
    }
    fv_tuning v;
    fv_status st = resolve_tuning(dim, unknowns, p, *t, &v);
    if (st != FV_OK) return st;
    std::lock_guard<std::mutex> g(g_tune_mu);
    *tune_slot(dim, unknowns, p) = v;
    return FV_OK;
}

fv_status fv_get_tuning(int32_t dim, int32_t unknowns, int32_t p, fv_tuning *t) {
    clear_error();
    fv_status st = check_class(dim, unknowns, p);
    if (st != FV_OK) return st;
    if (!t) return fail(FV_ERR_INVALID_ARG, "tuning must be non-null");
    *t = tuning_for(dim, unknowns, p);
    return FV_OK;
}

const char *fv_status_string(fv_status s) {
    switch (s) {
        case FV_OK: return "ok";
        case FV_ERR_INVALID_ARG: return "invalid argument";
        case FV_ERR_UNSUPPORTED: return "unsupported";
        case FV_ERR_NO_DEVICE: return "no device";
        case FV_ERR_LAUNCH: return "launch failed";
        case FV_ERR_OOM: return "out of memory";
        case FV_ERR_BUDGET: return "over budget";
        case FV_ERR_OVERLAP: return "overlapping buffers";
    }
    return "unknown status";
}

const char *fv_last_error(void) { return g_last_error; }

int32_t fv_version(void) { return 100; }

#ifndef FV_BUILD_ID
#define FV_BUILD_ID "unknown"
#endif
const char *fv_build_id(void) { return FV_BUILD_ID; }

}  // extern "C"
