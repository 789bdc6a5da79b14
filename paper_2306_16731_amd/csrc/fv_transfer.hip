// fv_transfer.hip -- one step of patches that live scattered in host memory.
//
// The paper's patches are separate allocations on the CPU heap that are
// brought to the accelerator one by one; those scattered transfers dominate
// its runtime (Sec. 5, Fig. 4), and recycling device allocations instead of
// freeing them ("managed memory", Sec. 4) was its best remedy.  Three ways to
// move such patches through the fused update:
//   per patch   every patch copied to a recycled device area with its own
//               synchronous hipMemcpy from pageable memory, one launch over
//               the batch, every patch copied back the same way (the paper's
//               explicit copy with recycled allocations);
//   staged      host threads gather all patches into one pinned buffer, one
//               copy to the device, one launch, one copy back, host threads
//               scatter the results (bulk transfer, nothing overlapped);
//   pipelined   the batch cut into chunks of whole patches; each of
//               `host_threads` threads takes chunks in turn and carries each
//               through gather into pinned staging, hipMemcpyAsync to the
//               device, the fused update, the copy back (on the thread's own
//               stream) and the scatter, with `slots` chunks of its own in
//               flight: gathers, scatters, both copy directions and the
//               updates of different chunks overlap.
// The device-resident pool (patches kept in HBM between steps) is the fourth
// point of comparison and needs no code here.
#include <emmintrin.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fv_host.h"

namespace fv {
namespace {

constexpr int64_t kDefaultChunk = 8ll << 20;
constexpr int32_t kDefaultSlots = 2;
constexpr int32_t kDefaultThreads = 8;
constexpr int64_t kZeroCopyChunk = 32ll << 20;
constexpr int32_t kZeroCopySlots = 4;

// Fixed set of host threads running one job at a time: a job is `parts`
// calls body(0) .. body(parts - 1), part 0 on the calling thread and part k
// on worker k - 1.
class HostPool {
public:
    ~HostPool() { resize(0); }
    int size() const { return (int)workers_.size(); }

    void resize(int n) {
        if (n == size()) return;
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
            ++epoch_;
        }
        cv_.notify_all();
        for (auto &w : workers_) w.join();
        workers_.clear();
        stop_ = false;
        // each worker starts from the epoch current now, not from whatever it reads once it runs
        // (a job posted before it first looks would otherwise never be seen)
        const uint64_t e0 = epoch_;
        for (int w = 0; w < n; ++w) workers_.emplace_back([this, w, e0]() { loop(w, e0); });
    }

    // parts <= size() + 1
    void run_parts(int parts, const std::function<void(int)> &body) {
        if (parts <= 1 || size() == 0) {
            for (int k = 0; k < parts; ++k) body(k);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            body_ = &body;
            parts_ = parts;
            pending_ = size();
            ++epoch_;
        }
        cv_.notify_all();
        body(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this]() { return pending_ == 0; });
        body_ = nullptr;
    }

    // body(t) for every t in [first, first + count), in equal ranges over the
    // calling thread and at most threads - 1 workers
    void run(int32_t first, int32_t count, int threads, const std::function<void(int32_t)> &body) {
        const int most = std::max(1, std::min(threads, size() + 1));
        const int parts = count < 2 * most ? 1 : most;
        run_parts(parts, [&](int k) {
            const int32_t lo = first + (int32_t)((int64_t)count * k / parts);
            const int32_t hi = first + (int32_t)((int64_t)count * (k + 1) / parts);
            for (int32_t t = lo; t < hi; ++t) body(t);
        });
    }

private:
    void loop(int w, uint64_t seen) {
        for (;;) {
            const std::function<void(int)> *body = nullptr;
            int parts = 0;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&]() { return epoch_ != seen; });
                seen = epoch_;
                if (stop_) return;
                body = body_;
                parts = parts_;
            }
            if (w + 1 < parts) (*body)(w + 1);
            {
                std::lock_guard<std::mutex> g(mu_);
                if (--pending_ == 0) done_cv_.notify_one();
            }
        }
    }

    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    uint64_t epoch_ = 0;
    bool stop_ = false;
    const std::function<void(int)> *body_ = nullptr;
    int parts_ = 1, pending_ = 0;
};

struct Slot {
    double *h_in = nullptr, *h_out = nullptr, *h_lam = nullptr;  // pinned staging
    double *d_in = nullptr, *d_out = nullptr, *d_lam = nullptr;  // device chunk
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int32_t first = 0, count = 0;  // patches of the chunk in flight; count 0 = idle
};

// Staging slots of one capacity (grow-only).
struct SlotSet {
    std::vector<Slot> slots;
    size_t doubles = 0;   // per slot
    int32_t patches = 0;  // eigenvalues per slot
};

// Zero-copy chunk in flight: device copies of the chunk, its table of patch
// pointers (host staging and device copy), its eigenvalues.
struct ZSlot {
    double *d_in = nullptr, *d_out = nullptr, *d_lam = nullptr, *h_lam = nullptr;
    const double **h_ptr = nullptr, **d_ptr = nullptr;  // [2 * patches]: inputs, then outputs
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int32_t first = 0, count = 0;
};

struct ZSlotSet {
    std::vector<ZSlot> slots;
    size_t doubles = 0;
    int32_t patches = 0;
};

// Per-device state, grow-only, kept until the process ends.
struct Transfer {
    std::mutex mu;
    SlotSet chunks;               // pipelined
    ZSlotSet zchunks;             // zero copy
    SlotSet whole;                // staged: one slot for the whole batch
    double *d_all = nullptr;      // per patch: recycled device area
    size_t all_doubles = 0;
    HostPool pool;
};

std::mutex g_mu;

// Per-device transfer state, kept until the process ends (the registry is never destroyed).
Transfer *transfer_for(int dev) {
    static auto *all = new std::vector<Transfer *>();
    std::vector<Transfer *> &g_transfer = *all;
    std::lock_guard<std::mutex> g(g_mu);
    if ((int)g_transfer.size() <= dev) g_transfer.resize(dev + 1, nullptr);
    if (!g_transfer[dev]) g_transfer[dev] = new Transfer();
    return g_transfer[dev];
}

void free_slot(Slot &s) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.h_in) (void)hipHostFree(s.h_in);
    if (s.h_out) (void)hipHostFree(s.h_out);
    if (s.h_lam) (void)hipHostFree(s.h_lam);
    if (s.d_in) (void)hipFree(s.d_in);
    if (s.d_out) (void)hipFree(s.d_out);
    if (s.d_lam) (void)hipFree(s.d_lam);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = Slot{};
}

fv_status ensure_slots(SlotSet &set, int32_t slots, size_t doubles, int32_t patches) {
    if ((int32_t)set.slots.size() >= slots && set.doubles >= doubles && set.patches >= patches) return FV_OK;
    const size_t want_doubles = std::max(set.doubles, doubles);
    const int32_t want_patches = std::max(set.patches, patches);
    const int32_t want_slots = std::max((int32_t)set.slots.size(), slots);
    for (auto &s : set.slots) free_slot(s);
    set.slots.assign(want_slots, Slot{});
    set.doubles = want_doubles;
    set.patches = want_patches;
    const size_t b = sizeof(double) * want_doubles, bl = sizeof(double) * want_patches;
    for (auto &s : set.slots) {
        const bool ok = hipHostMalloc(reinterpret_cast<void **>(&s.h_in), b, hipHostMallocDefault) == hipSuccess &&
                        hipHostMalloc(reinterpret_cast<void **>(&s.h_out), b, hipHostMallocDefault) == hipSuccess &&
                        hipHostMalloc(reinterpret_cast<void **>(&s.h_lam), bl, hipHostMallocDefault) == hipSuccess &&
                        hipMalloc(&s.d_in, b) == hipSuccess && hipMalloc(&s.d_out, b) == hipSuccess &&
                        hipMalloc(&s.d_lam, bl) == hipSuccess &&
                        hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
                        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            for (auto &y : set.slots) free_slot(y);
            set.slots.clear();
            set.doubles = 0;
            set.patches = 0;
            return fail(FV_ERR_OOM, "staging for %d chunks of %zu bytes", want_slots, b);
        }
    }
    return FV_OK;
}

void free_zslot(ZSlot &s) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.d_in) (void)hipFree(s.d_in);
    if (s.d_out) (void)hipFree(s.d_out);
    if (s.d_lam) (void)hipFree(s.d_lam);
    if (s.h_lam) (void)hipHostFree(s.h_lam);
    if (s.h_ptr) (void)hipHostFree(s.h_ptr);
    if (s.d_ptr) (void)hipFree(s.d_ptr);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = ZSlot{};
}

fv_status ensure_zslots(ZSlotSet &set, int32_t slots, size_t doubles, int32_t patches) {
    if ((int32_t)set.slots.size() >= slots && set.doubles >= doubles && set.patches >= patches) return FV_OK;
    const size_t want_doubles = std::max(set.doubles, doubles);
    const int32_t want_patches = std::max(set.patches, patches);
    const int32_t want_slots = std::max((int32_t)set.slots.size(), slots);
    for (auto &z : set.slots) free_zslot(z);
    set.slots.assign(want_slots, ZSlot{});
    set.doubles = want_doubles;
    set.patches = want_patches;
    const size_t b = sizeof(double) * want_doubles, bl = sizeof(double) * want_patches;
    const size_t bp = 2 * sizeof(double *) * want_patches;
    for (auto &z : set.slots) {
        const bool ok = hipMalloc(&z.d_in, b) == hipSuccess && hipMalloc(&z.d_out, b) == hipSuccess &&
                        hipMalloc(&z.d_lam, bl) == hipSuccess &&
                        hipHostMalloc(reinterpret_cast<void **>(&z.h_lam), bl, hipHostMallocDefault) == hipSuccess &&
                        hipHostMalloc(reinterpret_cast<void **>(&z.h_ptr), bp, hipHostMallocDefault) == hipSuccess &&
                        hipMalloc(reinterpret_cast<void **>(&z.d_ptr), bp) == hipSuccess &&
                        hipStreamCreateWithFlags(&z.stream, hipStreamNonBlocking) == hipSuccess &&
                        hipEventCreateWithFlags(&z.done, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            for (auto &y : set.slots) free_zslot(y);
            set.slots.clear();
            set.doubles = 0;
            set.patches = 0;
            return fail(FV_ERR_OOM, "zero-copy buffers for %d chunks of %zu bytes", want_slots, b);
        }
    }
    return FV_OK;
}

fv_status ensure_area(Transfer &x, size_t doubles) {
    if (x.all_doubles >= doubles) return FV_OK;
    if (x.d_all) (void)hipFree(x.d_all);
    x.d_all = nullptr;
    x.all_doubles = 0;
    if (hipMalloc(&x.d_all, sizeof(double) * doubles) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FV_ERR_OOM, "device area of %zu bytes", sizeof(double) * doubles);
    }
    x.all_doubles = doubles;
    return FV_OK;
}

// Copy n doubles with streaming stores (the destination lines are not read
// first and do not displace the cache: neither the pinned staging nor the
// caller's patches are read again by this thread).  Both pointers 8-byte
// aligned.  Callers fence (store_fence) before another agent reads dst.
void stream_copy(double *dst, const double *src, size_t n) {
    size_t i = 0;
    if ((reinterpret_cast<uintptr_t>(dst) & 15u) && n) {
        dst[0] = src[0];
        i = 1;
    }
    for (; i + 8 <= n; i += 8) {
        const __m128d a = _mm_loadu_pd(src + i), b = _mm_loadu_pd(src + i + 2);
        const __m128d c = _mm_loadu_pd(src + i + 4), d = _mm_loadu_pd(src + i + 6);
        _mm_stream_pd(dst + i, a);
        _mm_stream_pd(dst + i + 2, b);
        _mm_stream_pd(dst + i + 4, c);
        _mm_stream_pd(dst + i + 6, d);
    }
    for (; i + 2 <= n; i += 2) _mm_stream_pd(dst + i, _mm_loadu_pd(src + i));
    if (i < n) dst[i] = src[i];
}

// Make this thread's streaming stores visible before the data is handed on.
void store_fence() { _mm_sfence(); }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Call {
    const double *const *in;
    double *const *out;
    const int32_t *sizes;
    int32_t T, p, dim, nq;
    double dt, h, gamma;
    uint32_t flags;
    double *lambda_out;
    int64_t pd;     // doubles per patch
    size_t pbytes;  // bytes per patch
};

// Queue a chunk already gathered in s.h_in (patches first .. first + count - 1) on the slot's
// stream: copy in, output initialised to the input (halo volumes keep their values), update,
// copy back, event.  On an error the stream is drained before returning.
fv_status enqueue_chunk(Slot &s, const Call &c, int32_t first, int32_t count) {
    const size_t bytes = c.pbytes * (size_t)count;
    const BatchShape uniform{true, c.p, 0, (int64_t)count * c.pd};
    fv_status st = FV_OK;
    if (hipMemcpyAsync(s.d_in, s.h_in, bytes, hipMemcpyHostToDevice, s.stream) != hipSuccess ||
        hipMemcpyAsync(s.d_out, s.d_in, bytes, hipMemcpyDeviceToDevice, s.stream) != hipSuccess)
        st = fail(FV_ERR_LAUNCH, "copy of patches %d.. to the device failed", first);
    if (st == FV_OK)
        st = plain_update(s.d_in, s.d_out, c.sizes + first, nullptr, count, c.dim, c.nq, c.dt, c.h, c.gamma,
                          c.flags, c.lambda_out ? s.d_lam : nullptr, s.stream, uniform, nullptr);
    if (st == FV_OK &&
        (hipMemcpyAsync(s.h_out, s.d_out, bytes, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
         (c.lambda_out &&
          hipMemcpyAsync(s.h_lam, s.d_lam, sizeof(double) * count, hipMemcpyDeviceToHost, s.stream) != hipSuccess) ||
         hipEventRecord(s.done, s.stream) != hipSuccess))
        st = fail(FV_ERR_LAUNCH, "copy of patches %d.. to the host failed", first);
    if (st != FV_OK) {
        (void)hipStreamSynchronize(s.stream);
        (void)hipGetLastError();
        s.count = 0;
        return st;
    }
    s.first = first;
    s.count = count;
    return FV_OK;
}

// Every patch copied on its own, synchronously, through the recycled device area
// (input at [0, T pd), output at [T pd, 2 T pd), eigenvalues after them).
fv_status per_patch(Transfer &x, const Call &c, fv_transfer_stats *stats) {
    const size_t n = (size_t)c.T * c.pd;
    fv_status st = ensure_area(x, 2 * n + (size_t)c.T);
    if (st != FV_OK) return st;
    double *d_in = x.d_all, *d_out = x.d_all + n, *d_lam = x.d_all + 2 * n;
    const BatchShape uniform{true, c.p, 0, (int64_t)n};
    for (int32_t t = 0; t < c.T; ++t)
        if (hipMemcpy(d_in + (size_t)t * c.pd, c.in[t], c.pbytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail(FV_ERR_LAUNCH, "copy of patch %d to the device failed", t);
    // the output patches start as the input ones (halo volumes keep their values)
    if (hipMemcpy(d_out, d_in, sizeof(double) * n, hipMemcpyDeviceToDevice) != hipSuccess)
        return fail(FV_ERR_LAUNCH, "device copy failed");
    st = plain_update(d_in, d_out, c.sizes, nullptr, c.T, c.dim, c.nq, c.dt, c.h, c.gamma, c.flags,
                      c.lambda_out ? d_lam : nullptr, nullptr, uniform, nullptr);
    if (st != FV_OK) return st;
    if (hipDeviceSynchronize() != hipSuccess)
        return fail(FV_ERR_LAUNCH, "update failed: %s", hipGetErrorString(hipGetLastError()));
    for (int32_t t = 0; t < c.T; ++t)
        if (hipMemcpy(c.out[t], d_out + (size_t)t * c.pd, c.pbytes, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(FV_ERR_LAUNCH, "copy of patch %d to the host failed", t);
    if (c.lambda_out &&
        hipMemcpy(c.lambda_out, d_lam, sizeof(double) * c.T, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(FV_ERR_LAUNCH, "copy of the eigenvalues to the host failed");
    if (stats) {
        stats->bytes_to_device = (int64_t)(n * sizeof(double));
        stats->bytes_to_host = (int64_t)(n * sizeof(double)) + (c.lambda_out ? 8ll * c.T : 0);
    }
    return FV_OK;
}

// All patches through one pinned buffer: threaded gather, one copy each way, threaded scatter.
fv_status staged(Transfer &x, const Call &c, int threads, fv_transfer_stats *stats) {
    fv_status st = ensure_slots(x.whole, 1, (size_t)c.T * c.pd, c.T);
    if (st != FV_OK) return st;
    if (x.pool.size() < threads - 1) x.pool.resize(threads - 1);
    Slot &s = x.whole.slots[0];
    double host_s = 0.0;
    double t0 = now_s();
    x.pool.run(0, c.T, threads, [&](int32_t t) {
        stream_copy(s.h_in + (size_t)t * c.pd, c.in[t], (size_t)c.pd);
        store_fence();  // each thread's streaming stores complete before the copy engine reads the staging
    });
    host_s += now_s() - t0;
    st = enqueue_chunk(s, c, 0, c.T);
    if (st != FV_OK) return st;
    if (hipEventSynchronize(s.done) != hipSuccess) {
        s.count = 0;
        return fail(FV_ERR_LAUNCH, "staged step failed: %s", hipGetErrorString(hipGetLastError()));
    }
    s.count = 0;
    t0 = now_s();
    x.pool.run(0, c.T, threads, [&](int32_t t) {
        stream_copy(c.out[t], s.h_out + (size_t)t * c.pd, (size_t)c.pd);
        store_fence();
    });
    if (c.lambda_out) std::memcpy(c.lambda_out, s.h_lam, sizeof(double) * c.T);
    host_s += now_s() - t0;
    if (stats) {
        const int64_t n = (int64_t)c.T * (int64_t)c.pbytes;
        stats->bytes_to_device = n;
        stats->bytes_to_host = n + (c.lambda_out ? 8ll * c.T : 0);
        stats->host_copy_seconds = host_s;
    }
    return FV_OK;
}

// Chunks of whole patches; each of `workers` host threads takes chunks in turn and keeps
// `depth` of its own in flight, each through its own staging slot and stream.
fv_status pipelined(Transfer &x, const Call &c, const fv_transfer_config &cfg, int dev, fv_transfer_stats *stats) {
    const int32_t per_chunk = (int32_t)std::min<int64_t>(cfg.chunk_bytes / (int64_t)c.pbytes, c.T);
    const int32_t nchunks = (c.T + per_chunk - 1) / per_chunk;
    const int workers = (int)std::min<int32_t>(cfg.host_threads, nchunks);
    const int depth = cfg.slots;
    fv_status st = ensure_slots(x.chunks, workers * depth, (size_t)per_chunk * c.pd, per_chunk);
    if (st != FV_OK) return st;
    if (x.pool.size() < workers - 1) x.pool.resize(workers - 1);
    struct Result {
        fv_status st = FV_OK;
        std::string msg;
        double host_s = 0.0;
        int64_t to_dev = 0, to_host = 0;
    };
    std::vector<Result> res(workers);
    std::atomic<int32_t> next{0};
    std::atomic<bool> stop{false};

    x.pool.run_parts(workers, [&](int w) {
        Result &r = res[w];
        Slot *mine = x.chunks.slots.data() + (size_t)w * depth;
        auto failed = [&](fv_status s) {
            r.st = s;
            r.msg = fv_last_error();
            stop.store(true);
        };
        if (hipSetDevice(dev) != hipSuccess) {
            failed(fail(FV_ERR_LAUNCH, "worker %d could not select device %d", w, dev));
            return;
        }
        // wait for a slot's chunk and scatter its patches and eigenvalues to the caller's arrays
        auto retire = [&](Slot &s) -> bool {
            if (s.count == 0) return true;
            const hipError_t e = hipEventSynchronize(s.done);
            const int32_t first = s.first, count = s.count;
            s.count = 0;
            if (e != hipSuccess) {
                failed(fail(FV_ERR_LAUNCH, "chunk at patch %d failed: %s", first, hipGetErrorString(e)));
                return false;
            }
            const double t0 = now_s();
            for (int32_t t = first; t < first + count; ++t)
                stream_copy(c.out[t], s.h_out + (size_t)(t - first) * c.pd, (size_t)c.pd);
            store_fence();
            if (c.lambda_out) std::memcpy(c.lambda_out + first, s.h_lam, sizeof(double) * count);
            r.host_s += now_s() - t0;
            return true;
        };
        for (int k = 0; !stop.load(std::memory_order_relaxed); ++k) {
            const int32_t chunk = next.fetch_add(1);
            if (chunk >= nchunks) break;
            Slot &s = mine[k % depth];
            if (!retire(s)) break;
            const int32_t first = chunk * per_chunk, count = std::min(per_chunk, c.T - first);
            const double t0 = now_s();
            for (int32_t t = first; t < first + count; ++t)
                stream_copy(s.h_in + (size_t)(t - first) * c.pd, c.in[t], (size_t)c.pd);
            store_fence();  // before the copy engine reads the staging
            r.host_s += now_s() - t0;
            const fv_status e = enqueue_chunk(s, c, first, count);
            if (e != FV_OK) {
                failed(e);
                break;
            }
            r.to_dev += (int64_t)c.pbytes * count;
            r.to_host += (int64_t)c.pbytes * count + (c.lambda_out ? 8ll * count : 0);
        }
        // every chunk in flight is waited for, also after an error
        for (int k = 0; k < depth; ++k) {
            if (r.st == FV_OK) {
                retire(mine[k]);
            } else if (mine[k].count) {
                (void)hipStreamSynchronize(mine[k].stream);
                mine[k].count = 0;
            }
        }
    });
    fv_transfer_stats sum{0, 0, 0.0, 0.0};
    for (const Result &r : res) {
        if (r.st != FV_OK) return fail(r.st, "%s", r.msg.c_str());
        sum.bytes_to_device += r.to_dev;
        sum.bytes_to_host += r.to_host;
        sum.host_copy_seconds += r.host_s;
    }
    if (stats) *stats = sum;
    return FV_OK;
}

// ------------------------------------------------------------------ pinned patch memory
// Blocks handed out by fv_host_alloc, by host start address, with the address
// the device uses for them.
struct PinnedBlock {
    size_t bytes;
    double *dev;
};
std::mutex g_pin_mu;
std::map<uintptr_t, PinnedBlock> &pinned_blocks() {  // never destroyed, like the blocks it lists
    static auto *m = new std::map<uintptr_t, PinnedBlock>();
    return *m;
}

// The device address of host range [p, p + bytes) if it lies inside one pinned
// block, else null.
const double *pinned_device(const void *p, size_t bytes) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> g(g_pin_mu);
    auto it = pinned_blocks().upper_bound(a);
    if (it == pinned_blocks().begin()) return nullptr;
    --it;
    if (a + bytes > it->first + it->second.bytes) return nullptr;
    return it->second.dev + (a - it->first) / sizeof(double);
}

// Patch t of a chunk from (device-visible) host memory into both device copies:
// one block per patch, 16-byte moves where the patch and the copies allow them.
__global__ void __launch_bounds__(256) gather_patches(const double *const *__restrict__ src, double *__restrict__ d_in,
                                                      double *__restrict__ d_out, int64_t pd) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const int64_t t = blockIdx.x;
    const double *s = src[t];
    double *a = d_in + t * pd, *b = d_out + t * pd;
    if (((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(a)) & 15u) == 0 && pd % 2 == 0) {
        for (int64_t k = threadIdx.x; k < pd / 2; k += blockDim.x) {
            const dv2 v = reinterpret_cast<const dv2 *>(s)[k];
            reinterpret_cast<dv2 *>(a)[k] = v;
            reinterpret_cast<dv2 *>(b)[k] = v;
        }
    } else {
        for (int64_t k = threadIdx.x; k < pd; k += blockDim.x) {
            const double v = s[k];
            a[k] = v;
            b[k] = v;
        }
    }
}

// Patch t of a chunk from the device copy to (device-visible) host memory.
__global__ void __launch_bounds__(256) scatter_patches(const double *__restrict__ d_out, double *const *__restrict__ dst,
                                                       int64_t pd) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const int64_t t = blockIdx.x;
    const double *s = d_out + t * pd;
    double *d = dst[t];
    if (((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(d)) & 15u) == 0 && pd % 2 == 0) {
        for (int64_t k = threadIdx.x; k < pd / 2; k += blockDim.x)
            reinterpret_cast<dv2 *>(d)[k] = reinterpret_cast<const dv2 *>(s)[k];
    } else {
        for (int64_t k = threadIdx.x; k < pd; k += blockDim.x) d[k] = s[k];
    }
}

// Patches in memory from fv_host_alloc: the GPU reads and writes them in place.  Chunks of
// whole patches, `slots` of them in flight on their own streams: table of patch addresses up,
// gather kernel (PCIe reads), update, scatter kernel (PCIe writes), eigenvalues down.
fv_status zero_copy(Transfer &x, const Call &c, const fv_transfer_config &cfg, const std::vector<const double *> &din,
                    const std::vector<const double *> &dout, fv_transfer_stats *stats) {
    const int32_t per_chunk = (int32_t)std::min<int64_t>(cfg.chunk_bytes / (int64_t)c.pbytes, c.T);
    const int32_t nchunks = (c.T + per_chunk - 1) / per_chunk;
    const int32_t nslots = std::min<int32_t>(cfg.slots, nchunks);
    fv_status st = ensure_zslots(x.zchunks, nslots, (size_t)per_chunk * c.pd, per_chunk);
    if (st != FV_OK) return st;
    const BatchShape uniform{true, c.p, 0, (int64_t)per_chunk * c.pd};
    fv_status err = FV_OK;
    auto retire = [&](ZSlot &z) {
        if (z.count == 0) return;
        const hipError_t e = hipEventSynchronize(z.done);
        if (e != hipSuccess && err == FV_OK) err = fail(FV_ERR_LAUNCH, "chunk failed: %s", hipGetErrorString(e));
        if (e == hipSuccess && c.lambda_out) std::memcpy(c.lambda_out + z.first, z.h_lam, sizeof(double) * z.count);
        z.count = 0;
    };
    for (int32_t chunk = 0; chunk < nchunks && err == FV_OK; ++chunk) {
        ZSlot &z = x.zchunks.slots[chunk % nslots];
        retire(z);
        if (err != FV_OK) break;
        const int32_t first = chunk * per_chunk, count = std::min(per_chunk, c.T - first);
        for (int32_t t = 0; t < count; ++t) {
            z.h_ptr[t] = din[first + t];
            z.h_ptr[count + t] = dout[first + t];
        }
        bool ok = hipMemcpyAsync(z.d_ptr, z.h_ptr, 2 * sizeof(double *) * count, hipMemcpyHostToDevice, z.stream) ==
                  hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(gather_patches, dim3((unsigned)count), dim3(256), 0, z.stream, z.d_ptr, z.d_in, z.d_out,
                               c.pd);
            ok = hipGetLastError() == hipSuccess;
        }
        if (ok) {
            st = plain_update(z.d_in, z.d_out, c.sizes + first, nullptr, count, c.dim, c.nq, c.dt, c.h, c.gamma,
                              c.flags, c.lambda_out ? z.d_lam : nullptr, z.stream, uniform, nullptr);
            ok = st == FV_OK;
        }
        if (ok) {
            hipLaunchKernelGGL(scatter_patches, dim3((unsigned)count), dim3(256), 0, z.stream, z.d_out,
                               const_cast<double *const *>(z.d_ptr + count), c.pd);
            ok = hipGetLastError() == hipSuccess;
        }
        if (ok && c.lambda_out)
            ok = hipMemcpyAsync(z.h_lam, z.d_lam, sizeof(double) * count, hipMemcpyDeviceToHost, z.stream) ==
                 hipSuccess;
        if (ok) ok = hipEventRecord(z.done, z.stream) == hipSuccess;
        if (!ok) {
            err = st != FV_OK ? st : fail(FV_ERR_LAUNCH, "zero-copy chunk at patch %d failed", first);
            (void)hipStreamSynchronize(z.stream);
            (void)hipGetLastError();
            break;
        }
        z.first = first;
        z.count = count;
    }
    // every chunk in flight is waited for, also after an error
    for (auto &z : x.zchunks.slots) {
        if (err == FV_OK) {
            retire(z);
        } else if (z.count) {
            (void)hipStreamSynchronize(z.stream);
            z.count = 0;
        }
    }
    if (err != FV_OK) return err;
    if (stats) {
        const int64_t n = (int64_t)c.T * (int64_t)c.pbytes;
        stats->bytes_to_device = n;
        stats->bytes_to_host = n + (c.lambda_out ? 8ll * c.T : 0);
        stats->host_copy_seconds = 0.0;
    }
    return FV_OK;
}

}  // namespace
}  // namespace fv

using namespace fv;

extern "C" fv_status fv_host_alloc(size_t bytes, void **ptr) {
    clear_error();
    if (!ptr) return fail(FV_ERR_INVALID_ARG, "ptr must be non-null");
    *ptr = nullptr;
    if (bytes == 0) return fail(FV_ERR_INVALID_ARG, "bytes must be > 0");
    DeviceContext *ctx = nullptr;
    fv_status st = current_context(&ctx);
    if (st != FV_OK) return st;
    void *h = nullptr;
    if (hipHostMalloc(&h, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FV_ERR_OOM, "pinned allocation of %zu bytes", bytes);
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return fail(FV_ERR_LAUNCH, "no device address for pinned memory");
    }
    {
        std::lock_guard<std::mutex> g(g_pin_mu);
        pinned_blocks()[reinterpret_cast<uintptr_t>(h)] = PinnedBlock{bytes, static_cast<double *>(d)};
    }
    *ptr = h;
    return FV_OK;
}

extern "C" fv_status fv_host_free(void *ptr) {
    clear_error();
    if (!ptr) return FV_OK;
    {
        std::lock_guard<std::mutex> g(g_pin_mu);
        auto it = pinned_blocks().find(reinterpret_cast<uintptr_t>(ptr));
        if (it == pinned_blocks().end()) return fail(FV_ERR_INVALID_ARG, "pointer was not returned by fv_host_alloc");
        pinned_blocks().erase(it);
    }
    if (hipHostFree(ptr) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FV_ERR_LAUNCH, "hipHostFree failed");
    }
    return FV_OK;
}

extern "C" fv_status fv_host_patches_update(const double *const *patches_in, double *const *patches_out,
                                            const int32_t *sizes, int32_t num_patches, int32_t dim, int32_t unknowns,
                                            double dt, double h, double gamma, uint32_t flags, double *lambda_out,
                                            const fv_transfer_config *config, fv_transfer_stats *stats) {
    clear_error();
    const double t_start = now_s();
    if (stats) *stats = fv_transfer_stats{0, 0, 0.0, 0.0};
    fv_status st = check_scalars(dim, unknowns, dt, h, gamma, flags);
    if (st != FV_OK) return st;
    if (num_patches < 0) return fail(FV_ERR_INVALID_ARG, "num_patches must be >= 0");
    fv_transfer_config cfg{kDefaultChunk, kDefaultSlots, kDefaultThreads, FV_TRANSFER_PIPELINED, 0};
    if (config) {
        cfg = *config;
        // zero copy moves larger chunks on more streams (no host copies to overlap with)
        const bool zc = cfg.mode == FV_TRANSFER_ZERO_COPY;
        if (cfg.chunk_bytes == 0) cfg.chunk_bytes = zc ? kZeroCopyChunk : kDefaultChunk;
        if (cfg.slots == 0) cfg.slots = zc ? kZeroCopySlots : kDefaultSlots;
        if (cfg.host_threads == 0) cfg.host_threads = kDefaultThreads;
    }
    if (cfg.mode != FV_TRANSFER_PIPELINED && cfg.mode != FV_TRANSFER_PER_PATCH && cfg.mode != FV_TRANSFER_STAGED &&
        cfg.mode != FV_TRANSFER_ZERO_COPY)
        return fail(FV_ERR_INVALID_ARG, "unknown transfer mode %d", cfg.mode);
    if (cfg.slots < 1 || cfg.slots > FV_TRANSFER_MAX_SLOTS)
        return fail(FV_ERR_INVALID_ARG, "slots must be in [1, %d]", FV_TRANSFER_MAX_SLOTS);
    if (cfg.host_threads < 1 || cfg.host_threads > FV_TRANSFER_MAX_THREADS)
        return fail(FV_ERR_INVALID_ARG, "host_threads must be in [1, %d]", FV_TRANSFER_MAX_THREADS);
    if (cfg.chunk_bytes < 0) return fail(FV_ERR_INVALID_ARG, "chunk_bytes must be >= 0");
    if (num_patches == 0) return FV_OK;
    if (!patches_in || !patches_out || !sizes)
        return fail(FV_ERR_INVALID_ARG, "patches_in, patches_out and sizes must be non-null");
    const int32_t p = sizes[0];
    if (p < 1 || p > max_p(dim)) return fail(FV_ERR_INVALID_ARG, "p=%d outside [1, %d] for %dD", p, max_p(dim), dim);
    for (int32_t t = 0; t < num_patches; ++t) {
        if (sizes[t] != p)
            return fail(FV_ERR_UNSUPPORTED, "patch %d has size %d, patch 0 %d: one size per call", t, sizes[t], p);
        if (!patches_in[t] || !patches_out[t]) return fail(FV_ERR_INVALID_ARG, "patch %d has a null pointer", t);
        if ((reinterpret_cast<uintptr_t>(patches_in[t]) | reinterpret_cast<uintptr_t>(patches_out[t])) & 7u)
            return fail(FV_ERR_INVALID_ARG, "patch %d is not 8-byte aligned", t);
    }
    const int64_t pd = patch_doubles(p, dim, unknowns);
    const size_t pbytes = sizeof(double) * (size_t)pd;
    // no output patch may overlap an input patch or another output patch (all patches have
    // one length, so it is enough to compare neighbours in address order)
    {
        std::vector<std::pair<uintptr_t, int>> starts;
        starts.reserve(2 * (size_t)num_patches);
        for (int32_t t = 0; t < num_patches; ++t) {
            starts.emplace_back(reinterpret_cast<uintptr_t>(patches_in[t]), 0);
            starts.emplace_back(reinterpret_cast<uintptr_t>(patches_out[t]), 1);
        }
        std::sort(starts.begin(), starts.end());
        for (size_t k = 1; k < starts.size(); ++k)
            if ((starts[k].second == 1 || starts[k - 1].second == 1) && starts[k].first - starts[k - 1].first < pbytes)
                return fail(FV_ERR_OVERLAP, "an output patch overlaps another patch");
    }
    // zero copy: every patch must lie in memory from fv_host_alloc (the kernels dereference it)
    std::vector<const double *> zin, zout;
    if (cfg.mode == FV_TRANSFER_ZERO_COPY) {
        zin.resize(num_patches);
        zout.resize(num_patches);
        for (int32_t t = 0; t < num_patches; ++t) {
            zin[t] = pinned_device(patches_in[t], pbytes);
            zout[t] = pinned_device(patches_out[t], pbytes);
            if (!zin[t] || !zout[t])
                return fail(FV_ERR_INVALID_ARG, "patch %d does not lie in memory from fv_host_alloc", t);
        }
    }
    if ((cfg.mode == FV_TRANSFER_PIPELINED || cfg.mode == FV_TRANSFER_ZERO_COPY) && cfg.chunk_bytes < (int64_t)pbytes)
        return fail(FV_ERR_INVALID_ARG, "chunk_bytes below one patch (%zu bytes)", pbytes);
    DeviceContext *ctx = nullptr;
    st = current_context(&ctx);
    if (st != FV_OK) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FV_ERR_NO_DEVICE, "no current device");
    Transfer *x = transfer_for(dev);
    std::lock_guard<std::mutex> g(x->mu);
    const Call c{patches_in, patches_out, sizes, num_patches, p, dim, unknowns, dt, h, gamma, flags, lambda_out,
                 pd, pbytes};
    switch (cfg.mode) {
        case FV_TRANSFER_PER_PATCH: st = per_patch(*x, c, stats); break;
        case FV_TRANSFER_STAGED: st = staged(*x, c, cfg.host_threads, stats); break;
        case FV_TRANSFER_ZERO_COPY: st = zero_copy(*x, c, cfg, zin, zout, stats); break;
        default: st = pipelined(*x, c, cfg, dev, stats); break;
    }
    if (st == FV_OK && stats) stats->seconds = now_s() - t_start;
    return st;
}
