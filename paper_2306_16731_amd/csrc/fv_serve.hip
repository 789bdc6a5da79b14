// fv_serve.hip -- serving form: a request loop over device-resident patch state.
//
// A traversal of an adaptive mesh hands the kernel batches of patches as it
// goes (task fusion of enclave tasks, Sec. 2.1); the paper's measurements are
// dominated by moving those patches host <-> device and by allocating device
// memory per kernel call, which it replaces by recycled ("managed") device
// memory (Sec. 4, "Data transfer").  Here the patch state never leaves the
// device: every registered mesh keeps two state slots per patch in HBM, each
// patch ping-pongs between them on its own (a per-patch parity), and a batch
// names a range of a mesh's patches.  Batches are admitted in arrival order
// while the resident state plus the batches in flight fit an HBM byte budget
// (otherwise they wait; none is dropped), launched on the server's stream,
// and retired when their completion event has fired, which records the
// arrival-to-completion latency.
//
// Two launch modes: FV_SERVE_FUSED builds the batch's task list (one wave per
// task, tasks in memory order) in pinned staging memory, which the kernel reads
// in place, and runs the whole batch in one fused launch; FV_SERVE_PLAIN runs each batch through the plain per-batch
// path (validation, grouping by size, one launch per size class).
//
// Meshes of different dimensions (a 2D mesh of mixed patch sizes next to a 3D
// one) share one server, one stream and one budget.  Failures: a batch whose
// completion event reports an error (anything but "not ready") is re-run from
// its input slot, which no update overwrites, into its output slot again, up
// to max_retries times, unless a later batch in flight has already used its
// output; then, or when the retries are spent, poll / drain / run_trace
// return FV_ERR_LAUNCH with the detail.  A batch still running deadline_ms
// after its launch also makes them return FV_ERR_LAUNCH instead of waiting on.
// fv_server_inject forces either outcome from the host for tests: the batch
// runs normally and only its completion check is overridden.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "fvpatch.h"
#include "fv_host.h"
#include "fv_internal.h"

namespace {

using clock_type = std::chrono::steady_clock;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(clock_type::now().time_since_epoch()).count();
}

struct Mesh {
    int32_t dim = 2, nq = 5;
    double h = 1.0;
    std::vector<int32_t> sizes;
    std::vector<int64_t> off;   // offset of each patch inside one slot (doubles)
    std::vector<uint8_t> cur;   // slot holding each patch's current state
    int64_t slot_doubles = 0;
    double *buf = nullptr;      // two slots: [0, slot_doubles) and [slot_doubles, 2 slot_doubles)
};

struct Request {
    int64_t ticket = 0;
    int32_t mesh = 0, first = 0, count = 0;
    int32_t retries = 0;  // re-runs after failed completions so far
    double dt = 0.0;
    int64_t arrival_ns = 0;
};

// A test hook's override of a batch's completion check.
struct Injection {
    int32_t kind = 0;   // FV_INJECT_FAIL or FV_INJECT_HANG
    int32_t times = 0;  // FV_INJECT_FAIL: completion checks still to report a failure
};

// Pinned staging of one in-flight batch's descriptors, which its kernels read in place over the
// bus (no copy to device memory first), and its lambda (recycled, never freed while the server lives).
struct Staging {
    void *host = nullptr;
    void *host_dev = nullptr;  // the device's address of `host`
    size_t cap = 0;
    double *lambda = nullptr;  // device [cap_patches]
    int32_t cap_patches = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
};

struct Inflight {
    Request req;
    int staging = -1;
    int64_t bytes = 0;
    int64_t cells = 0;
    int64_t launch_ns = 0;
    hipEvent_t done = nullptr;  // event recorded after the batch's launches
};

}  // namespace

struct fv_server {
    fv_server_config cfg{};
    int device = -1;
    hipStream_t stream = nullptr;
    int64_t resident_bytes = 0;
    int64_t inflight_bytes = 0;
    std::vector<Mesh> meshes;
    std::deque<Request> queue;
    std::deque<Inflight> inflight;
    std::vector<Staging> staging;
    std::vector<hipEvent_t> spare_events;
    std::vector<double> latency_ms;
    std::vector<fv_batch_record> log;  // one record per completed batch
    std::map<int64_t, Injection> inject;
    int64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, cells_updated = 0, peak_queue = 0, peak_inflight = 0;
    int64_t failed = 0, retried = 0;
    int64_t first_arrival_ns = -1, last_completion_ns = -1;
    int64_t t0_ns = 0;  // creation time: origin of the batch log's times
};

namespace fv {
namespace {

int64_t batch_bytes(const Request &r) {
    // the batch's working set, counted against the budget: its descriptors (in and out offsets, ids,
    // tasks; in pinned staging) and its lambda
    return (int64_t)r.count * (8 + 8 + 4 + 16 + 8);
}

fv_status ensure_staging(fv_server *s, Staging &st, int32_t count) {
    const size_t need = (size_t)count * (8 + 8 + 4 + sizeof(WaveTask)) + 16;
    if (st.cap >= need && st.cap_patches >= count) return FV_OK;
    if (st.busy) return fail(FV_ERR_LAUNCH, "staging buffer in use");
    if (st.host) (void)hipHostFree(st.host);
    if (st.lambda) (void)hipFree(st.lambda);
    st.host = st.host_dev = nullptr;
    st.lambda = nullptr;
    st.cap = 0;
    st.cap_patches = 0;
    const int32_t cp = std::max<int32_t>(count, 4096);
    const size_t cap = (size_t)cp * (8 + 8 + 4 + sizeof(WaveTask)) + 16;  // + padding before the task list
    if (hipHostMalloc(&st.host, cap, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&st.lambda, sizeof(double) * cp) != hipSuccess)
        return fail(FV_ERR_OOM, "staging allocation failed");
    if (hipHostGetDevicePointer(&st.host_dev, st.host, 0) != hipSuccess || !st.host_dev)
        return fail(FV_ERR_LAUNCH, "no device address for the pinned staging");
    st.cap = cap;
    st.cap_patches = cp;
    (void)s;
    return FV_OK;
}

// Launch one batch (fused mode): task list of the wave kernel for 2D p <= 62,
// per-class launches otherwise.  Descriptors go through the staging buffer.
fv_status launch_fused(fv_server *s, Mesh &m, const Request &r, Staging &st) {
    const int dim = m.dim, nq = m.nq;
    const int pmax = max_p(dim);
    const int32_t n = r.count;
    int64_t *hin = static_cast<int64_t *>(st.host);
    int64_t *hout = hin + n;
    int32_t *hid = reinterpret_cast<int32_t *>(hout + n);
    WaveTask *htask = reinterpret_cast<WaveTask *>(hid + n + (n & 1));
    // counting sort by size, largest first
    int32_t count[FV_MAX_P_2D + 1] = {0};
    for (int32_t k = 0; k < n; ++k) count[m.sizes[r.first + k]]++;
    int32_t start[FV_MAX_P_2D + 2] = {0};
    int32_t cursor = 0;
    for (int p = pmax; p >= 1; --p) {
        start[p] = cursor;
        cursor += count[p];
    }
    int32_t fill[FV_MAX_P_2D + 2];
    std::memcpy(fill, start, sizeof(fill));
    bool even = true, odd_rows_only = true;
    bool odd_offset[FV_MAX_P_2D + 1] = {false};  // per size: some entry starts at an odd double
    const bool whole_rows = (s->cfg.flags & (FV_HALO_PERIODIC | FV_HALO_FROM_IN)) != 0;  // of the fused launch
    for (int32_t k = 0; k < n; ++k) {
        const int32_t t = r.first + k;
        const int32_t j = fill[m.sizes[t]]++;
        const int64_t base_in = m.cur[t] ? m.slot_doubles : 0;
        const int64_t base_out = m.cur[t] ? 0 : m.slot_doubles;
        hin[j] = base_in + m.off[t];
        hout[j] = base_out + m.off[t];
        hid[j] = k;
        if ((hin[j] | hout[j]) & 1) {
            even = false;
            odd_offset[m.sizes[t]] = true;
        }
    }
    int32_t ntask = 0, ring_words = 0, prefetch = 0;
    int64_t best_cells = -1;
    struct Cls { int p, first, count; bool even; };  // even: 16-byte bursts (even offsets and patch length)
    std::vector<Cls> classes;
    for (int p = pmax; p >= 1; --p) {
        if (!count[p]) continue;
        if (dim == 2 && wave2d_fits(p)) {
            const fv_tuning tu = tuning_for(dim, nq, p);
            // rows == 0: the fixed-size form of the kernel, which a class built in that form
            // always runs here (as in a plan's fused launch)
            const bool fixed = tu.kernel == FV_KERNEL_FIXED || wave2d_fixed(p, nq);
            const int rows = fixed ? 0 : (tu.kernel == FV_KERNEL_WAVE && tu.rows > 0 ? tu.rows : 6);
            const int ppw = 64 / (p + 2);
            for (int32_t f = 0; f < count[p]; f += ppw)
                htask[ntask++] = WaveTask{p, rows, start[p] + f, std::min<int32_t>(ppw, count[p] - f)};
            ring_words = std::max(ring_words, fixed ? wave2d_fixed_ring_words(p, whole_rows) : wave2d_ring_words(p, nq, rows));
            if ((int64_t)count[p] * p * p > best_cells) {
                best_cells = (int64_t)count[p] * p * p;
                prefetch = (tu.kernel == FV_KERNEL_WAVE || tu.kernel == FV_KERNEL_FIXED) ? tu.prefetch : 0;
            }
            if (((p + 2) * nq) % 2) even = false;
            if (!(fixed && fixed_odd_rows(dim, p, nq))) odd_rows_only = false;
        } else {
            classes.push_back(Cls{p, start[p], count[p], !odd_offset[p] && patch_doubles(p, dim, nq) % 2 == 0});
        }
    }
    // one wave per task: tasks in memory order keep the resident waves on neighbouring patches
    std::stable_sort(htask, htask + ntask,
                     [&](const WaveTask &a, const WaveTask &b) { return hin[a.first] < hin[b.first]; });
    // the kernels read the descriptors in place: the staging stays untouched until the batch retires
    const int64_t *din = static_cast<const int64_t *>(st.host_dev);
    const int64_t *dout = din + n;
    const int32_t *did = reinterpret_cast<const int32_t *>(dout + n);
    const WaveTask *dtask = reinterpret_cast<const WaveTask *>(did + n + (n & 1));
    const double r_host = r.dt / m.h;
    if (ntask > 0) {
        TaskLaunch T;
        T.in = m.buf;
        T.out = m.buf;
        T.offsets = din;
        T.out_offsets = dout;
        T.ids = did;
        T.tasks = dtask;
        T.num_tasks = ntask;
        T.nq = nq;
        T.ring_words = ring_words;
        T.prefetch = prefetch;
        T.vec2 = (even || odd_rows_only) && ((reinterpret_cast<uintptr_t>(m.buf) & 15u) == 0);
        T.persistent = false;
        T.r = r_host;
        T.gamma = s->cfg.gamma;
        T.flags = s->cfg.flags;
        T.lambda_out = st.lambda;
        hipError_t e = launch_update2d_tasks(T, s->stream);
        if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "fused launch failed: %s", hipGetErrorString(e));
    }
    for (const auto &c : classes) {
        UpdateLaunch L;
        L.in = m.buf;
        L.out = m.buf;
        L.offsets = din + c.first;
        L.out_offsets = dout + c.first;
        L.ids = did + c.first;
        L.num_items = c.count;
        L.p = c.p;
        L.dim = dim;
        L.nq = nq;
        L.r = r_host;
        L.gamma = s->cfg.gamma;
        L.flags = s->cfg.flags;
        L.lambda_out = st.lambda;
        L.vec2 = c.even && ((reinterpret_cast<uintptr_t>(m.buf) & 15u) == 0);
        apply_tuning(L);
        if (L.kernel == FV_KERNEL_WAVE) L.kernel = FV_KERNEL_BLOCK;
        if (L.kernel == FV_KERNEL_TILE) L.vec2 = false;
        hipError_t e = launch_update(L, s->stream);
        if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "class launch failed: %s", hipGetErrorString(e));
    }
    return FV_OK;
}

// Launch one batch through the plain per-batch path.
fv_status launch_plain(fv_server *s, Mesh &m, const Request &r, Staging &st) {
    const int32_t n = r.count;
    std::vector<int64_t> in_off(n), out_off(n);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t t = r.first + k;
        in_off[k] = (m.cur[t] ? m.slot_doubles : 0) + m.off[t];
        out_off[k] = (m.cur[t] ? 0 : m.slot_doubles) + m.off[t];
    }
    BatchShape shape;
    fv_status stt = check_layout(m.sizes.data() + r.first, in_off.data(), n, m.dim, m.nq, &shape);
    if (stt != FV_OK) return stt;
    return plain_update(m.buf, m.buf, m.sizes.data() + r.first, in_off.data(), n, m.dim, m.nq, r.dt, m.h,
                        s->cfg.gamma, s->cfg.flags, st.lambda, s->stream, shape, out_off.data());
}

hipEvent_t take_event(fv_server *s) {
    if (!s->spare_events.empty()) {
        hipEvent_t e = s->spare_events.back();
        s->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

enum class Check { Done, Pending, Failed };

// The completion check of an in-flight batch: its event's status, overridden by
// a test injection (a forced failure is reported only once the batch has run).
Check check_done(fv_server *s, const Inflight &f, hipError_t *err) {
    hipError_t e = hipEventQuery(f.done);
    auto it = s->inject.find(f.req.ticket);
    if (it != s->inject.end()) {
        if (it->second.kind == FV_INJECT_HANG) return Check::Pending;
        if (it->second.kind == FV_INJECT_FAIL && it->second.times > 0 && e == hipSuccess) {
            if (--it->second.times == 0) s->inject.erase(it);
            e = hipErrorLaunchFailure;
        }
    }
    *err = e;
    if (e == hipSuccess) return Check::Done;
    if (e == hipErrorNotReady) return Check::Pending;
    return Check::Failed;
}

void restore_parity(fv_server *s, const Request &r) {
    Mesh &m = s->meshes[r.mesh];
    for (int32_t k = 0; k < r.count; ++k) m.cur[r.first + k] ^= 1u;
}

void release_inflight(fv_server *s, Inflight &f) {
    s->inflight_bytes -= f.bytes;
    s->staging[f.staging].busy = false;
    s->spare_events.push_back(f.done);
}

// The oldest in-flight batch reported an error.  Its input slot still holds the
// patches' state from before it unless a later batch in flight on the same
// patches has read its output and written that slot: then the batch is lost.
// Otherwise its patches are set back to that state and it is queued first again
// (a re-run writes its output slot anew), or, with its retries spent, dropped.
fv_status handle_failure(fv_server *s, hipError_t e) {
    Inflight f = s->inflight.front();
    const Request &r = f.req;
    for (size_t k = 1; k < s->inflight.size(); ++k) {
        const Request &g = s->inflight[k].req;
        if (g.mesh == r.mesh && g.first < r.first + r.count && r.first < g.first + g.count) {
            release_inflight(s, f);
            s->inflight.pop_front();
            s->failed++;
            return fail(FV_ERR_LAUNCH,
                        "batch %lld (mesh %d, patches [%d, %d)) failed (%s) after batch %lld had used its output: "
                        "the state of those patches is lost",
                        (long long)r.ticket, r.mesh, r.first, r.first + r.count, hipGetErrorString(e),
                        (long long)g.ticket);
        }
    }
    restore_parity(s, r);
    release_inflight(s, f);
    s->inflight.pop_front();
    if (r.retries >= s->cfg.max_retries) {
        s->failed++;
        return fail(FV_ERR_LAUNCH,
                    "batch %lld (mesh %d, patches [%d, %d)) failed (%s) after %d re-runs; its patches keep their "
                    "state from before it",
                    (long long)r.ticket, r.mesh, r.first, r.first + r.count, hipGetErrorString(e), r.retries);
    }
    Request again = r;
    again.retries++;
    s->retried++;
    s->queue.push_front(again);
    return FV_OK;
}

// Retire finished batches in order, recording their latency.  wait: keep
// checking the oldest batch until it finishes (or its deadline passes).
fv_status retire(fv_server *s, bool wait) {
    while (!s->inflight.empty()) {
        Inflight &f = s->inflight.front();
        hipError_t e = hipSuccess;
        const Check c = check_done(s, f, &e);
        if (c == Check::Pending) {
            const int64_t t = now_ns();
            if (s->cfg.deadline_ms > 0.0 && (double)(t - f.launch_ns) * 1e-6 > s->cfg.deadline_ms)
                return fail(FV_ERR_LAUNCH, "batch %lld still running %.3f ms after its launch (deadline %.3f ms)",
                            (long long)f.req.ticket, (double)(t - f.launch_ns) * 1e-6, s->cfg.deadline_ms);
            if (!wait) break;
            std::this_thread::yield();
            continue;
        }
        if (c == Check::Failed) {
            const fv_status st = handle_failure(s, e);
            if (st != FV_OK) return st;
            continue;
        }
        const int64_t t = now_ns();
        s->latency_ms.push_back((double)(t - f.req.arrival_ns) * 1e-6);
        fv_batch_record rec;
        rec.ticket = f.req.ticket;
        rec.arrival_ns = f.req.arrival_ns - s->t0_ns;
        rec.launch_ns = f.launch_ns - s->t0_ns;
        rec.done_ns = t - s->t0_ns;
        rec.cells = f.cells;
        rec.mesh = f.req.mesh;
        rec.count = f.req.count;
        rec.retries = f.req.retries;
        rec.reserved = 0;
        s->log.push_back(rec);
        s->completed++;
        s->cells_updated += f.cells;
        s->last_completion_ns = t;
        release_inflight(s, f);
        s->inflight.pop_front();
    }
    return FV_OK;
}

// Admit queued batches while the budget and the in-flight limit allow.
fv_status admit(fv_server *s) {
    while (!s->queue.empty()) {
        const Request &r = s->queue.front();
        const int64_t b = batch_bytes(r);
        if ((int64_t)s->inflight.size() >= s->cfg.max_inflight) break;
        if (s->resident_bytes + s->inflight_bytes + b > s->cfg.budget_bytes) {
            if (s->inflight.empty())
                return fail(FV_ERR_BUDGET, "batch of %d patches does not fit the budget even alone", r.count);
            break;
        }
        int si = -1;
        for (int k = 0; k < (int)s->staging.size(); ++k)
            if (!s->staging[k].busy) {
                si = k;
                break;
            }
        if (si < 0) break;
        Staging &st = s->staging[si];
        fv_status e = ensure_staging(s, st, r.count);
        if (e != FV_OK) return e;
        Mesh &m = s->meshes[r.mesh];
        e = (s->cfg.mode == FV_SERVE_PLAIN) ? launch_plain(s, m, r, st) : launch_fused(s, m, r, st);
        if (e != FV_OK) return e;
        Inflight f;
        f.req = r;
        f.staging = si;
        f.bytes = b;
        f.launch_ns = now_ns();
        f.done = take_event(s);
        if (!f.done || hipEventRecord(f.done, s->stream) != hipSuccess) return fail(FV_ERR_LAUNCH, "event record failed");
        for (int32_t k = 0; k < r.count; ++k) {
            const int32_t t = r.first + k;
            m.cur[t] ^= 1u;
            f.cells += (int64_t)std::pow(m.sizes[t], m.dim);
        }
        st.busy = true;
        s->inflight_bytes += b;
        s->inflight.push_back(f);
        s->peak_inflight = std::max<int64_t>(s->peak_inflight, (int64_t)s->inflight.size());
        s->queue.pop_front();
    }
    return FV_OK;
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

void fill_stats(const fv_server *s, fv_server_stats *out) {
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->queued = (int64_t)s->queue.size();
    out->inflight = (int64_t)s->inflight.size();
    out->peak_queued = s->peak_queue;
    out->peak_inflight = s->peak_inflight;
    out->cells_updated = s->cells_updated;
    out->failed = s->failed;
    out->retried = s->retried;
    out->resident_bytes = s->resident_bytes;
    out->budget_bytes = s->cfg.budget_bytes;
    out->p50_ms = percentile(s->latency_ms, 0.50);
    out->p99_ms = percentile(s->latency_ms, 0.99);
    out->max_ms = s->latency_ms.empty() ? 0.0 : *std::max_element(s->latency_ms.begin(), s->latency_ms.end());
    double sum = 0.0;
    for (double x : s->latency_ms) sum += x;
    out->mean_ms = s->latency_ms.empty() ? 0.0 : sum / (double)s->latency_ms.size();
    if (s->first_arrival_ns >= 0 && s->last_completion_ns > s->first_arrival_ns)
        out->cell_updates_per_s = (double)s->cells_updated / ((double)(s->last_completion_ns - s->first_arrival_ns) * 1e-9);
}

fv_status check_server(fv_server *s) {
    if (!s) return fail(FV_ERR_INVALID_ARG, "server must be non-null");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != s->device)
        return fail(FV_ERR_INVALID_ARG, "server was created on device %d, current is %d", s->device, dev);
    return FV_OK;
}

}  // namespace
}  // namespace fv

using namespace fv;

extern "C" {

fv_status fv_server_create(fv_server **server, const fv_server_config *cfg) {
    clear_error();
    if (!server || !cfg) return fail(FV_ERR_INVALID_ARG, "server and cfg must be non-null");
    *server = nullptr;
    fv_status st = check_scalars(2, 5, 1.0, 1.0, cfg->gamma, cfg->flags);
    if (st != FV_OK) return st;
    if (cfg->budget_bytes <= 0) return fail(FV_ERR_INVALID_ARG, "budget_bytes must be > 0");
    if (cfg->mode != FV_SERVE_FUSED && cfg->mode != FV_SERVE_PLAIN) return fail(FV_ERR_INVALID_ARG, "unknown mode %d", cfg->mode);
    if (cfg->max_inflight < 0 || cfg->max_inflight > 1024) return fail(FV_ERR_INVALID_ARG, "max_inflight must be in [0, 1024]");
    if (cfg->max_retries < 0 || cfg->max_retries > 16) return fail(FV_ERR_INVALID_ARG, "max_retries must be in [0, 16]");
    if (!std::isfinite(cfg->deadline_ms) || cfg->deadline_ms < 0.0)
        return fail(FV_ERR_INVALID_ARG, "deadline_ms must be finite and >= 0");
    DeviceContext *ctx = nullptr;
    if ((st = current_context(&ctx)) != FV_OK) return st;
    auto *s = new fv_server();
    s->cfg = *cfg;
    if (s->cfg.max_inflight == 0) s->cfg.max_inflight = 8;
    hipGetDevice(&s->device);
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return fail(FV_ERR_LAUNCH, "stream creation failed");
    }
    s->staging.resize(s->cfg.max_inflight);
    s->t0_ns = now_ns();
    *server = s;
    return FV_OK;
}

fv_status fv_server_add_mesh(fv_server *s, int32_t dim, int32_t unknowns, double h, const int32_t *sizes,
                             int32_t num_patches, const double *host_state, int32_t *mesh_id) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    if ((st = check_scalars(dim, unknowns, 1.0, h, s->cfg.gamma, 0)) != FV_OK) return st;
    if (!sizes || !host_state || !mesh_id || num_patches < 1)
        return fail(FV_ERR_INVALID_ARG, "sizes, host_state, mesh_id and num_patches >= 1 are required");
    Mesh m;
    m.dim = dim;
    m.nq = unknowns;
    m.h = h;
    m.sizes.assign(sizes, sizes + num_patches);
    m.off.resize(num_patches);
    m.cur.assign(num_patches, 0);
    int64_t o = 0;
    const int pmax = max_p(dim);
    for (int32_t t = 0; t < num_patches; ++t) {
        if (sizes[t] < 1 || sizes[t] > pmax) return fail(FV_ERR_INVALID_ARG, "sizes[%d]=%d outside [1, %d]", t, sizes[t], pmax);
        m.off[t] = o;
        o += patch_doubles(sizes[t], dim, unknowns);
    }
    m.slot_doubles = o + (o & 1);  // keep the second slot 16-byte aligned
    const int64_t bytes = 2 * m.slot_doubles * (int64_t)sizeof(double);
    if (s->resident_bytes + s->inflight_bytes + bytes > s->cfg.budget_bytes)
        return fail(FV_ERR_BUDGET, "mesh of %lld bytes does not fit the budget (%lld resident of %lld)", (long long)bytes,
                    (long long)s->resident_bytes, (long long)s->cfg.budget_bytes);
    if (hipMalloc(&m.buf, bytes) != hipSuccess) return fail(FV_ERR_OOM, "device allocation of %lld bytes failed", (long long)bytes);
    // both slots start from the given state (halo volumes included)
    if (hipMemcpy(m.buf, host_state, o * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m.buf + m.slot_doubles, host_state, o * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m.buf);
        return fail(FV_ERR_LAUNCH, "upload of the mesh failed");
    }
    s->resident_bytes += bytes;
    s->meshes.push_back(std::move(m));
    *mesh_id = (int32_t)s->meshes.size() - 1;
    return FV_OK;
}

fv_status fv_server_submit(fv_server *s, int32_t mesh_id, int32_t first, int32_t count, double dt, int64_t arrival_ns,
                           int64_t *ticket) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    if (mesh_id < 0 || mesh_id >= (int32_t)s->meshes.size()) return fail(FV_ERR_INVALID_ARG, "unknown mesh %d", mesh_id);
    const Mesh &m = s->meshes[mesh_id];
    if (count < 1 || first < 0 || (int64_t)first + count > (int64_t)m.sizes.size())
        return fail(FV_ERR_INVALID_ARG, "range [%d, %d) outside the mesh of %zu patches", first, first + count, m.sizes.size());
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(FV_ERR_INVALID_ARG, "dt must be finite and > 0");
    Request r;
    r.ticket = s->next_ticket++;
    r.mesh = mesh_id;
    r.first = first;
    r.count = count;
    r.dt = dt;
    r.arrival_ns = arrival_ns > 0 ? arrival_ns : now_ns();
    if (s->first_arrival_ns < 0 || r.arrival_ns < s->first_arrival_ns) s->first_arrival_ns = r.arrival_ns;
    s->queue.push_back(r);
    s->submitted++;
    s->peak_queue = std::max<int64_t>(s->peak_queue, (int64_t)s->queue.size());
    if (ticket) *ticket = r.ticket;
    return FV_OK;
}

fv_status fv_server_poll(fv_server *s, fv_server_stats *stats) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    st = retire(s, false);
    if (st == FV_OK) st = admit(s);
    fill_stats(s, stats);
    return st;
}

fv_status fv_server_drain(fv_server *s, fv_server_stats *stats) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    while (!s->queue.empty() || !s->inflight.empty()) {
        if ((st = admit(s)) != FV_OK) return st;  // FV_ERR_BUDGET if a batch can never fit
        if ((st = retire(s, true)) != FV_OK) {
            fill_stats(s, stats);
            return st;
        }
    }
    fill_stats(s, stats);
    return FV_OK;
}

fv_status fv_server_run_trace(fv_server *s, const fv_serve_request *reqs, int64_t n, fv_server_stats *stats) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    if (!reqs || n < 0) return fail(FV_ERR_INVALID_ARG, "reqs must be non-null");
    for (int64_t k = 1; k < n; ++k)
        if (reqs[k].arrival_ns < reqs[k - 1].arrival_ns) return fail(FV_ERR_INVALID_ARG, "arrivals must be non-decreasing");
    const int64_t t0 = now_ns();
    for (int64_t k = 0; k < n; ++k) {
        const int64_t due = t0 + reqs[k].arrival_ns;
        while (now_ns() < due) {
            if ((st = retire(s, false)) != FV_OK || (st = admit(s)) != FV_OK) {
                fill_stats(s, stats);
                return st;
            }
        }
        st = fv_server_submit(s, reqs[k].mesh, reqs[k].first, reqs[k].count, reqs[k].dt, due, nullptr);
        if (st != FV_OK) return st;
        if ((st = retire(s, false)) != FV_OK || (st = admit(s)) != FV_OK) {
            fill_stats(s, stats);
            return st;
        }
    }
    return fv_server_drain(s, stats);
}

fv_status fv_server_read_mesh(fv_server *s, int32_t mesh_id, double *host_state) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    if (mesh_id < 0 || mesh_id >= (int32_t)s->meshes.size() || !host_state) return fail(FV_ERR_INVALID_ARG, "bad mesh or buffer");
    if ((st = fv_server_drain(s, nullptr)) != FV_OK) return st;
    const Mesh &m = s->meshes[mesh_id];
    for (size_t t = 0; t < m.sizes.size(); ++t) {
        const int64_t n = patch_doubles(m.sizes[t], m.dim, m.nq);
        const double *src = m.buf + (m.cur[t] ? m.slot_doubles : 0) + m.off[t];
        if (hipMemcpyAsync(host_state + m.off[t], src, n * sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess)
            return fail(FV_ERR_LAUNCH, "read-back failed");
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(FV_ERR_LAUNCH, "read-back failed");
    return FV_OK;
}

fv_status fv_server_inject(fv_server *s, int64_t ticket, int32_t kind, int32_t times) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    if (ticket < 1) return fail(FV_ERR_INVALID_ARG, "tickets start at 1");
    if (kind == 0) {
        s->inject.erase(ticket);
        return FV_OK;
    }
    if (kind != FV_INJECT_FAIL && kind != FV_INJECT_HANG) return fail(FV_ERR_INVALID_ARG, "unknown injection %d", kind);
    if (kind == FV_INJECT_FAIL && times < 1) return fail(FV_ERR_INVALID_ARG, "times must be >= 1");
    s->inject[ticket] = Injection{kind, times};
    return FV_OK;
}

fv_status fv_server_batch_log(fv_server *s, fv_batch_record *records, int64_t capacity, int64_t *count) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    if (!count || capacity < 0 || (capacity > 0 && !records))
        return fail(FV_ERR_INVALID_ARG, "count must be non-null and records hold capacity entries");
    const int64_t n = std::min<int64_t>(capacity, (int64_t)s->log.size());
    if (n > 0) std::memcpy(records, s->log.data(), sizeof(fv_batch_record) * (size_t)n);
    *count = (int64_t)s->log.size();
    return FV_OK;
}

fv_status fv_server_stats_get(fv_server *s, fv_server_stats *stats) {
    clear_error();
    fv_status st = check_server(s);
    if (st != FV_OK) return st;
    if (!stats) return fail(FV_ERR_INVALID_ARG, "stats must be non-null");
    fill_stats(s, stats);
    return FV_OK;
}

fv_status fv_server_destroy(fv_server *s) {
    clear_error();
    if (!s) return FV_OK;
    (void)hipStreamSynchronize(s->stream);
    for (auto &f : s->inflight) (void)hipEventDestroy(f.done);
    for (auto e : s->spare_events) (void)hipEventDestroy(e);
    for (auto &st : s->staging) {
        if (st.host) (void)hipHostFree(st.host);
        if (st.lambda) (void)hipFree(st.lambda);
    }
    for (auto &m : s->meshes)
        if (m.buf) (void)hipFree(m.buf);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return FV_OK;
}

}  // extern "C"
