// fv_plan.hip -- batching form: a fixed batch composition turned once into a
// device work list, then one fused launch per step over all patch sizes, and
// k steps with a device-side time step captured in one hipGraph.
//
// The paper bundles T patch updates into one kernel call (task fusion, Sec.
// 2.1) and proposes, without being able to run it, to precompile the fixed
// task graph so the GPU resolves the dependencies (Sec. 5, and the outlook of Sec. 6).  Here the
// plan sorts the patches by size, cuts each size class into wave tasks
// (floor(64 / (p+2)) patches per task; the fixed-size body for the sizes built
// in that form, else the runtime-size body with the class's tuned rows), and
// runs all classes in ONE launch of the 2D wave kernel whose waves walk the
// task list: a persistent grid (as many waves as fit on the device, tasks
// largest first) or one wave per task (tasks in memory order).  Classes the
// wave kernel cannot take (3D, or 2D p > 62) are launched per class inside the
// same step.  A plan may instead launch every class on its own kernel with its
// tuned parameters (FV_PLAN_PER_CLASS): the descriptors are still built once,
// and each class runs at its own kernel's occupancy, where the fused launch
// reserves the largest class's LDS ring for every wave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "fvpatch.h"
#include "fv_host.h"
#include "fv_internal.h"

struct fv_plan {
    int device = -1;
    int32_t dim = 2, nq = 5, num_patches = 0;
    uint32_t flags = 0;
    bool persistent = true;
    int64_t lo = 0, hi = 0;  // extent in doubles
    // device descriptors: offsets / ids sorted into tasks and groups, the task list
    int64_t *d_offsets = nullptr;
    int32_t *d_ids = nullptr;
    fv::WaveTask *d_tasks = nullptr;
    int32_t num_tasks = 0;
    int32_t ring_words = 0;
    int32_t prefetch = 0;
    bool even_offsets = true;  // every wave-task patch starts at an even double and has even rows
    bool odd_rows_only = true;  // every wave task runs a fixed-size body with odd rows (16-byte bursts need
                                // only aligned buffers)
    struct Group {
        int32_t p, first, count;
        bool even;  // every patch of the class starts at an even double and spans an even number of them
        // regular: the class's patches are evenly spaced, base + i stride, with consecutive lambda
        // indices id0 + i; it then launches without descriptors, as a plain call does
        bool regular;
        int64_t base, stride;
        int32_t id0;
    };
    std::vector<Group> groups;  // classes launched per class (3D, 2D p > 62; every class with FV_PLAN_PER_CLASS)
    // launch parameters of each size class, fixed at creation (index p; kernel -1: no such class)
    std::vector<fv_tuning> tune;
    double *d_rexec = nullptr;  // dt / h of an execute that takes its dt from device memory
    // captured multi-step run
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t steps = 0;
    double *d_r = nullptr;  // dt / h per captured step
    unsigned long long *d_slot = nullptr;  // max-eigenvalue bits and block counter of the step-size reduction
};

namespace fv {
namespace {

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
[[maybe_unused]] bool overlap(uintptr_t a0, uintptr_t a1, uintptr_t b0, uintptr_t b1) { return a0 < b1 && b0 < a1; }

fv_status plan_buffers(const fv_plan *pl, const double *in, const double *out, const double *lambda_out) {
    return check_buffers(in, out, lambda_out, pl->num_patches, pl->lo, pl->hi);
}

fv_status check_device(const fv_plan *pl) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FV_ERR_NO_DEVICE, "hipGetDevice failed");
    if (dev != pl->device) return fail(FV_ERR_INVALID_ARG, "plan was created on device %d, current is %d", pl->device, dev);
    return FV_OK;
}

// Enqueue one step of the plan: the fused task launch and the per-class launches.
fv_status enqueue_step(const fv_plan *pl, const double *in, double *out, double r, const double *r_dev, double gamma,
                       double *lambda_out, hipStream_t stream) {
    if (pl->num_tasks > 0) {
        TaskLaunch T;
        T.in = in;
        T.out = out;
        T.offsets = pl->d_offsets;
        T.ids = pl->d_ids;
        T.tasks = pl->d_tasks;
        T.num_tasks = pl->num_tasks;
        T.nq = pl->nq;
        T.ring_words = pl->ring_words;
        T.prefetch = pl->prefetch;
        T.vec2 = (pl->even_offsets || pl->odd_rows_only) && aligned16(in) && aligned16(out);
        T.persistent = pl->persistent;
        T.r = r;
        T.r_dev = r_dev;
        T.gamma = gamma;
        T.flags = pl->flags;
        T.lambda_out = lambda_out;
        hipError_t e = launch_update2d_tasks(T, stream);
        if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "fused launch failed: %s", hipGetErrorString(e));
    }
    for (const auto &g : pl->groups) {
        UpdateLaunch L;
        L.in = in;
        L.out = out;
        L.offsets = pl->d_offsets + g.first;
        L.ids = pl->d_ids + g.first;
        L.num_items = g.count;
        L.p = g.p;
        L.dim = pl->dim;
        L.nq = pl->nq;
        L.r = r;
        L.r_dev = r_dev;
        L.gamma = gamma;
        L.flags = pl->flags;
        L.lambda_out = lambda_out;
        L.vec2 = g.even && aligned16(in) && aligned16(out);
        if (g.regular) {
            L.in = in + g.base;
            L.out = out + g.base;
            L.offsets = nullptr;
            L.ids = nullptr;
            L.stride = g.stride;
            L.lambda_out = lambda_out ? lambda_out + g.id0 : nullptr;
            L.vec2 = g.stride % 2 == 0 && patch_doubles(g.p, L.dim, L.nq) % 2 == 0 && aligned16(L.in) &&
                     aligned16(L.out);
        }
        apply_tuning(L, pl->tune[g.p]);
        if (L.dim == 2 && L.kernel == FV_KERNEL_WAVE && !wave2d_fits(L.p)) L.kernel = FV_KERNEL_BLOCK;
        if (L.kernel == FV_KERNEL_FIXED && fixed_odd_rows(L.dim, L.p, L.nq)) L.vec2 = aligned16(L.out);
        hipError_t e = launch_update(L, stream);
        if (e != hipSuccess) return fail(FV_ERR_LAUNCH, "class launch (p=%d) failed: %s", g.p, hipGetErrorString(e));
    }
    return FV_OK;
}

void release_graph(fv_plan *pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->d_r) (void)hipFree(pl->d_r);
    if (pl->d_slot) (void)hipFree(pl->d_slot);
    pl->d_slot = nullptr;
    pl->exec = nullptr;
    pl->graph = nullptr;
    pl->d_r = nullptr;
    pl->steps = 0;
}

void release(fv_plan *pl) {
    release_graph(pl);
    if (pl->d_rexec) (void)hipFree(pl->d_rexec);
    if (pl->d_offsets) (void)hipFree(pl->d_offsets);
    if (pl->d_ids) (void)hipFree(pl->d_ids);
    if (pl->d_tasks) (void)hipFree(pl->d_tasks);
    delete pl;
}

}  // namespace
}  // namespace fv

using namespace fv;

extern "C" {

fv_status fv_plan_create(fv_plan **plan, const int32_t *sizes, const int64_t *offsets, int32_t num_patches,
                         int32_t dim, int32_t unknowns, uint32_t flags, const fv_tune_entry *tune_table,
                         int32_t tune_entries) {
    clear_error();
    if (!plan) return fail(FV_ERR_INVALID_ARG, "plan must be non-null");
    *plan = nullptr;
    fv_status st = check_scalars(dim, unknowns, 1.0, 1.0, 2.0, flags & (FV_HALO_PERIODIC | FV_HALO_FROM_IN));
    if (st != FV_OK) return st;
    if (flags & ~(FV_HALO_PERIODIC | FV_HALO_FROM_IN | FV_PLAN_NO_PERSIST | FV_PLAN_PER_CLASS))
        return fail(FV_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
    if ((flags & FV_PLAN_NO_PERSIST) && (flags & FV_PLAN_PER_CLASS))
        return fail(FV_ERR_INVALID_ARG, "FV_PLAN_NO_PERSIST and FV_PLAN_PER_CLASS exclude each other");
    if (num_patches < 1) return fail(FV_ERR_INVALID_ARG, "a plan needs at least one patch");
    if (tune_entries < 0 || (tune_entries > 0 && !tune_table))
        return fail(FV_ERR_INVALID_ARG, "tune_table must hold tune_entries (>= 0) entries");
    BatchShape shape;
    st = check_layout(sizes, offsets, num_patches, dim, unknowns, &shape);
    if (st != FV_OK) return st;
    // the plan's own launch parameters: its table's entries for its (dim, unknowns), validated
    // like fv_set_tuning's; other classes take the installed (process-wide) or default ones
    const int pmax_t = max_p(dim);
    std::vector<fv_tuning> own(pmax_t + 1, fv_tuning{-1, 0, 0, 0});
    for (int32_t k = 0; k < tune_entries; ++k) {
        const fv_tune_entry &e = tune_table[k];
        if (e.dim != dim || e.unknowns != unknowns) continue;
        if (e.p < 1 || e.p > pmax_t) return fail(FV_ERR_INVALID_ARG, "tune_table[%d]: p=%d outside [1, %d]", k, e.p, pmax_t);
        if (own[e.p].kernel >= 0) return fail(FV_ERR_INVALID_ARG, "tune_table: two entries for p=%d", e.p);
        if ((st = resolve_tuning(dim, unknowns, e.p, e.tuning, &own[e.p])) != FV_OK) return st;
    }
    DeviceContext *ctx = nullptr;
    st = current_context(&ctx);
    if (st != FV_OK) return st;

    auto *pl = new fv_plan();
    hipGetDevice(&pl->device);
    pl->dim = dim;
    pl->nq = unknowns;
    pl->flags = flags & (FV_HALO_PERIODIC | FV_HALO_FROM_IN);
    pl->persistent = !(flags & (FV_PLAN_NO_PERSIST | FV_PLAN_PER_CLASS));
    const bool per_class = (flags & FV_PLAN_PER_CLASS) != 0;
    const bool whole_rows = (pl->flags & (FV_HALO_PERIODIC | FV_HALO_FROM_IN)) != 0;  // of the fused launch
    pl->num_patches = num_patches;
    pl->lo = shape.lo;
    pl->hi = shape.hi;
    pl->tune.assign(pmax_t + 1, fv_tuning{-1, 0, 0, 0});

    // counting sort by size, largest first
    const int pmax = max_p(dim);
    std::vector<int32_t> count(pmax + 1, 0);
    for (int32_t t = 0; t < num_patches; ++t) count[sizes[t]]++;
    std::vector<int64_t> hoff(num_patches);
    std::vector<int32_t> hid(num_patches);
    std::vector<WaveTask> tasks;
    int32_t cursor = 0;
    int32_t best_cells = -1;
    std::vector<int32_t> start(pmax + 1, 0);
    for (int p = pmax; p >= 1; --p) {
        start[p] = cursor;
        cursor += count[p];
    }
    {
        std::vector<int32_t> fill(start);
        for (int32_t t = 0; t < num_patches; ++t) {
            const int32_t k = fill[sizes[t]]++;
            hoff[k] = offsets ? offsets[t] : (int64_t)t * patch_doubles(sizes[t], dim, unknowns);
            hid[k] = t;
        }
    }
    for (int p = pmax; p >= 1; --p) {
        if (!count[p]) continue;
        pl->tune[p] = own[p].kernel >= 0 ? own[p] : tuning_for(dim, unknowns, p);
        if (dim == 2 && wave2d_fits(p) && !per_class) {
            const fv_tuning tu = pl->tune[p];
            // rows == 0: the fixed-size form of the kernel.  A class built in that form runs it
            // in the fused launch whatever its tuning: a tuned runtime-size body keeps its rows
            // there but not its block size or prefetch (one of each per fused launch), and
            // measured slower than the fixed-size body
            const bool fixed = tu.kernel == FV_KERNEL_FIXED || wave2d_fixed(p, unknowns);
            const int rows = fixed ? 0 : (tu.kernel == FV_KERNEL_WAVE && tu.rows > 0 ? tu.rows : 6);
            const int ppw = 64 / (p + 2);
            for (int32_t f = 0; f < count[p]; f += ppw)
                tasks.push_back(WaveTask{p, rows, start[p] + f, std::min<int32_t>(ppw, count[p] - f)});
            pl->ring_words = std::max(pl->ring_words,
                                      fixed ? wave2d_fixed_ring_words(p, whole_rows) : wave2d_ring_words(p, unknowns, rows));
            const int64_t cells = (int64_t)count[p] * p * p;
            if (cells > best_cells) {
                best_cells = (int32_t)std::min<int64_t>(cells, INT32_MAX);
                pl->prefetch = (tu.kernel == FV_KERNEL_WAVE || tu.kernel == FV_KERNEL_FIXED) ? tu.prefetch : 0;
            }
            if (((p + 2) * unknowns) % 2) pl->even_offsets = false;
            for (int32_t k = start[p]; k < start[p] + count[p]; ++k)
                if (hoff[k] & 1) pl->even_offsets = false;
            if (!(fixed && fixed_odd_rows(dim, p, unknowns))) pl->odd_rows_only = false;
        } else {
            bool even = patch_doubles(p, dim, unknowns) % 2 == 0;
            for (int32_t k = start[p]; k < start[p] + count[p] && even; ++k) even = (hoff[k] & 1) == 0;
            const int32_t f = start[p], c = count[p];
            const int64_t stride = c > 1 ? hoff[f + 1] - hoff[f] : patch_doubles(p, dim, unknowns);
            bool regular = stride >= patch_doubles(p, dim, unknowns);
            for (int32_t k = 1; k < c && regular; ++k)
                regular = hoff[f + k] == hoff[f] + (int64_t)k * stride && hid[f + k] == hid[f] + k;
            pl->groups.push_back(fv_plan::Group{p, f, c, even, regular, hoff[f], stride, hid[f]});
        }
    }
    // One wave per task: workgroups start in task order, so tasks in memory order keep the
    // resident waves on neighbouring patches (DRAM page locality); a persistent grid keeps
    // largest-first, which balances the waves' shares.
    if (!pl->persistent)
        std::stable_sort(tasks.begin(), tasks.end(),
                         [&](const WaveTask &a, const WaveTask &b) { return hoff[a.first] < hoff[b.first]; });
    pl->num_tasks = (int32_t)tasks.size();

    // device copies of the work list
    bool ok = hipMalloc(&pl->d_rexec, sizeof(double)) == hipSuccess &&
              hipMalloc(&pl->d_offsets, sizeof(int64_t) * num_patches) == hipSuccess &&
              hipMalloc(&pl->d_ids, sizeof(int32_t) * num_patches) == hipSuccess &&
              (tasks.empty() || hipMalloc(&pl->d_tasks, sizeof(WaveTask) * tasks.size()) == hipSuccess);
    if (!ok) {
        release(pl);
        return fail(FV_ERR_OOM, "device allocation of the work list failed");
    }
    ok = hipMemcpy(pl->d_offsets, hoff.data(), sizeof(int64_t) * num_patches, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(pl->d_ids, hid.data(), sizeof(int32_t) * num_patches, hipMemcpyHostToDevice) == hipSuccess &&
         (tasks.empty() ||
          hipMemcpy(pl->d_tasks, tasks.data(), sizeof(WaveTask) * tasks.size(), hipMemcpyHostToDevice) == hipSuccess);
    if (!ok) {
        release(pl);
        return fail(FV_ERR_LAUNCH, "upload of the work list failed");
    }
    *plan = pl;
    return FV_OK;
}

fv_status fv_plan_execute(fv_plan *plan, const double *patches_in, double *patches_out, double dt,
                          const double *dt_dev, double h, double gamma, double *lambda_out, void *stream) {
    clear_error();
    if (!plan) return fail(FV_ERR_INVALID_ARG, "plan must be non-null");
    fv_status st = check_scalars(plan->dim, plan->nq, dt_dev ? 1.0 : dt, h, gamma, 0);
    if (st != FV_OK) return st;
    if ((st = check_device(plan)) != FV_OK) return st;
    if ((st = plan_buffers(plan, patches_in, patches_out, lambda_out)) != FV_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!dt_dev) return enqueue_step(plan, patches_in, patches_out, dt / h, nullptr, gamma, lambda_out, s);
    if (!aligned8(dt_dev)) return fail(FV_ERR_INVALID_ARG, "dt_dev must be 8-byte aligned");
    {
        const uintptr_t d0 = reinterpret_cast<uintptr_t>(dt_dev), d1 = d0 + sizeof(double);
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(patches_out + plan->lo),
                        a1 = reinterpret_cast<uintptr_t>(patches_out + plan->hi);
        const uintptr_t l0 = reinterpret_cast<uintptr_t>(lambda_out),
                        l1 = reinterpret_cast<uintptr_t>(lambda_out + (lambda_out ? plan->num_patches : 0));
        if (overlap(d0, d1, a0, a1) || overlap(d0, d1, l0, l1))
            return fail(FV_ERR_OVERLAP, "dt_dev overlaps patches_out or lambda_out");
    }
    // r = dt / h on the device (correctly rounded, as the host's), read by the step's launches
    if (launch_ratio(dt_dev, h, plan->d_rexec, s) != hipSuccess)
        return fail(FV_ERR_LAUNCH, "launch of the step-size ratio failed");
    return enqueue_step(plan, patches_in, patches_out, 0.0, plan->d_rexec, gamma, lambda_out, s);
}

fv_status fv_plan_get_tuning(const fv_plan *plan, int32_t p, fv_tuning *tuning) {
    clear_error();
    if (!plan || !tuning) return fail(FV_ERR_INVALID_ARG, "plan and tuning must be non-null");
    if (p < 1 || p >= (int32_t)plan->tune.size() || plan->tune[p].kernel < 0)
        return fail(FV_ERR_INVALID_ARG, "the plan has no patches of size %d", p);
    *tuning = plan->tune[p];
    return FV_OK;
}

fv_status fv_plan_capture_steps(fv_plan *plan, int32_t steps, double *buf_a, double *buf_b, double h, double gamma,
                                double cfl, double *lambda_out, double *dt_dev, void *stream) {
    clear_error();
    if (!plan) return fail(FV_ERR_INVALID_ARG, "plan must be non-null");
    if (steps < 1 || steps > 100000) return fail(FV_ERR_INVALID_ARG, "steps must be in [1, 100000]");
    fv_status st = check_scalars(plan->dim, plan->nq, 1.0, h, gamma, 0);
    if (st != FV_OK) return st;
    if (!std::isfinite(cfl) || !(cfl > 0.0)) return fail(FV_ERR_INVALID_ARG, "cfl must be finite and > 0");
    if (!lambda_out || !dt_dev) return fail(FV_ERR_INVALID_ARG, "lambda_out and dt_dev are required");
    if (!aligned8(dt_dev)) return fail(FV_ERR_INVALID_ARG, "dt_dev must be 8-byte aligned");
    if (!stream) return fail(FV_ERR_INVALID_ARG, "capture needs a non-null stream");
    if ((st = check_device(plan)) != FV_OK) return st;
    if ((st = plan_buffers(plan, buf_a, buf_b, lambda_out)) != FV_OK) return st;
    {
        const uintptr_t d0 = reinterpret_cast<uintptr_t>(dt_dev), d1 = reinterpret_cast<uintptr_t>(dt_dev + steps + 1);
        const uintptr_t l0 = reinterpret_cast<uintptr_t>(lambda_out), l1 = reinterpret_cast<uintptr_t>(lambda_out + plan->num_patches);
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(buf_a + plan->lo), a1 = reinterpret_cast<uintptr_t>(buf_a + plan->hi);
        const uintptr_t b0 = reinterpret_cast<uintptr_t>(buf_b + plan->lo), b1 = reinterpret_cast<uintptr_t>(buf_b + plan->hi);
        if (overlap(d0, d1, l0, l1) || overlap(d0, d1, a0, a1) || overlap(d0, d1, b0, b1))
            return fail(FV_ERR_OVERLAP, "dt_dev overlaps another buffer");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    release_graph(plan);
    if (hipMalloc(&plan->d_r, sizeof(double) * (steps + 1)) != hipSuccess ||
        hipMalloc(&plan->d_slot, 2 * sizeof(unsigned long long)) != hipSuccess) {
        release_graph(plan);
        return fail(FV_ERR_OOM, "device allocation failed");
    }
    // zeroed once, outside the graph; every step-size launch leaves them zero
    if (hipMemsetAsync(plan->d_slot, 0, 2 * sizeof(unsigned long long), s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        release_graph(plan);
        return fail(FV_ERR_LAUNCH, "clearing the reduction slot failed");
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
        release_graph(plan);
        return fail(FV_ERR_LAUNCH, "hipStreamBeginCapture failed");
    }
    fv_status cap = FV_OK;
    if (launch_ratio(dt_dev, h, plan->d_r, s) != hipSuccess) cap = fail(FV_ERR_LAUNCH, "capture of the first step size failed");
    for (int32_t k = 0; k < steps && cap == FV_OK; ++k) {
        const double *src = (k % 2 == 0) ? buf_a : buf_b;
        double *dst = (k % 2 == 0) ? buf_b : buf_a;
        cap = enqueue_step(plan, src, dst, 0.0, plan->d_r + k, gamma, lambda_out, s);
        if (cap == FV_OK && launch_next_dt(lambda_out, plan->num_patches, cfl, h, plan->dim, dt_dev + k + 1,
                                           plan->d_r + k + 1, plan->d_slot,
                                           reinterpret_cast<unsigned int *>(plan->d_slot + 1), s) != hipSuccess)
            cap = fail(FV_ERR_LAUNCH, "capture of the step-size kernel failed");
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (cap != FV_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        release_graph(plan);
        return cap != FV_OK ? cap : fail(FV_ERR_LAUNCH, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    }
    plan->graph = g;
    if (hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        release_graph(plan);
        return fail(FV_ERR_LAUNCH, "hipGraphInstantiate failed");
    }
    plan->steps = steps;
    return FV_OK;
}

fv_status fv_plan_replay(fv_plan *plan, void *stream) {
    clear_error();
    if (!plan) return fail(FV_ERR_INVALID_ARG, "plan must be non-null");
    if (!plan->exec) return fail(FV_ERR_INVALID_ARG, "no captured steps: call fv_plan_capture_steps first");
    fv_status st = check_device(plan);
    if (st != FV_OK) return st;
    if (hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(FV_ERR_LAUNCH, "hipGraphLaunch failed");
    return FV_OK;
}

fv_status fv_plan_info(const fv_plan *plan, fv_plan_stats *info) {
    clear_error();
    if (!plan || !info) return fail(FV_ERR_INVALID_ARG, "plan and info must be non-null");
    info->num_patches = plan->num_patches;
    info->num_tasks = plan->num_tasks;
    info->num_class_launches = (int32_t)plan->groups.size();
    info->prefetch = plan->prefetch;
    info->lds_per_wave_bytes = (int32_t)(plan->ring_words * sizeof(double));
    info->persistent = plan->persistent ? 1 : 0;
    info->captured_steps = plan->steps;
    return FV_OK;
}

fv_status fv_plan_destroy(fv_plan *plan) {
    clear_error();
    if (!plan) return FV_OK;
    (void)hipDeviceSynchronize();  // no replay or launch of this plan may still be running
    release(plan);
    return FV_OK;
}

}  // extern "C"
