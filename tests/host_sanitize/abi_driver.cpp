// abi_driver.cpp -- drives every entry point of include/fvpatch.h through the
// library's host code, linked against the CPU stand-in of the HIP runtime
// (fake_hip.cpp), under AddressSanitizer and UndefinedBehaviorSanitizer.
// Kernels do not run, so no result is checked here (the GPU tests do that);
// what is checked is the host side: every status, and -- by the sanitizers and
// the stand-in runtime -- memory errors, undefined behaviour, launch
// configurations, kernel pointer arguments and the lifetime of the device memory
// that graph executables refer to.  Each scenario mirrors a use the tests or
// the benchmark make of the library; the flavour scenario replays the
// comparison matrix of the benchmark, buffers freed and reallocated between
// batch sizes.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "fvpatch.h"

// calls of the stand-in runtime's allocation and free routines so far (fake_hip.cpp)
extern "C" long fake_hip_alloc_calls();
// a pause the stand-in runtime takes at the start of every kernel launch (fake_hip.cpp)
extern "C" void fake_hip_set_launch_sleep_us(int us);

namespace {

std::atomic<int> g_calls{0};

void expect(fv_status got, fv_status want, const char *what, int line) {
    ++g_calls;
    if (got != want) {
        std::fprintf(stderr, "line %d: %s returned %d (%s: %s), expected %d\n", line, what, (int)got,
                     fv_status_string(got), fv_last_error(), (int)want);
        std::exit(2);
    }
}
#define OK(call) expect((call), FV_OK, #call, __LINE__)
#define FAILS(call, st) expect((call), (st), #call, __LINE__)

int64_t patch_doubles(int p, int dim, int nq) {
    const int64_t w = p + 2;
    return (dim == 2 ? w * w : w * w * w) * nq;
}

double *dev_alloc(size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) std::abort();
    std::memset(p, 0, n * sizeof(double));
    return static_cast<double *>(p);
}
void dev_free(void *p) { (void)hipFree(p); }

struct Layout {
    std::vector<int32_t> sizes;
    std::vector<int64_t> offsets;
    int64_t extent = 0;
};

// Mixed sizes, shuffled placement with gaps (odd ones included).
Layout scattered(int T, const std::vector<int> &choices, int dim, int nq, unsigned seed) {
    std::mt19937 rng(seed);
    Layout L;
    L.sizes.resize(T);
    for (int t = 0; t < T; ++t) L.sizes[t] = choices[rng() % choices.size()];
    std::vector<int> order(T);
    for (int t = 0; t < T; ++t) order[t] = t;
    std::shuffle(order.begin(), order.end(), rng);
    L.offsets.resize(T);
    int64_t pos = 0;
    for (int t : order) {
        pos += rng() % 4;
        L.offsets[t] = pos;
        pos += patch_doubles(L.sizes[t], dim, nq);
    }
    L.extent = pos + 3;
    return L;
}

void plain_updates() {
    std::puts("scenario: plain updates");
    for (int dim : {2, 3}) {
        for (int nq : {5, 4}) {
            if (dim == 3 && nq == 4) continue;
            const std::vector<int> ch = dim == 2 ? std::vector<int>{1, 3, 5, 9, 16, 17, 40, 63, 64}
                                                 : std::vector<int>{1, 4, 6, 8, 11, 24};
            for (unsigned seed = 0; seed < 3; ++seed) {
                Layout L = scattered(dim == 2 ? 700 : 120, ch, dim, nq, seed);
                double *in = dev_alloc(L.extent), *out = dev_alloc(L.extent), *lam = dev_alloc(L.sizes.size());
                const int T = (int)L.sizes.size();
                for (uint32_t flags : {0u, (uint32_t)FV_HALO_PERIODIC, (uint32_t)FV_HALO_FROM_IN})
                    OK(fv_patch_batch_update(in, out, L.sizes.data(), L.offsets.data(), T, dim, nq, 1e-3, 0.02, 1.4,
                                             flags, seed ? lam : nullptr, nullptr));
                // sorted offsets of equal sizes, evenly spaced and contiguous
                const int p = ch[seed % ch.size()];
                std::vector<int32_t> same(T, p);
                std::vector<int64_t> even(T);
                for (int t = 0; t < T; ++t) even[t] = 1 + t * (patch_doubles(p, dim, nq) + 2);
                if (even[T - 1] + patch_doubles(p, dim, nq) <= L.extent) {
                    OK(fv_patch_batch_update(in, out, same.data(), even.data(), T, dim, nq, 1e-3, 0.02, 1.4, 0, lam,
                                             nullptr));
                }
                const int Tc = (int)(L.extent / patch_doubles(p, dim, nq));
                std::vector<int32_t> sc(Tc, p);
                OK(fv_patch_batch_update(in, out, sc.data(), nullptr, Tc, dim, nq, 1e-3, 0.02, 1.4,
                                         FV_HALO_PERIODIC, nullptr, nullptr));
                FAILS(fv_patch_batch_update(in, in, L.sizes.data(), L.offsets.data(), T, dim, nq, 1e-3, 0.02, 1.4, 0,
                                            nullptr, nullptr),
                      FV_ERR_OVERLAP);
                dev_free(in);
                dev_free(out);
                dev_free(lam);
            }
        }
    }
    OK(fv_patch_batch_update(nullptr, nullptr, nullptr, nullptr, 0, 2, 5, 1e-3, 0.02, 1.4, 0, nullptr, nullptr));
    // descriptor ring: more calls than slots, growing batches
    for (int k = 1; k <= 9; ++k) {
        Layout L = scattered(100 * k * k, {3, 5, 9, 17}, 2, 5, 100 + k);
        double *in = dev_alloc(L.extent), *out = dev_alloc(L.extent);
        OK(fv_patch_batch_update(in, out, L.sizes.data(), L.offsets.data(), (int)L.sizes.size(), 2, 5, 1e-3, 0.02,
                                 1.4, 0, nullptr, nullptr));
        dev_free(in);
        dev_free(out);
    }
}

void noalloc_updates() {
    std::puts("scenario: the no-allocation entry point");
    for (int round = 0; round < 2; ++round) {
        for (int dim : {2, 3}) {
            const std::vector<int> ch = dim == 2 ? std::vector<int>{3, 5, 9, 17, 40} : std::vector<int>{4, 6, 8, 11};
            // the second round takes smaller batches through the same descriptor array
            Layout L = scattered(round == 0 ? 900 : 150, ch, dim, 5, 40 + round);
            const int T = (int)L.sizes.size();
            double *in = dev_alloc(L.extent), *out = dev_alloc(L.extent), *lam = dev_alloc(T);
            const long a1 = fake_hip_alloc_calls();
            for (uint32_t flags : {0u, (uint32_t)FV_HALO_PERIODIC, (uint32_t)FV_HALO_FROM_IN})
                OK(fv_patch_batch_update_noalloc(in, out, L.sizes.data(), L.offsets.data(), T, dim, 5, 1e-3, 0.02,
                                                 1.4, flags, round ? lam : nullptr, nullptr));
            std::vector<int32_t> same(T, ch[0]);
            OK(fv_patch_batch_update_noalloc(in, out, same.data(), nullptr, T / 2, dim, 5, 1e-3, 0.02, 1.4, 0, lam,
                                             nullptr));
            FAILS(fv_patch_batch_update_noalloc(in, in, L.sizes.data(), L.offsets.data(), T, dim, 5, 1e-3, 0.02, 1.4,
                                                0, nullptr, nullptr),
                  FV_ERR_OVERLAP);
            if (fake_hip_alloc_calls() != a1) {
                std::fprintf(stderr, "fv_patch_batch_update_noalloc allocated or freed memory\n");
                std::exit(3);
            }
            dev_free(in);
            dev_free(out);
            dev_free(lam);
        }
    }
    std::vector<int32_t> big(FV_NOALLOC_MAX_PATCHES + 1, 3);
    FAILS(fv_patch_batch_update_noalloc(reinterpret_cast<double *>(64), reinterpret_cast<double *>(1 << 30),
                                        big.data(), nullptr, (int)big.size(), 2, 5, 1e-3, 0.02, 1.4, 0, nullptr,
                                        nullptr),
          FV_ERR_INVALID_ARG);
}

// Calls from more threads than the library keeps descriptor slots, each on its own buffers, with
// batches that grow so that slots are reallocated while other threads' calls are under way.
void concurrent_updates() {
    std::puts("scenario: calls from 12 threads at once");
    fake_hip_set_launch_sleep_us(200);  // each call holds its descriptor slot across a slow launch
    std::vector<std::thread> pool;
    for (int w = 0; w < 12; ++w) {
        pool.emplace_back([w] {
            for (int k = 0; k < 10; ++k) {
                // up to 12,000 patches: (offset, id) lists beyond the slots' first 64 KiB
                Layout L = scattered(300 + 1300 * ((w + k) % 10), {3, 5}, 2, 5, 1000u * w + k);
                const int T = (int)L.sizes.size();
                double *in = dev_alloc(L.extent), *out = dev_alloc(L.extent), *lam = dev_alloc(T);
                OK(fv_patch_batch_update(in, out, L.sizes.data(), L.offsets.data(), T, 2, 5, 1e-3, 0.02, 1.4,
                                         (uint32_t)(k % 3 == 0 ? FV_HALO_PERIODIC : 0), lam, nullptr));
                if (k % 3 == 1)
                    OK(fv_patch_batch_update_noalloc(in, out, L.sizes.data(), L.offsets.data(), T, 2, 5, 1e-3, 0.02,
                                                     1.4, 0, lam, nullptr));
                dev_free(in);
                dev_free(out);
                dev_free(lam);
            }
        });
    }
    for (auto &t : pool) t.join();
    fake_hip_set_launch_sleep_us(0);
}

void pde_updates() {
    std::puts("scenario: the other PDEs");
    struct P { int pde, dim, np; double prm[3]; };
    const P pdes[] = {{FV_PDE_SHALLOW_WATER, 2, 2, {9.81, 0.5, 0}}, {FV_PDE_ADVECTION, 2, 3, {0.7, -0.4, 0.25}},
                      {FV_PDE_ADVECTION, 3, 3, {0.7, -0.4, 0.25}},  {FV_PDE_ACOUSTICS, 2, 2, {1.2, 2.0, 0}},
                      {FV_PDE_ACOUSTICS, 3, 2, {1.2, 2.0, 0}},      {FV_PDE_ACOUSTICS_NCP, 2, 2, {1.2, 2.0, 0}},
                      {FV_PDE_EULER, 2, 1, {1.4, 0, 0}}};
    for (const P &x : pdes) {
        int32_t nq = 0, np = 0;
        OK(fv_pde_unknowns(x.pde, x.dim, &nq, &np));
        const std::vector<int> ch = x.dim == 2 ? std::vector<int>{3, 5, 16, 30} : std::vector<int>{4, 8, 13};
        Layout L = scattered(60, ch, x.dim, nq, 7);
        double *in = dev_alloc(L.extent), *out = dev_alloc(L.extent), *lam = dev_alloc(60);
        for (uint32_t flags : {0u, (uint32_t)FV_HALO_PERIODIC})
            OK(fv_pde_batch_update(x.pde, x.prm, np, in, out, L.sizes.data(), L.offsets.data(), 60, x.dim, 1e-4, 0.02,
                                   flags, lam, nullptr));
        dev_free(in);
        dev_free(out);
        dev_free(lam);
    }
}

void plans() {
    std::puts("scenario: plans");
    for (int dim : {2, 3}) {
        const std::vector<int> ch = dim == 2 ? std::vector<int>{3, 4, 5, 9, 17, 63} : std::vector<int>{4, 5, 8};
        Layout L = scattered(dim == 2 ? 2000 : 150, ch, dim, 5, 11);
        const int T = (int)L.sizes.size();
        double *a = dev_alloc(L.extent), *b = dev_alloc(L.extent), *lam = dev_alloc(T), *dt = dev_alloc(9);
        fv_tune_entry table[3] = {{dim, 5, 4, {FV_KERNEL_BLOCK, 0, 0, 0}},
                                  {dim, 5, 5, {dim == 2 ? FV_KERNEL_TILE : FV_KERNEL_BLOCK, 0, 0, 0}},
                                  {3 - dim + 2, 5, 7, {FV_KERNEL_BLOCK, 0, 0, 0}}};
        for (uint32_t mode : {0u, (uint32_t)FV_PLAN_NO_PERSIST, (uint32_t)FV_PLAN_PER_CLASS}) {
            fv_plan *plan = nullptr;
            OK(fv_plan_create(&plan, L.sizes.data(), L.offsets.data(), T, dim, 5, mode | FV_HALO_PERIODIC, table, 3));
            fv_plan_stats st;
            OK(fv_plan_info(plan, &st));
            fv_tuning tu;
            OK(fv_plan_get_tuning(plan, 4, &tu));
            FAILS(fv_plan_get_tuning(plan, 2, &tu), FV_ERR_INVALID_ARG);
            OK(fv_plan_execute(plan, a, b, 1e-3, nullptr, 0.02, 1.4, lam, nullptr));
            OK(fv_plan_execute(plan, b, a, 0.0, dt, 0.02, 1.4, nullptr, nullptr));
            FAILS(fv_plan_execute(plan, a, b, 0.0, b + 8, 0.02, 1.4, lam, nullptr), FV_ERR_OVERLAP);
            hipStream_t s = nullptr;
            (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            OK(fv_plan_capture_steps(plan, 4, a, b, 0.02, 1.4, 0.4, lam, dt, s));
            OK(fv_plan_replay(plan, s));
            OK(fv_plan_replay(plan, s));
            OK(fv_plan_capture_steps(plan, 8, a, b, 0.02, 1.4, 0.4, lam, dt, s));  // replaces the first capture
            OK(fv_plan_replay(plan, s));
            OK(fv_plan_destroy(plan));  // before the buffers it captured are freed
            (void)hipStreamDestroy(s);
        }
        dev_free(a);
        dev_free(b);
        dev_free(lam);
        dev_free(dt);
    }
}

void flavour_matrix() {
    std::puts("scenario: the comparison flavours (the benchmark's matrix)");
    const int flavours[] = {FV_FLAVOUR_BATCHED, FV_FLAVOUR_PATCH_WISE, FV_FLAVOUR_TASK_GRAPH};
    for (int dim : {2, 3}) {
        for (int p : {4, 6, 8}) {
            for (int T : {16, 256, 4096}) {
                if (dim == 3 && T == 4096 && p == 8) continue;  // keeps the stand-in's memory small
                const int64_t n = patch_doubles(p, dim, 5) * T;
                double *a = dev_alloc(n), *c = dev_alloc(n), *lam = dev_alloc(T);
                std::vector<int32_t> sizes(T, p);
                for (bool red : {true, false}) {
                    for (int f : flavours) {
                        const int steps = f == FV_FLAVOUR_TASK_GRAPH ? 2 : 3;
                        for (int k = 0; k < steps; ++k)
                            OK(fv_flavour_update(f, k % 2 ? c : a, k % 2 ? a : c, sizes.data(), nullptr, T, dim, 5,
                                                 1e-3, 0.02, 1.4, 0, red ? lam : nullptr, nullptr));
                    }
                }
                // and with an offsets array (uploaded by the call)
                std::vector<int64_t> offs(T);
                for (int t = 0; t < T; ++t) offs[t] = t * patch_doubles(p, dim, 5);
                for (int f : flavours)
                    OK(fv_flavour_update(f, a, c, sizes.data(), offs.data(), T, dim, 5, 1e-3, 0.02, 1.4,
                                         FV_HALO_PERIODIC, lam, nullptr));
                dev_free(a);  // the benchmark frees the buffers between batch sizes
                dev_free(c);
                dev_free(lam);
            }
        }
    }
    std::vector<int32_t> mixed = {4, 6};
    FAILS(fv_flavour_update(FV_FLAVOUR_BATCHED, (double *)0x1000, (double *)0x100000, mixed.data(), nullptr, 2, 2, 5,
                            1e-3, 0.02, 1.4, 0, nullptr, nullptr),
          FV_ERR_INVALID_ARG);
}

void serving() {
    std::puts("scenario: serving");
    for (int32_t mode : {FV_SERVE_FUSED, FV_SERVE_PLAIN}) {
        fv_server_config cfg{};
        cfg.budget_bytes = 1LL << 32;
        cfg.gamma = 1.4;
        cfg.flags = FV_HALO_PERIODIC;
        cfg.mode = mode;
        cfg.max_inflight = 4;
        cfg.max_retries = 2;
        cfg.deadline_ms = 20.0;
        fv_server *s = nullptr;
        OK(fv_server_create(&s, &cfg));
        Layout m2 = scattered(3000, {3, 5, 9, 17}, 2, 5, 21);
        std::vector<int32_t> s3(200, 8);
        std::vector<double> h2(patch_doubles(17, 2, 5) * 3000), h3(patch_doubles(8, 3, 5) * 200);
        int32_t id2 = -1, id3 = -1;
        OK(fv_server_add_mesh(s, 2, 5, 0.02, m2.sizes.data(), 3000, h2.data(), &id2));
        OK(fv_server_add_mesh(s, 3, 5, 0.01, s3.data(), 200, h3.data(), &id3));
        std::mt19937 rng(5);
        std::vector<fv_serve_request> trace;
        int pos2 = 0, pos3 = 0;
        for (int k = 0; k < 300; ++k) {
            fv_serve_request r{};
            r.arrival_ns = (int64_t)k * 50000;
            const bool three = rng() % 5 == 0;
            r.mesh = three ? id3 : id2;
            int &pos = three ? pos3 : pos2;
            const int M = three ? 200 : 3000;
            r.first = pos;
            r.count = std::min<int>(1 + rng() % 400, M - pos);
            pos = (pos + r.count) % M;
            r.dt = 1e-4;
            trace.push_back(r);
        }
        fv_server_stats st;
        OK(fv_server_run_trace(s, trace.data(), (int64_t)trace.size(), &st));
        if (st.completed != 300) std::exit(3);
        std::vector<fv_batch_record> log(400);
        int64_t nlog = 0;
        OK(fv_server_batch_log(s, log.data(), (int64_t)log.size(), &nlog));
        OK(fv_server_batch_log(s, nullptr, 0, &nlog));
        // failure paths, forced from the host
        int64_t t1 = 0, t2 = 0, t3 = 0;
        OK(fv_server_submit(s, id2, 0, 100, 1e-4, 0, &t1));
        OK(fv_server_submit(s, id2, 200, 100, 1e-4, 0, &t2));
        OK(fv_server_inject(s, t1, FV_INJECT_FAIL, 1));
        OK(fv_server_inject(s, t2, FV_INJECT_FAIL, 9));
        FAILS(fv_server_drain(s, &st), FV_ERR_LAUNCH);  // t2 runs out of re-runs
        OK(fv_server_drain(s, &st));
        OK(fv_server_submit(s, id3, 0, 50, 1e-4, 0, &t3));
        OK(fv_server_submit(s, id3, 25, 50, 1e-4, 0, nullptr));
        OK(fv_server_inject(s, t3, FV_INJECT_FAIL, 1));
        FAILS(fv_server_drain(s, &st), FV_ERR_LAUNCH);  // a later batch used its output
        OK(fv_server_drain(s, &st));
        OK(fv_server_submit(s, id2, 10, 10, 1e-4, 0, &t1));
        OK(fv_server_inject(s, t1, FV_INJECT_HANG, 0));
        OK(fv_server_poll(s, &st));
        FAILS(fv_server_drain(s, &st), FV_ERR_LAUNCH);  // deadline
        OK(fv_server_inject(s, t1, 0, 0));
        OK(fv_server_drain(s, &st));
        FAILS(fv_server_inject(s, 0, FV_INJECT_FAIL, 1), FV_ERR_INVALID_ARG);
        FAILS(fv_server_submit(s, id2, 2990, 20, 1e-4, 0, nullptr), FV_ERR_INVALID_ARG);
        OK(fv_server_read_mesh(s, id2, h2.data()));
        OK(fv_server_read_mesh(s, id3, h3.data()));
        OK(fv_server_stats_get(s, &st));
        OK(fv_server_destroy(s));
    }
}

void meshes() {
    std::puts("scenario: patch meshes");
    for (int dim : {2, 3}) {
        const int n = dim == 2 ? 9 : 4, p = dim == 2 ? 16 : 8, T = dim == 2 ? n * n : n * n * n;
        std::vector<int32_t> sizes(T, p), nb(T * 2 * dim);
        for (int t = 0; t < T; ++t)
            for (int f = 0; f < 2 * dim; ++f) nb[t * 2 * dim + f] = (t + 1 + f) % T;
        const int64_t N = patch_doubles(p, dim, 5) * T;
        double *a = dev_alloc(N), *b = dev_alloc(N), *lam = dev_alloc(T), *dt = dev_alloc(T), *h = dev_alloc(T);
        fv_mesh *m = nullptr;
        OK(fv_mesh_create(&m, sizes.data(), nullptr, nb.data(), T, dim, 5));
        OK(fv_mesh_halo_fill(m, a, nullptr));
        OK(fv_mesh_step(m, a, b, dt, h, 1.4, lam, nullptr));
        OK(fv_local_dt(lam, h, T, dim, 0.4, dt, nullptr));
        OK(fv_mesh_destroy(m));
        dev_free(a);
        dev_free(b);
        dev_free(lam);
        dev_free(dt);
        dev_free(h);
    }
}

void transfers() {
    std::puts("scenario: patches in host memory");
    for (int dim : {2, 3}) {
        const int p = dim == 2 ? 16 : 8, T = dim == 2 ? 900 : 150;
        const int64_t pd = patch_doubles(p, dim, 5);
        std::vector<std::vector<double>> src(T, std::vector<double>(pd)), dst(T, std::vector<double>(pd));
        std::vector<const double *> in(T);
        std::vector<double *> out(T);
        for (int t = 0; t < T; ++t) {
            in[t] = src[t].data();
            out[t] = dst[t].data();
        }
        std::vector<int32_t> sizes(T, p);
        std::vector<double> lam(T);
        for (int mode : {FV_TRANSFER_PIPELINED, FV_TRANSFER_STAGED, FV_TRANSFER_PER_PATCH}) {
            fv_transfer_config cfg{};
            cfg.mode = mode;
            cfg.chunk_bytes = 1 << 20;
            cfg.host_threads = 4;
            fv_transfer_stats ts;
            OK(fv_host_patches_update(in.data(), out.data(), sizes.data(), T, dim, 5, 1e-3, 0.02, 1.4, 0, lam.data(),
                                      &cfg, &ts));
        }
        void *blk_in = nullptr, *blk_out = nullptr;
        OK(fv_host_alloc(T * pd * sizeof(double), &blk_in));
        OK(fv_host_alloc(T * pd * sizeof(double), &blk_out));
        for (int t = 0; t < T; ++t) {
            in[t] = static_cast<double *>(blk_in) + t * pd;
            out[t] = static_cast<double *>(blk_out) + t * pd;
        }
        fv_transfer_config z{};
        z.mode = FV_TRANSFER_ZERO_COPY;
        z.chunk_bytes = 1 << 20;
        OK(fv_host_patches_update(in.data(), out.data(), sizes.data(), T, dim, 5, 1e-3, 0.02, 1.4, FV_HALO_PERIODIC,
                                  nullptr, &z, nullptr));
        OK(fv_host_free(blk_in));
        OK(fv_host_free(blk_out));
        FAILS(fv_host_free(out[0] + 1), FV_ERR_INVALID_ARG);
    }
}

void tuning() {
    std::puts("scenario: tuning tables");
    fv_tuning t{FV_KERNEL_WAVE, 128, 3, 8};
    OK(fv_set_tuning(2, 5, 12, &t));
    OK(fv_get_tuning(2, 5, 12, &t));
    OK(fv_set_tuning(2, 5, 12, nullptr));
    fv_tuning bad{FV_KERNEL_FIXED, 0, 0, 0};
    FAILS(fv_set_tuning(2, 5, 12, &bad), FV_ERR_UNSUPPORTED);
}

}  // namespace

int main() {
    std::printf("library %d, build %s\n", fv_version(), fv_build_id());
    plain_updates();
    noalloc_updates();
    concurrent_updates();
    pde_updates();
    plans();
    flavour_matrix();
    serving();
    meshes();
    transfers();
    tuning();
    std::printf("ok: %d checked calls\n", g_calls.load());
    return 0;
}
