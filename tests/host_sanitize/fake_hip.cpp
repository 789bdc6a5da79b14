// fake_hip.cpp -- a CPU stand-in for the HIP runtime calls the library makes,
// for running the library's host code (validation, descriptor building, plans,
// graph assembly, the serving loop, the transfer pipeline) under AddressSanitizer
// and UndefinedBehaviorSanitizer without a GPU.  It is test infrastructure: it
// is linked only into the sanitizer driver, never into the library.
//
// "Device" memory is host memory from malloc (so the sanitizer tracks it).
// Kernels do not run: a launch only checks its configuration and that every
// pointer argument is null or points into live memory the runtime handed out
// (device, pinned host, or a static device variable's address).  Argument types
// come from the kernel's mangled name, registered by the library's module
// constructor.  Graphs record their kernel nodes' pointer arguments; freeing an
// allocation that a live graph executable refers to is reported, and so is a
// graph launch or a launch whose pointers lead into freed memory.  A memset
// recorded into a graph under stream capture is reported too.  Streams and
// events are objects whose use after destruction the sanitizer sees; every
// enqueued operation completes at once.  Any violation prints a message and
// the stack and aborts.
#include <atomic>
#include <cxxabi.h>
#include <hip/hip_runtime_api.h>
#include <sanitizer/common_interface_defs.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

std::atomic<long> g_alloc_calls{0};
std::atomic<int> g_launch_sleep_us{0};  // a pause at the start of every launch (widens race windows)

// Every registry is constructed on first use and never destroyed: the library's
// module constructors register kernels before this file's static objects would
// be initialised.
std::recursive_mutex &mu() {
    static auto *m = new std::recursive_mutex();
    return *m;
}
#define g_mu mu()

[[noreturn]] void violation(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void violation(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "FAKE-HIP VIOLATION: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
    __sanitizer_print_stack_trace();
    std::abort();
}

enum class Kind { Device, Host, Symbol };

struct Alloc {
    size_t size;
    Kind kind;
};
std::map<uintptr_t, Alloc> &live_map() {  // start -> allocation
    static auto *m = new std::map<uintptr_t, Alloc>();
    return *m;
}
std::vector<std::pair<uintptr_t, uintptr_t>> &dead_ranges() {  // freed ranges (recent)
    static auto *v = new std::vector<std::pair<uintptr_t, uintptr_t>>();
    return *v;
}
#define g_live live_map()
#define g_dead dead_ranges()

// Live allocation containing p, or null.
const std::pair<const uintptr_t, Alloc> *live_at(uintptr_t p) {
    auto it = g_live.upper_bound(p);
    if (it == g_live.begin()) return nullptr;
    --it;
    return p < it->first + std::max<size_t>(it->second.size, 1) ? &*it : nullptr;
}

bool was_freed(uintptr_t p) {
    for (auto it = g_dead.rbegin(); it != g_dead.rend(); ++it)
        if (p >= it->first && p < it->second) return true;
    return false;
}

// ----------------------------------------------------------------- kernels
struct KernelInfo {
    std::string name;
    std::vector<bool> is_pointer;  // per parameter
    int max_dynamic_lds = 64 * 1024;
};
std::map<const void *, KernelInfo> &kernel_map() {  // host stub -> info
    static auto *m = new std::map<const void *, KernelInfo>();
    return *m;
}
std::map<const void *, void *> &symbol_map() {  // host shadow of a static device variable -> its memory
    static auto *m = new std::map<const void *, void *>();
    return *m;
}
#define g_kernels kernel_map()
#define g_symbols symbol_map()

// Parameter types of a demangled signature "ret ns::name<...>(T1, T2, ...)".
std::vector<bool> pointer_params(const std::string &sig) {
    std::vector<bool> out;
    if (sig.empty() || sig.back() != ')') return out;
    int depth = 0;
    size_t open = std::string::npos;
    for (size_t i = sig.size(); i-- > 0;) {
        const char c = sig[i];
        if (c == ')') ++depth;
        if (c == '(' && --depth == 0) {
            open = i;
            break;
        }
    }
    if (open == std::string::npos) return out;
    const std::string params = sig.substr(open + 1, sig.size() - open - 2);
    if (params.empty() || params == "void") return out;
    std::string cur;
    depth = 0;
    auto push = [&](std::string t) {
        while (!t.empty() && t.back() == ' ') t.pop_back();
        for (const char *suffix : {" __restrict", " restrict", " const"}) {
            const size_t n = std::strlen(suffix);
            while (t.size() >= n && t.compare(t.size() - n, n, suffix) == 0) {
                t.resize(t.size() - n);
                while (!t.empty() && t.back() == ' ') t.pop_back();
            }
        }
        out.push_back(!t.empty() && t.back() == '*');
    };
    for (char c : params) {
        if (c == '<' || c == '(' || c == '[' || c == '{') ++depth;
        if (c == '>' || c == ')' || c == ']' || c == '}') --depth;
        if (c == ',' && depth == 0) {
            push(cur);
            cur.clear();
        } else {
            cur.push_back(c);
        }
    }
    push(cur);
    return out;
}

const KernelInfo &kernel(const void *f) {
    auto it = g_kernels.find(f);
    if (it == g_kernels.end()) violation("launch of an unregistered kernel %p", f);
    return it->second;
}

// Pointer argument values of a launch (args[i] points at argument i).
std::vector<uintptr_t> pointer_args(const KernelInfo &k, void **args) {
    std::vector<uintptr_t> v;
    for (size_t i = 0; i < k.is_pointer.size(); ++i) {
        if (!k.is_pointer[i]) continue;
        uintptr_t p = 0;
        std::memcpy(&p, args[i], sizeof p);
        v.push_back(p);
    }
    return v;
}

void check_pointers(const KernelInfo &k, const std::vector<uintptr_t> &ptrs, const char *what) {
    for (uintptr_t p : ptrs) {
        if (!p) continue;
        if (live_at(p)) continue;
        if (was_freed(p)) violation("%s of %s: pointer argument %p leads into freed memory", what, k.name.c_str(),
                                    (void *)p);
        violation("%s of %s: pointer argument %p is not memory the runtime handed out", what, k.name.c_str(),
                  (void *)p);
    }
}

void check_config(const KernelInfo &k, dim3 grid, dim3 block, size_t shmem) {
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) violation("launch of %s with an empty grid", k.name.c_str());
    if (block.x == 0 || block.y == 0 || block.z == 0 || (size_t)block.x * block.y * block.z > 1024)
        violation("launch of %s with block %ux%ux%u", k.name.c_str(), block.x, block.y, block.z);
    if (grid.x > 0x7fffffffu) violation("launch of %s with grid.x %u", k.name.c_str(), grid.x);
    if (shmem > (size_t)k.max_dynamic_lds)
        violation("launch of %s with %zu bytes of dynamic LDS, above its limit %d", k.name.c_str(), shmem,
                  k.max_dynamic_lds);
}

// ----------------------------------------------------------------- streams, events, graphs
struct Graph;
struct Stream {
    unsigned magic = 0x5757;
    Graph *capture = nullptr;
};
struct Event {
    unsigned magic = 0xe7e7;
    bool recorded = false;
};
struct Node {
    const KernelInfo *k = nullptr;  // null: a memory node
    std::vector<uintptr_t> ptrs;
};
struct Graph {
    std::vector<Node> nodes;
};
struct Exec {
    std::vector<Node> nodes;
};
std::map<Exec *, bool> &exec_map() {  // live executables
    static auto *m = new std::map<Exec *, bool>();
    return *m;
}
#define g_execs exec_map()

Stream *stream_of(hipStream_t s) {
    if (!s) return nullptr;
    Stream *st = reinterpret_cast<Stream *>(s);
    if (st->magic != 0x5757) violation("not a stream: %p", (void *)s);
    return st;
}

struct CallConfig {
    dim3 grid, block;
    size_t shmem;
    hipStream_t stream;
};
thread_local std::vector<CallConfig> t_config;
thread_local hipError_t t_last = hipSuccess;

int g_device = 0;
constexpr int kDevices = 1;

}  // namespace

extern "C" {

// ----------------------------------------------------------------- module registration
void **__hipRegisterFatBinary(const void *) {
    static void *handle[1];
    return handle;
}
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *hostFunction, char *, const char *deviceName, unsigned int, void *,
                           void *, void *, void *, int *) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    int status = 0;
    char *dem = abi::__cxa_demangle(deviceName, nullptr, nullptr, &status);
    KernelInfo k;
    k.name = status == 0 && dem ? dem : deviceName;
    if (status != 0) violation("cannot demangle kernel name %s", deviceName);
    k.is_pointer = pointer_params(k.name);
    std::free(dem);
    g_kernels[hostFunction] = k;
}
void __hipRegisterVar(void **, void *var, char *, const char *, int, size_t size, int, int) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    // the device copy of a static device variable: memory of its own, handed out by
    // hipGetSymbolAddress (the host shadow `var` itself is not device memory)
    void *dev = std::calloc(1, size ? size : 1);
    g_live[reinterpret_cast<uintptr_t>(dev)] = Alloc{size, Kind::Symbol};
    g_symbols[var] = dev;
}
hipError_t hipGetSymbolAddress(void **devPtr, const void *symbol) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    auto it = g_symbols.find(symbol);
    if (it == g_symbols.end()) return hipErrorInvalidSymbol;
    *devPtr = it->second;
    return hipSuccess;
}

hipError_t __hipPushCallConfiguration(dim3 gridDim, dim3 blockDim, size_t sharedMem, hipStream_t stream) {
    t_config.push_back(CallConfig{gridDim, blockDim, sharedMem, stream});
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *gridDim, dim3 *blockDim, size_t *sharedMem, hipStream_t *stream) {
    if (t_config.empty()) violation("__hipPopCallConfiguration without a pushed configuration");
    const CallConfig c = t_config.back();
    t_config.pop_back();
    *gridDim = c.grid;
    *blockDim = c.block;
    *sharedMem = c.shmem;
    *stream = c.stream;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void *f, dim3 grid, dim3 block, void **args, size_t shmem, hipStream_t stream) {
    if (const int us = g_launch_sleep_us.load()) std::this_thread::sleep_for(std::chrono::microseconds(us));
    std::lock_guard<std::recursive_mutex> g(g_mu);
    const KernelInfo &k = kernel(f);
    check_config(k, grid, block, shmem);
    const std::vector<uintptr_t> ptrs = pointer_args(k, args);
    check_pointers(k, ptrs, "launch");
    Stream *st = stream_of(stream);
    if (st && st->capture) st->capture->nodes.push_back(Node{&k, ptrs});
    return hipSuccess;
}

hipError_t hipFuncSetAttribute(const void *f, hipFuncAttribute attr, int value) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    auto it = g_kernels.find(f);
    if (it == g_kernels.end()) return hipErrorInvalidDeviceFunction;
    if (attr == hipFuncAttributeMaxDynamicSharedMemorySize) {
        if (value < 0 || value > 160 * 1024) return hipErrorInvalidValue;
        it->second.max_dynamic_lds = value;
    }
    return hipSuccess;
}

hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *numBlocks, const void *f, int blockSize, size_t) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    if (g_kernels.find(f) == g_kernels.end()) return hipErrorInvalidDeviceFunction;
    *numBlocks = blockSize > 0 ? std::max(1, 2048 / blockSize) : 0;
    return hipSuccess;
}

// ----------------------------------------------------------------- device
hipError_t hipGetDeviceCount(int *n) {
    *n = kDevices;
    return hipSuccess;
}
hipError_t hipGetDevice(int *d) {
    *d = g_device;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) {
    if (d < 0 || d >= kDevices) return hipErrorInvalidDevice;
    g_device = d;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *prop, int d) {
    if (d < 0 || d >= kDevices) return hipErrorInvalidDevice;
    std::memset(prop, 0, sizeof *prop);
    std::snprintf(prop->name, sizeof prop->name, "fake MI355X");
    std::snprintf(prop->gcnArchName, sizeof prop->gcnArchName, "gfx950:sramecc+:xnack-");
    prop->multiProcessorCount = 256;
    prop->maxThreadsPerBlock = 1024;
    prop->warpSize = 64;
    prop->sharedMemPerBlock = 160 * 1024;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *value, hipDeviceAttribute_t attr, int d) {
    if (d < 0 || d >= kDevices) return hipErrorInvalidDevice;
    switch (attr) {
        case hipDeviceAttributeMaxSharedMemoryPerBlock: *value = 160 * 1024; break;
        case hipDeviceAttributeMultiprocessorCount: *value = 256; break;
        case hipDeviceAttributeMaxThreadsPerBlock: *value = 1024; break;
        case hipDeviceAttributeWarpSize: *value = 64; break;
        default: *value = 0; break;
    }
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipGetLastError(void) {
    const hipError_t e = t_last;
    t_last = hipSuccess;
    return e;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake runtime error"; }

// ----------------------------------------------------------------- memory
static hipError_t fake_alloc(void **ptr, size_t size, Kind kind) {
    g_alloc_calls.fetch_add(1);
    if (!ptr) return hipErrorInvalidValue;
    void *p = std::aligned_alloc(256, ((size ? size : 1) + 255) / 256 * 256);
    if (!p) return hipErrorOutOfMemory;
    std::lock_guard<std::recursive_mutex> g(g_mu);
    g_live[reinterpret_cast<uintptr_t>(p)] = Alloc{size, kind};
    *ptr = p;
    return hipSuccess;
}
static hipError_t fake_free(void *p, Kind kind) {
    if (!p) return hipSuccess;
    std::lock_guard<std::recursive_mutex> g(g_mu);
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    auto it = g_live.find(a);
    if (it == g_live.end()) violation("free of %p, which is not the start of a live allocation", p);
    if (it->second.kind != kind) violation("free of %p with the wrong call (device vs pinned host)", p);
    const uintptr_t end = a + std::max<size_t>(it->second.size, 1);
    for (const auto &e : g_execs)
        for (const Node &n : e.first->nodes)
            for (uintptr_t q : n.ptrs)
                if (q >= a && q < end)
                    violation("free of %p while a live graph executable refers to it (node %s)", p,
                              n.k ? n.k->name.c_str() : "<memory node>");
    g_live.erase(it);
    g_dead.emplace_back(a, end);
    if (g_dead.size() > 4096) g_dead.erase(g_dead.begin(), g_dead.begin() + 2048);
    std::free(p);
    return hipSuccess;
}
hipError_t hipMalloc(void **ptr, size_t size) { return fake_alloc(ptr, size, Kind::Device); }
hipError_t hipFree(void *p) {
    g_alloc_calls.fetch_add(1);
    return fake_free(p, Kind::Device);
}
hipError_t hipHostMalloc(void **ptr, size_t size, unsigned int) { return fake_alloc(ptr, size, Kind::Host); }
hipError_t hipHostFree(void *p) {
    g_alloc_calls.fetch_add(1);
    return fake_free(p, Kind::Host);
}
// calls of the allocation and free routines so far (the driver checks that the
// no-allocation entry point makes none)
long fake_hip_alloc_calls() { return g_alloc_calls.load(); }
void fake_hip_set_launch_sleep_us(int us) { g_launch_sleep_us.store(us); }
hipError_t hipHostGetDevicePointer(void **devPtr, void *hstPtr, unsigned int) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    const auto *a = live_at(reinterpret_cast<uintptr_t>(hstPtr));
    if (!a || a->second.kind != Kind::Host) return hipErrorInvalidValue;
    *devPtr = hstPtr;
    return hipSuccess;
}

static void check_copy_range(const void *p, size_t n, const char *what) {
    // device-side ranges must lie in one allocation; host ranges are the sanitizer's to check
    std::lock_guard<std::recursive_mutex> g(g_mu);
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    const auto *al = live_at(a);
    if (!al) return;  // host memory (pageable): the sanitizer checks the copy itself
    if (a + n > al->first + al->second.size)
        violation("%s: %zu bytes at %p run past the end of their allocation", what, n, p);
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
    check_copy_range(dst, n, "hipMemcpy destination");
    check_copy_range(src, n, "hipMemcpy source");
    std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s) {
    Stream *st = stream_of(s);
    if (st && st->capture) {
        std::lock_guard<std::recursive_mutex> g(g_mu);
        st->capture->nodes.push_back(Node{nullptr, {reinterpret_cast<uintptr_t>(dst), reinterpret_cast<uintptr_t>(src)}});
    }
    return hipMemcpy(dst, src, n, k);
}
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t s) {
    Stream *st = stream_of(s);
    if (st && st->capture) violation("hipMemsetAsync recorded into a graph under stream capture");
    check_copy_range(dst, n, "hipMemsetAsync");
    std::memset(dst, v, n);
    return hipSuccess;
}

// ----------------------------------------------------------------- streams and events
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    *s = reinterpret_cast<hipStream_t>(new Stream());
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    Stream *st = stream_of(s);
    if (st && st->capture) violation("stream destroyed while capturing");
    st->magic = 0;
    delete st;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    Stream *st = stream_of(s);
    if (st && st->capture) violation("hipStreamSynchronize on a capturing stream");
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    Stream *st = stream_of(s);
    if (!st) return hipErrorInvalidValue;  // the null stream cannot be captured
    if (st->capture) violation("nested stream capture");
    st->capture = new Graph();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *graph) {
    Stream *st = stream_of(s);
    if (!st || !st->capture) return hipErrorIllegalState;
    *graph = reinterpret_cast<hipGraph_t>(st->capture);
    st->capture = nullptr;
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int) {
    *e = reinterpret_cast<hipEvent_t>(new Event());
    return hipSuccess;
}
static Event *event_of(hipEvent_t e) {
    Event *ev = reinterpret_cast<Event *>(e);
    if (!ev || ev->magic != 0xe7e7) violation("not an event: %p", (void *)e);
    return ev;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    Event *ev = event_of(e);
    ev->magic = 0;
    delete ev;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    Event *ev = event_of(e);
    Stream *st = stream_of(s);
    if (st && st->capture) violation("event recorded on a capturing stream");
    ev->recorded = true;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int flags) {
    Event *ev = event_of(e);
    stream_of(s);
    if (flags != 0) violation("hipStreamWaitEvent flags %u", flags);
    if (!ev->recorded) violation("stream waits for an event that was never recorded");
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    event_of(e);
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    event_of(e);
    return hipSuccess;
}

// ----------------------------------------------------------------- graphs
hipError_t hipGraphCreate(hipGraph_t *g, unsigned int) {
    *g = reinterpret_cast<hipGraph_t>(new Graph());
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete reinterpret_cast<Graph *>(g);
    return hipSuccess;
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t *node, hipGraph_t graph, const hipGraphNode_t *, size_t,
                                 const hipKernelNodeParams *p) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    const KernelInfo &k = kernel(p->func);
    check_config(k, p->gridDim, p->blockDim, p->sharedMemBytes);
    Node n{&k, pointer_args(k, p->kernelParams)};
    check_pointers(k, n.ptrs, "graph node");
    Graph *gr = reinterpret_cast<Graph *>(graph);
    gr->nodes.push_back(n);
    *node = reinterpret_cast<hipGraphNode_t>(gr->nodes.size());  // an opaque non-null handle
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t graph, hipGraphNode_t *, char *, size_t) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    Exec *e = new Exec();
    e->nodes = reinterpret_cast<Graph *>(graph)->nodes;
    g_execs[e] = true;
    *exec = reinterpret_cast<hipGraphExec_t>(e);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    Exec *e = reinterpret_cast<Exec *>(exec);
    if (!g_execs.count(e)) violation("launch of a graph executable that does not exist");
    Stream *st = stream_of(s);
    if (st && st->capture) violation("graph launched into a capture");
    for (const Node &n : e->nodes)
        if (n.k) check_pointers(*n.k, n.ptrs, "graph launch");
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
    std::lock_guard<std::recursive_mutex> g(g_mu);
    Exec *e = reinterpret_cast<Exec *>(exec);
    if (!g_execs.erase(e)) violation("destroy of a graph executable that does not exist");
    delete e;
    return hipSuccess;
}

}  // extern "C"
