/*
 * fvpatch.h -- C ABI of the MI355X (gfx950) Finite Volume patch-update library.
 *
 * The library advances a batch of T small, halo-padded Cartesian patches by
 * one explicit Euler time step of the Rusanov Finite Volume scheme for the
 * compressible Euler equations, in IEEE FP64, and optionally returns every
 * patch's maximum wave speed of the new solution for the CFL condition.
 *
 * What is computed (paper: "SYCL compute kernels for ExaHyPE",
 * arXiv:2306.16731):
 *   - the conservative update of a volume c (Sec. 2.2, the update formula
 *     and Alg. 1), read as
 *         Q_new(c) = Q(c) + (dt/h) ((D_x + D_y) + D_z),
 *         D_n = Fhat_n(c - e_n/2) - Fhat_n(c + e_n/2);
 *   - the Rusanov flux through a face (Eq. 2), read as
 *         Fhat = 1/2 (F_n(Q_L) + F_n(Q_R)) - 1/2 max(l_n(Q_L), l_n(Q_R)) (Q_R - Q_L);
 *   - the Euler user terms F_n and l_n = lambda_max,n = |u_n| + c (Sec. 2.2,
 *     Sec. 5: B = S = delta = 0), ideal gas p = (gamma-1)(E - |m|^2/(2 rho)),
 *     c = sqrt(gamma p / rho);
 *   - the per-patch maximum eigenvalue of the new solution (end of Sec. 2.2):
 *         lambda_t = max over interior c and axes n < d of l_n(Q_new(c)),
 *     NaN-propagating.
 * Only interior and face-halo volumes are read (the ranges of Alg. 1);
 * corner (2D) and edge/corner (3D) halo volumes never enter the result.
 *
 * Data layout (the kernel's input is N (p+2)^d T doubles including the halo,
 * Sec. 2.3): patch t of interior size p_t starts at double offset offsets[t]
 * of the buffer; its (p_t+2)^d volumes are stored x fastest, then y, then z,
 * each volume holding its N unknowns contiguously (array of structures):
 *     index(t, i, j, k, q) = offsets[t] + ((k (p_t+2) + j) (p_t+2) + i) N + q,
 *     i, j, k in [0, p_t + 1], halo volumes at 0 and p_t + 1.
 * Unknowns: N = 5, Q = (rho, m_x, m_y, m_z, E), in 2D and 3D (in 2D m_z is
 * a passive momentum: advected, no z flux, part of the kinetic energy); or
 * N = 4, Q = (rho, m_x, m_y, E), in 2D (the paper's N = 2 + d).
 *
 * Output: the update writes the new interior volumes of every patch into the
 * output buffer at the SAME offsets.  With FV_HALO_PERIODIC it also writes
 * each patch's face halo as the self-wrap of its new interior (halo 0 takes
 * interior p, halo p+1 takes interior 1, per axis; corners untouched), so the
 * output can be fed straight back as the next step's input.  Other output
 * volumes are not touched (unless FV_HALO_FROM_IN gives the halo volumes
 * over, see below).  Input and output must not overlap (use two buffers and
 * swap them between steps).
 *
 * Memory and ownership: patch and lambda buffers are DEVICE memory owned by
 * the caller; `sizes` and `offsets` are HOST arrays owned by the caller and
 * read during the call only.  The library owns only internal descriptor
 * buffers, plans and servers, freed by their destroy calls.
 *
 * Streams: calls that take `stream` (a hipStream_t; NULL = the null stream)
 * enqueue work on it and return without waiting for the device.  Results are
 * valid once the stream has been synchronised.
 *
 * Errors: every call returns an fv_status.  All argument checks run on the
 * host before any device work is enqueued; on error nothing is enqueued and
 * fv_last_error() returns a human-readable detail (thread-local).  Device
 * faults surface at the caller's next synchronisation, as HIP errors.
 */
#ifndef FVPATCH_H
#define FVPATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fv_status {
    FV_OK = 0,
    FV_ERR_INVALID_ARG = -1, /* null pointer, bad value, bad alignment, size out of range */
    FV_ERR_UNSUPPORTED = -2, /* valid request this build does not implement (dim, N, p, device) */
    FV_ERR_NO_DEVICE = -3,   /* no HIP device visible */
    FV_ERR_LAUNCH = -4,      /* a HIP call failed while enqueueing work */
    FV_ERR_OOM = -5,         /* device or pinned host allocation failed */
    FV_ERR_BUDGET = -6,      /* serving: request exceeds the device-memory budget */
    FV_ERR_OVERLAP = -7      /* buffers or patch ranges overlap */
} fv_status;

/* flags */
#define FV_HALO_PERIODIC 0x2u /* also write the self-wrapped face halo of each output patch */
/* Without FV_HALO_PERIODIC: the caller allows the update to overwrite halo
 * volumes of the output with the input's values at the same positions.  The
 * 2D row-marching kernels (p + 2 <= 64: the default for those sizes) and the
 * 3D kernels built for p = 4 and 8 then write each interior row whole, its
 * two x-halo volumes included, which saves HBM time: partly written cache
 * lines cost more than whole ones.  Every
 * output halo volume is afterwards either untouched or equal to the input's;
 * the interior and lambda are the same as without the flag.  Ignored with
 * FV_HALO_PERIODIC. */
#define FV_HALO_FROM_IN 0x4u

/* Largest interior size per axis this build accepts, per dimension. */
#define FV_MAX_P_2D 64
#define FV_MAX_P_3D 24
/* Every patch lies below this offset (in doubles). */
#define FV_MAX_OFFSET (1LL << 48)

/*
 * fv_patch_batch_update -- one explicit Euler step over a batch of patches
 * (the plain per-batch launch).
 *
 *   patches_in   device, read-only: all input patches (layout above).
 *   patches_out  device: receives the new interior (and the periodic face
 *                halo) of every patch at the same offsets; must not overlap
 *                patches_in over the batch's extent (FV_ERR_OVERLAP).
 *   sizes        host [num_patches]: interior volumes per axis p_t,
 *                1 <= p_t <= FV_MAX_P_2D (2D) / FV_MAX_P_3D (3D).
 *   offsets      host [num_patches]: start of patch t in doubles; every
 *                patch lies in [0, FV_MAX_OFFSET) (2^48 doubles, far beyond
 *                any device's memory; the bound keeps address arithmetic
 *                from wrapping); the patches' ranges must not overlap
 *                (FV_ERR_OVERLAP).  NULL
 *                means contiguous patches, offsets[t] = t (p+2)^d N, and then
 *                every sizes[t] must be equal.
 *   num_patches  T >= 0; T == 0 is a no-op that returns FV_OK.
 *   dim          2 or 3.
 *   unknowns     N: 5 (2D, 3D) or 4 (2D).
 *   dt, h        time step size and mesh width: finite and > 0.
 *   gamma        ratio of specific heats: finite and > 1.
 *   flags        0, FV_HALO_PERIODIC and/or FV_HALO_FROM_IN.
 *   lambda_out   device [num_patches] or NULL: per-patch max eigenvalue of
 *                the new solution; NULL skips the reduction.
 *   stream       hipStream_t or NULL.
 * Pointers must be 8-byte aligned.  The call is re-entrant and may be made
 * from several threads at once: calls on the same device share a ring of
 * pinned descriptor slots, each held by one call from filling to launch and
 * reused after the launches that read it have run (a call waits for a slot
 * when more calls than slots are under way).
 */
fv_status fv_patch_batch_update(const double *patches_in, double *patches_out,
                                const int32_t *sizes, const int64_t *offsets,
                                int32_t num_patches, int32_t dim, int32_t unknowns,
                                double dt, double h, double gamma, uint32_t flags,
                                double *lambda_out, void *stream);

/* Most patches one fv_patch_batch_update_noalloc call takes. */
#define FV_NOALLOC_MAX_PATCHES 262144

/*
 * fv_patch_batch_update_noalloc -- fv_patch_batch_update for callers that
 * cannot allocate memory: code that runs between hipGraph captures, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results
 * (bit for bit) and errors as fv_patch_batch_update, plus:
 *   - num_patches <= FV_NOALLOC_MAX_PATCHES, else FV_ERR_INVALID_ARG before
 *     any device work;
 *   - the call never allocates device or pinned memory (no hipMalloc,
 *     hipHostMalloc or hipFree): patches that are not equal-size and evenly
 *     spaced take their size-sorted descriptors (12 bytes per patch) through
 *     a fixed array of 3 MiB in the library's device image (each GPU the
 *     library runs on holds its own copy until the process ends) and a fixed
 *     host staging array, copied with one hipMemcpyAsync from pageable
 *     memory (so a call may wait for the previous call's copy, which follows
 *     the work queued before it on that stream);
 *   - every call on one GPU shares that array: calls are serialised on the
 *     host, and calls on ONE stream are ordered; calls that overlap on two
 *     streams of one GPU race on the descriptors and give undefined results.
 * The first call on a device also resolves the array's device address and
 * creates one event (set-up work, done once per device).  Not capturable
 * into a hipGraph (the pageable copy).
 */
fv_status fv_patch_batch_update_noalloc(const double *patches_in, double *patches_out,
                                        const int32_t *sizes, const int64_t *offsets,
                                        int32_t num_patches, int32_t dim, int32_t unknowns,
                                        double dt, double h, double gamma, uint32_t flags,
                                        double *lambda_out, void *stream);

/*
 * Launch parameters of the update kernel for one patch class (dim, unknowns,
 * p).  The library picks defaults; the autotuner measures candidates and
 * installs the fastest.  Installed settings are process-wide defaults: they
 * apply to every later plain launch on every device and to plans built
 * afterwards for classes their own tuning table does not cover.
 *
 *   kernel    FV_KERNEL_AUTO, FV_KERNEL_BLOCK (plane-marching kernel, any
 *             size), FV_KERNEL_WAVE (2D only: one padded patch row per
 *             wavefront, p + 2 <= 64), FV_KERNEL_TILE (2D only: whole
 *             patches per block, one thread per interior volume, p*p <= 1024)
 *             or FV_KERNEL_FIXED (a kernel compiled for one patch size,
 *             unknowns = 5: the 2D wave kernel for p in {3, 5, 9, 16, 17},
 *             a 3D kernel with one patch cross-section per wavefront for
 *             3D p in {4, 6, 8}; the default for those classes)
 *   block     threads per block, a multiple of 64 (0 = default); the wave
 *             kernel takes at most 256, the tile kernel at least p*p, the
 *             fixed-size kernel exactly 64
 *   prefetch  rows each lane keeps in flight in the wave kernel, 1..4
 *             (0 = default); set by the build for the fixed-size kernel
 *             (0 or that value)
 *   rows      output rows the wave kernel stages in LDS per patch before
 *             writing them in one burst, 1..16 (0 = default); set by the
 *             build for the fixed-size kernel (0 or that value)
 */
#define FV_KERNEL_AUTO 0
#define FV_KERNEL_BLOCK 1
#define FV_KERNEL_WAVE 2
#define FV_KERNEL_TILE 3
#define FV_KERNEL_FIXED 4

typedef struct fv_tuning {
    int32_t kernel;
    int32_t block;
    int32_t prefetch;
    int32_t rows;
} fv_tuning;

/* Install `tuning` for the class (NULL restores the defaults).  Returns
 * FV_ERR_INVALID_ARG for values out of range, FV_ERR_UNSUPPORTED for a
 * kernel that cannot run the class. */
fv_status fv_set_tuning(int32_t dim, int32_t unknowns, int32_t p, const fv_tuning *tuning);

/* Current parameters of the class (the installed ones, else the defaults). */
fv_status fv_get_tuning(int32_t dim, int32_t unknowns, int32_t p, fv_tuning *tuning);

/*
 * ---- Batching form: plans --------------------------------------------------
 *
 * A plan fixes a batch composition (sizes, offsets) once: it sorts the
 * patches by size, cuts every size class into wave tasks (the fixed-size body
 * for p in {3, 5, 9, 16, 17} with N = 5, else the runtime-size body with the
 * class's tuned rows), and uploads that work list.  Each step is then ONE
 * fused launch over all 2D classes with p + 2 <= 64 -- a persistent grid
 * walking the tasks largest first (default), or one wave per task with the
 * tasks in memory order (FV_PLAN_NO_PERSIST) -- plus one launch per remaining
 * class (3D, or 2D p > 62); FV_PLAN_PER_CLASS launches every class on its own
 * kernel instead.  On large mixed batches one wave per task is the fastest
 * of the three (its fixed-size bodies also keep more rows in flight); the
 * autotuner times the three for a given batch.  Each plan may carry its own
 * tuning table.  The plan
 * also captures k steps, with the time step formed on the device from each
 * step's eigenvalues, into one hipGraph that replays without host round
 * trips.  This is the paper's task fusion of T patch updates into one kernel
 * (Sec. 2.1) with the precompiled task graph it proposes (Sec. 5; outlook, Sec. 6).
 * Plans are single-owner objects; they keep their own device memory.
 */
typedef struct fv_plan fv_plan;

#define FV_PLAN_NO_PERSIST 0x100u /* plan flag: one wave per task instead of a persistent grid */
#define FV_PLAN_PER_CLASS 0x200u  /* plan flag: no fused launch; each size class is launched on its own
                                     kernel, at that kernel's occupancy (the fused launch holds every
                                     wave to the LDS of its largest class) */

typedef struct fv_plan_stats {
    int32_t num_patches;
    int32_t num_tasks;          /* wave tasks of the fused launch */
    int32_t num_class_launches; /* classes launched on their own each step */
    int32_t prefetch;           /* row prefetch of the fused launch (0 = default) */
    int32_t lds_per_wave_bytes; /* LDS a wave of the fused launch uses */
    int32_t persistent;         /* 1: persistent grid */
    int32_t captured_steps;     /* steps in the captured graph, 0 if none */
} fv_plan_stats;

/* Launch parameters for one patch class in a plan's own tuning table. */
typedef struct fv_tune_entry {
    int32_t dim;
    int32_t unknowns;
    int32_t p;
    fv_tuning tuning; /* as for fv_set_tuning */
} fv_tune_entry;

/* Build a plan for the composition (sizes, offsets as for
 * fv_patch_batch_update; offsets NULL = contiguous, equal sizes).  flags:
 * FV_HALO_PERIODIC or FV_HALO_FROM_IN, and FV_PLAN_NO_PERSIST or
 * FV_PLAN_PER_CLASS.
 * tune_table (host [tune_entries], NULL when tune_entries = 0; read during
 * the call only): the plan's own launch parameters per size class, e.g. an
 * autotuner's table.  Entries for another (dim, unknowns) are ignored; each
 * other entry is checked as fv_set_tuning checks its argument (its error is
 * returned), two entries for one p are FV_ERR_INVALID_ARG.  A class without
 * an entry takes the parameters installed by fv_set_tuning at creation time,
 * else the defaults.  The plan keeps what it resolved: fv_set_tuning later,
 * or another plan's table, does not change it (fv_plan_get_tuning reports
 * it).  In the fused launch a class built in the fixed-size form runs that
 * body whatever its tuning; tuning chooses the kernels of per-class launches
 * (FV_PLAN_PER_CLASS, 3D, 2D p > 62) and the rows of runtime-size bodies. */
fv_status fv_plan_create(fv_plan **plan, const int32_t *sizes, const int64_t *offsets, int32_t num_patches,
                         int32_t dim, int32_t unknowns, uint32_t flags, const fv_tune_entry *tune_table,
                         int32_t tune_entries);

/* Launch parameters the plan resolved for its patches of size p
 * (FV_ERR_INVALID_ARG if it has none of that size). */
fv_status fv_plan_get_tuning(const fv_plan *plan, int32_t p, fv_tuning *tuning);

/* One step of every patch of the plan: like fv_patch_batch_update on the
 * plan's composition.  Asynchronous on `stream`.
 * dt_dev: NULL, or a device double holding the step size, read when the step
 * runs (dt is then ignored): a device-side time step, e.g. one a previous
 * kernel derived from the eigenvalues; dt / h is formed on the device,
 * correctly rounded, so the result equals a host dt of the same value bit for
 * bit.  It must not overlap patches_out or lambda_out (FV_ERR_OVERLAP).  The
 * plan holds one device word for dt / h: executes with dt_dev on different
 * streams must not overlap in time. */
fv_status fv_plan_execute(fv_plan *plan, const double *patches_in, double *patches_out, double dt,
                          const double *dt_dev, double h, double gamma, double *lambda_out, void *stream);

/* Capture `steps` steps into a graph: step k reads buf_a (k even) or buf_b
 * (k odd) and writes the other (the result of an even number of steps is in
 * buf_a).  Step 0 uses dt_dev[0], which the caller writes before each replay;
 * after step k the eigenvalues in lambda_out (device [num_patches]) fix
 * dt_dev[k+1] = cfl h / (dim max lambda) on the device (NaN-propagating).
 * dt_dev: device [steps + 1].  `stream` must be a non-null stream; before
 * capturing, the call clears two internal words on `stream` and waits for it.
 * Replaces a previous capture of the plan.  The graph refers to buf_a, buf_b,
 * lambda_out and dt_dev: they must stay allocated until the plan is destroyed
 * or captures again. */
fv_status fv_plan_capture_steps(fv_plan *plan, int32_t steps, double *buf_a, double *buf_b, double h, double gamma,
                                double cfl, double *lambda_out, double *dt_dev, void *stream);

/* Launch the captured graph on `stream`. */
fv_status fv_plan_replay(fv_plan *plan, void *stream);

/* Shape of the plan's work list. */
fv_status fv_plan_info(const fv_plan *plan, fv_plan_stats *info);

/* Wait for the device, then free the plan (NULL is a no-op). */
fv_status fv_plan_destroy(fv_plan *plan);

/*
 * ---- Serving form: a request loop over device-resident patch state --------
 *
 * A mesh traversal hands the kernel batches of patches as it goes (task
 * fusion of enclave tasks, Sec. 2.1).  The server keeps every registered
 * mesh's patch state resident in HBM -- two state slots per patch, each patch
 * ping-ponging on its own -- so no patch data crosses PCIe after registration
 * (the recycled device memory of Sec. 4 "Data transfer", without the copies).
 * Meshes may differ in dimension, unknowns and mesh width (a 2D mesh of mixed
 * patch sizes next to a 3D one): they share the server's stream and budget.
 * A batch names a contiguous range of one mesh's patches and a time step.
 * Batches are admitted in arrival order while the resident bytes plus the
 * bytes of the batches in flight fit `budget_bytes` and fewer than
 * `max_inflight` are running; otherwise they wait (none is dropped).  Each
 * batch's latency runs from its arrival to the moment the loop sees its
 * completion event.  Servers are single-owner objects with their own stream.
 *
 * Failures.  A batch whose completion event reports an error (any status but
 * "not ready") is re-run: its patches' state from before it is still in their
 * input slots (no update writes in place), so the batch is queued first again
 * and writes its output slots anew, up to max_retries times.  When its
 * retries are spent (its patches then keep their state from before it), or
 * when a later batch in flight has already read its output (the state of
 * those patches is lost), fv_server_poll / _drain / _run_trace return
 * FV_ERR_LAUNCH with the detail in fv_last_error(); the server can go on.
 * With deadline_ms > 0 a batch still running that long after its launch makes
 * them return FV_ERR_LAUNCH instead of waiting (the batch stays in flight).
 */
typedef struct fv_server fv_server;

#define FV_SERVE_FUSED 0 /* one fused launch per batch (task list, largest patches first) */
#define FV_SERVE_PLAIN 1 /* each batch through the plain per-batch path (one launch per size class) */

typedef struct fv_server_config {
    int64_t budget_bytes; /* HBM budget for resident state plus in-flight batches */
    double gamma;         /* ratio of specific heats */
    uint32_t flags;       /* 0, FV_HALO_PERIODIC or FV_HALO_FROM_IN */
    int32_t mode;         /* FV_SERVE_FUSED or FV_SERVE_PLAIN */
    int32_t max_inflight; /* batches running at once (0 = 8), at most 1024 */
    int32_t max_retries;  /* re-runs of a batch whose completion reports an error, 0..16 */
    double deadline_ms;   /* > 0: longest a batch may run before poll / drain fail; 0 = none */
} fv_server_config;

typedef struct fv_serve_request {
    int64_t arrival_ns; /* fv_server_run_trace: offset from the start of the run */
    int32_t mesh;
    int32_t first;      /* patch range [first, first + count) of the mesh */
    int32_t count;
    int32_t reserved;
    double dt;
} fv_serve_request;

typedef struct fv_server_stats {
    int64_t submitted, completed, queued, inflight, peak_queued, peak_inflight;
    int64_t cells_updated;  /* interior volumes updated by completed batches */
    int64_t failed;         /* batches given up after errors */
    int64_t retried;        /* re-runs after errors */
    int64_t resident_bytes, budget_bytes;
    double p50_ms, p99_ms, max_ms, mean_ms; /* arrival-to-completion latency of completed batches */
    double cell_updates_per_s;               /* completed cells / (last completion - first arrival) */
} fv_server_stats;

/* One completed batch (fv_server_batch_log); times in ns since the server's creation. */
typedef struct fv_batch_record {
    int64_t ticket;
    int64_t arrival_ns;  /* arrival */
    int64_t launch_ns;   /* its launches were enqueued */
    int64_t done_ns;     /* the loop saw its completion */
    int64_t cells;       /* interior volumes updated */
    int32_t mesh;
    int32_t count;       /* patches */
    int32_t retries;     /* re-runs it took */
    int32_t reserved;
} fv_batch_record;

fv_status fv_server_create(fv_server **server, const fv_server_config *cfg);

/* Register a mesh: num_patches patches of the given sizes in `dim`
 * dimensions with `unknowns` unknowns (as for fv_patch_batch_update) and mesh
 * width h, stored contiguously in host_state (layout as for
 * fv_patch_batch_update with offsets NULL but sizes free to differ); uploads
 * it into both slots.  FV_ERR_BUDGET if its two slots do not fit the budget. */
fv_status fv_server_add_mesh(fv_server *server, int32_t dim, int32_t unknowns, double h, const int32_t *sizes,
                             int32_t num_patches, const double *host_state, int32_t *mesh_id);

/* Queue a batch (arrival_ns <= 0: now, on the server's steady clock in ns).
 * *ticket (optional) receives its ticket: 1, 2, ... in submission order. */
fv_status fv_server_submit(fv_server *server, int32_t mesh_id, int32_t first, int32_t count, double dt,
                           int64_t arrival_ns, int64_t *ticket);

/* Retire finished batches and admit queued ones; never blocks. */
fv_status fv_server_poll(fv_server *server, fv_server_stats *stats);

/* Run every queued batch to completion. */
fv_status fv_server_drain(fv_server *server, fv_server_stats *stats);

/* Replay a trace in the loop: request k is submitted when
 * reqs[k].arrival_ns has elapsed since the call started (arrivals
 * non-decreasing), the loop polling in between; then drains. */
fv_status fv_server_run_trace(fv_server *server, const fv_serve_request *reqs, int64_t n, fv_server_stats *stats);

/* Drain, then copy the mesh's current state into host_state (layout of
 * fv_server_add_mesh). */
fv_status fv_server_read_mesh(fv_server *server, int32_t mesh_id, double *host_state);

fv_status fv_server_stats_get(fv_server *server, fv_server_stats *stats);

/* Records of the completed batches in completion order: the first
 * min(capacity, completed) into `records`; *count = all of them. */
fv_status fv_server_batch_log(fv_server *server, fv_batch_record *records, int64_t capacity, int64_t *count);

/* Test hook for the failure handling (the GPU is never made to fault): the
 * batch with this ticket runs normally, but its completion check reports
 *   FV_INJECT_FAIL  a launch failure, on its next `times` completions (each
 *                   re-run completes once);
 *   FV_INJECT_HANG  "not ready", until the injection is cleared;
 * kind 0 clears the ticket's injection. */
#define FV_INJECT_FAIL 1
#define FV_INJECT_HANG 2
fv_status fv_server_inject(fv_server *server, int64_t ticket, int32_t kind, int32_t times);

/* Wait for the server's stream, then free everything it holds (NULL: no-op). */
fv_status fv_server_destroy(fv_server *server);

/* ------------------------------------------------------------------------
 * Patch mesh: the steps either side of the update (Sec. 2.2).  Before its
 * update every patch is equipped with a halo layer taken from the patches
 * that touch its faces, and after it the patch's maximum eigenvalue sets its
 * own next step size (local time stepping).
 *
 * A mesh is a fixed set of num_patches patches of one size p (layout as in
 * fv_patch_batch_update: sizes / offsets on the host, offsets NULL =
 * contiguous) and a face-neighbour table: neighbors (host, [num_patches *
 * 2 * dim]) holds at t*2*dim + 2*a + s the patch that touches patch t across
 * its face on axis a (0 = x, 1 = y, 2 = z), side s (0: the face at index 0,
 * 1: the face at p+1), or -1 for a face without a neighbour.  The halo
 * layer on side 0 of axis a takes the neighbour's interior layer at p, on
 * side 1 its interior layer at 1, at the same coordinates along the other
 * axes.  Corner / edge halo volumes are never read or written.  The tables
 * are copied to the device at creation; the caller's arrays may be freed.
 * ------------------------------------------------------------------------ */
typedef struct fv_mesh fv_mesh;

/* Validate and upload a mesh.  Errors: FV_ERR_INVALID_ARG (dim, unknowns,
 * num_patches <= 0, sizes, offsets, a neighbour index outside -1 ..
 * num_patches-1), FV_ERR_UNSUPPORTED (patches of different sizes),
 * FV_ERR_OVERLAP (patch ranges overlap), FV_ERR_NO_DEVICE, FV_ERR_OOM. */
fv_status fv_mesh_create(fv_mesh **mesh, const int32_t *sizes, const int64_t *offsets, const int32_t *neighbors,
                         int32_t num_patches, int32_t dim, int32_t unknowns);

/* Write every face halo of `patches` (device) from the neighbours' interiors,
 * in place (only halo volumes are written, only interior volumes read);
 * faces without a neighbour keep their halo.  Any patch size.  Asynchronous
 * on `stream`. */
fv_status fv_mesh_halo_fill(fv_mesh *mesh, double *patches, void *stream);

/* One explicit Euler step of every patch of the mesh, patch t by dt[t] with
 * volumes of width h[t] (dt, h: device arrays [num_patches]); the face halos
 * are read from the neighbours' interiors in patches_in during the update
 * (no separate fill; a face without a neighbour uses the patch's own halo).
 * patches_out gets the new interiors (its halo volumes are not written);
 * lambda_out (device [num_patches] or NULL) the maximum wave speed of each
 * new interior.  Built for 2D p in {3, 5, 9, 16, 17} and 3D p in {4, 6, 8}
 * with 5 unknowns (FV_ERR_UNSUPPORTED otherwise: use fv_mesh_halo_fill and
 * fv_patch_batch_update).  Errors also: FV_ERR_INVALID_ARG (null / unaligned
 * pointers, gamma, another device), FV_ERR_OVERLAP (in / out / lambda / dt /
 * h overlap), FV_ERR_LAUNCH. */
fv_status fv_mesh_step(fv_mesh *mesh, const double *patches_in, double *patches_out, const double *dt,
                       const double *h, double gamma, double *lambda_out, void *stream);

/* Per-patch step sizes for local time stepping: dt_out[t] = cfl * h[t] /
 * (dim * lambda[t]) on the device (all device arrays [num_patches]); the same
 * expression as the global step size, per patch.  num_patches = 0: no-op. */
fv_status fv_local_dt(const double *lambda, const double *h, int32_t num_patches, int32_t dim, double cfl,
                      double *dt_out, void *stream);

/* Wait for the device, then free the mesh's device tables (NULL: no-op). */
fv_status fv_mesh_destroy(fv_mesh *mesh);

/* ------------------------------------------------------------------------
 * Other PDEs: the generic solver of Eq. 1.  The paper's engine assembles its
 * solver from user terms -- flux F_n, non-conservative product
 * B_n(Q) dQ/dx_n, source S, largest wave speed lambda_max,n (Sec. 2.2) -- and
 * this call runs the same step for one of the built-in PDEs, each a set of
 * such terms (a device type in the library's csrc/fv_pde.h; a new PDE is a
 * new type of that shape).  The step, with B read as a central jump at every
 * face (the paper omits its treatment) and S as explicit Euler:
 *   Fhat = 1/2 (F_n(Q_L) + F_n(Q_R)) - 1/2 max(l_n(Q_L), l_n(Q_R)) (Q_R - Q_L)
 *   G+ / G- = Fhat -/+ 1/2 B_n((Q_L + Q_R) / 2) (Q_R - Q_L)
 *   Q_new = Q + (dt/h) sum_n [G+(c - e_n/2) - G-(c + e_n/2)] + dt S(Q)
 * over the evolved unknowns; a PDE's parameter unknowns keep their values.
 *
 *   FV_PDE_EULER           the Euler equations (N = 5); params {gamma}: the
 *                          same as fv_patch_batch_update with unknowns = 5.
 *   FV_PDE_SHALLOW_WATER   2D only.  Q = (h, hu, hv, b), the bathymetry b not
 *                          evolved; F_x = (hu, hu u, hv u), F_y = (hv, hu v,
 *                          hv v); B: the hydrostatic pressure g h d(h+b)/dx_n
 *                          in the n-momentum; S = (0, f hv, -f hu) (Coriolis);
 *                          l_n = |u_n| + sqrt(g h).  params {g > 0, f}.
 *   FV_PDE_ADVECTION       dq/dt + a . grad q = 0, N = 1; params {a_x, a_y,
 *                          a_z} (a_z ignored in 2D).
 *   FV_PDE_ACOUSTICS       linear acoustics, Q = (p, u_1 .. u_d), N = 1 + d:
 *                          F_n = (K0 u_n, p / rho0 e_n), l_n = sqrt(K0 / rho0);
 *                          params {rho0 > 0, K0 > 0}.
 *   FV_PDE_ACOUSTICS_NCP   the same system written as B_n dQ/dx_n with F = 0.
 *
 * Layout, offsets, flags (FV_HALO_PERIODIC; FV_HALO_FROM_IN is accepted and
 * lets the Euler kernels write whole rows), lambda_out (per-patch max of l_n
 * over the new interior), streams and errors as fv_patch_batch_update, with N
 * the PDE's unknowns; params: host [num_params], all finite.  The Euler
 * equations take every tuned kernel; the other PDEs run on the plane-marching
 * kernel (any p up to FV_MAX_P_2D / FV_MAX_P_3D).
 * Errors also: FV_ERR_INVALID_ARG (unknown PDE, wrong num_params, a parameter
 * out of range), FV_ERR_UNSUPPORTED (shallow water in 3D).
 * ------------------------------------------------------------------------ */
#define FV_PDE_EULER 0
#define FV_PDE_SHALLOW_WATER 1
#define FV_PDE_ADVECTION 2
#define FV_PDE_ACOUSTICS 3
#define FV_PDE_ACOUSTICS_NCP 4

/* Unknowns per volume and number of parameters of a PDE in dim dimensions. */
fv_status fv_pde_unknowns(int32_t pde, int32_t dim, int32_t *unknowns, int32_t *num_params);

fv_status fv_pde_batch_update(int32_t pde, const double *params, int32_t num_params, const double *patches_in,
                              double *patches_out, const int32_t *sizes, const int64_t *offsets,
                              int32_t num_patches, int32_t dim, double dt, double h, uint32_t flags,
                              double *lambda_out, void *stream);

/* ------------------------------------------------------------------------
 * The paper's three kernel realisations (Sec. 3) as comparison variants of
 * the fused update: the same step, the same microkernels in the same order
 * per volume (results equal to fv_patch_batch_update's bit for bit), mapped
 * differently onto the GPU:
 *   FV_FLAVOUR_BATCHED     one launch per algorithmic step over all volumes
 *                          of all patches (user terms, face fluxes, update,
 *                          eigenvalue reduction) with HBM temporaries;
 *   FV_FLAVOUR_PATCH_WISE  one work-group per patch, the steps in sequence
 *                          inside it with a barrier between them;
 *   FV_FLAVOUR_TASK_GRAPH  a task per (patch, microkernel): d independent
 *                          face-flux tasks and an update task per patch,
 *                          submitted from the host every call as dependent
 *                          commands (flux tasks on library streams, one per
 *                          axis; each update on `stream` after events from
 *                          its patch's flux tasks); asynchronous like the
 *                          others: the results are valid once `stream` has
 *                          been synchronised.
 * Arguments as fv_patch_batch_update; additionally FV_ERR_UNSUPPORTED
 * unless all patches have one size with at most 512 interior volumes and
 * unknowns = 5.  The batched and task-graph forms keep temporaries in a
 * grow-only device workspace owned by the library (one per device, kept
 * until the process ends, shared by all calls on that device: calls on
 * different streams must not overlap).  With offsets the call waits for its
 * stream once (offset upload).
 * ------------------------------------------------------------------------ */
#define FV_FLAVOUR_BATCHED 1
#define FV_FLAVOUR_PATCH_WISE 2
#define FV_FLAVOUR_TASK_GRAPH 3

fv_status fv_flavour_update(int32_t flavour, const double *patches_in, double *patches_out, const int32_t *sizes,
                            const int64_t *offsets, int32_t num_patches, int32_t dim, int32_t unknowns, double dt,
                            double h, double gamma, uint32_t flags, double *lambda_out, void *stream);

/* ------------------------------------------------------------------------
 * Patches in host memory (Sec. 4, data transfer; Sec. 5, Fig. 4).  In the
 * paper every patch is a separate allocation on the CPU heap, brought to the
 * accelerator one by one; those scattered copies dominate its runtime.  This
 * call takes such patches, moves them through the fused update and writes
 * the results back to host memory:
 *   FV_TRANSFER_PER_PATCH  each patch its own synchronous hipMemcpy to and
 *                          from a recycled device area, one launch over the
 *                          batch in between (the paper's explicit copy with
 *                          device allocations kept, not freed);
 *   FV_TRANSFER_STAGED     host_threads threads gather all patches into one
 *                          pinned buffer, one copy to the device, one launch,
 *                          one copy back, threaded scatter (bulk, no overlap);
 *   FV_TRANSFER_ZERO_COPY  patches in pinned memory from fv_host_alloc (every
 *                          patch, input and output, must lie in such a block;
 *                          FV_ERR_INVALID_ARG otherwise): chunks of about
 *                          chunk_bytes with `slots` in flight on the library's
 *                          streams; per chunk a gather kernel reads the
 *                          patches over PCIe into device memory, the update
 *                          runs, a scatter kernel writes them back; no host
 *                          copies (host_threads unused);
 *   FV_TRANSFER_PIPELINED  the batch cut into chunks of whole patches of about
 *                          chunk_bytes; each of host_threads threads takes
 *                          chunks in turn and carries each through gather into
 *                          pinned staging, hipMemcpyAsync to the device, the
 *                          update, the copy back on the thread's own stream
 *                          and the scatter, keeping `slots` chunks of its own
 *                          in flight: gathers, scatters, both copy directions
 *                          and updates of different chunks overlap.
 * patches_in / patches_out: host arrays [num_patches] of host pointers, patch
 * t a padded AoS patch of sizes[t] (all sizes equal) as in
 * fv_patch_batch_update, in pageable or pinned memory, 8-byte aligned.  The
 * copies into and out of the staging use streaming stores.  patches_out[t]
 * receives the whole patch: the new interior, and halo volumes equal to the
 * input's (FV_HALO_PERIODIC: its face halos wrapped from the new interior).
 * lambda_out: host [num_patches] or NULL.  dt, h, gamma, flags as in
 * fv_patch_batch_update; results equal its results bit for bit.
 * config: NULL = pipelined with the defaults; a 0 field = its default
 * (chunk_bytes 8 MiB, slots 2, host_threads 8; zero copy: 32 MiB, 4 slots).  Pinned staging and device
 * buffers are kept per device, grow-only, until the process ends: pipelined
 * 2 * host_threads * slots chunks of each kind, staged 2 batches of each.
 * stats: NULL or filled on success (bytes moved each way, wall time of the
 * call, host thread time spent gathering and scattering, summed over the
 * threads).  Synchronous: returns when every output is in host memory; the
 * library's streams are its own, none of the caller's is used; calls on one
 * device are serialised.
 * Errors: FV_ERR_INVALID_ARG (scalars, null pointers, config ranges, a chunk
 * smaller than one patch), FV_ERR_UNSUPPORTED (mixed sizes), FV_ERR_OVERLAP
 * (an output patch overlaps an input or another output patch),
 * FV_ERR_NO_DEVICE, FV_ERR_OOM, FV_ERR_LAUNCH (after an error the outputs of
 * some patches may be unwritten).  num_patches = 0: no-op.
 * ------------------------------------------------------------------------ */
#define FV_TRANSFER_PIPELINED 0
#define FV_TRANSFER_PER_PATCH 1
#define FV_TRANSFER_STAGED 2
#define FV_TRANSFER_ZERO_COPY 3
#define FV_TRANSFER_MAX_SLOTS 8
#define FV_TRANSFER_MAX_THREADS 64

typedef struct fv_transfer_config {
    int64_t chunk_bytes;  /* chunk (pipelined, zero copy), >= one patch; 0 = 8 MiB (zero copy 32 MiB) */
    int32_t slots;        /* chunks in flight per thread (pipelined; zero copy: in all), 1 .. FV_TRANSFER_MAX_SLOTS; 0 = 2 (zero copy 4) */
    int32_t host_threads; /* threads incl. the caller's, 1 .. FV_TRANSFER_MAX_THREADS; 0 = 8 */
    int32_t mode;         /* FV_TRANSFER_* */
    int32_t reserved;     /* 0 */
} fv_transfer_config;

typedef struct fv_transfer_stats {
    int64_t bytes_to_device;
    int64_t bytes_to_host;
    double seconds;           /* wall time of the call */
    double host_copy_seconds; /* gathering into / scattering from the staging, summed over threads */
} fv_transfer_stats;

/* Page-locked host memory for patches that the GPU reads and writes in place
 * (FV_TRANSFER_ZERO_COPY): *ptr receives `bytes` (> 0) of host memory,
 * 16-byte aligned, kept until fv_host_free.  Errors: FV_ERR_INVALID_ARG,
 * FV_ERR_NO_DEVICE, FV_ERR_OOM. */
fv_status fv_host_alloc(size_t bytes, void **ptr);

/* Free memory from fv_host_alloc (NULL: no-op; FV_ERR_INVALID_ARG for any other
 * pointer).  No call may be using it. */
fv_status fv_host_free(void *ptr);

fv_status fv_host_patches_update(const double *const *patches_in, double *const *patches_out, const int32_t *sizes,
                                 int32_t num_patches, int32_t dim, int32_t unknowns, double dt, double h,
                                 double gamma, uint32_t flags, double *lambda_out, const fv_transfer_config *config,
                                 fv_transfer_stats *stats);

/* Text for a status code (static storage). */
const char *fv_status_string(fv_status status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char *fv_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t fv_version(void);

/* Identity of the sources the library was built from: a 16-digit hex digest of
 * every source and header (static storage; "unknown" for a build that did not
 * set it).  Lets a loader refuse a library older than its sources. */
const char *fv_build_id(void);

#ifdef __cplusplus
}
#endif

#endif /* FVPATCH_H */
