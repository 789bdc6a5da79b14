// fv_internal.h -- library-private declarations shared by the host ABI code and
// the kernel launchers (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fv {

// Face neighbours and per-patch step data of a patch mesh (the mesh form of
// the fixed-size kernels: face halos are read from the neighbouring patches'
// interiors, every patch has its own dt and h).  Null in the batch forms.
struct MeshArgs {
    const int32_t *neighbors = nullptr;  // device [T][2 dim]: patch across face (axis a, side s) at 2a + s, or -1
    const double *dt = nullptr;          // device [T]
    const double *h = nullptr;           // device [T]
};

// One launch of the patch-update kernel over `num_items` patches of one size.
struct UpdateLaunch {
    const double *in = nullptr;
    double *out = nullptr;
    const int64_t *offsets = nullptr;  // device [num_items] or null: item * stride
    const int64_t *out_offsets = nullptr;  // device [num_items] or null: output at the input offsets
    const int32_t *ids = nullptr;      // device [num_items] or null: lambda index = item
    int32_t num_items = 0;
    int32_t p = 0;                     // interior volumes per axis
    int32_t dim = 2;
    int32_t nq = 5;
    int64_t stride = 0;                // doubles per patch when offsets == null
    double r = 0.0;                    // dt / h
    const double *r_dev = nullptr;     // device dt / h (overrides r when set: device-side time step)
    double gamma = 1.4;
    uint32_t flags = 0;
    double *lambda_out = nullptr;      // device [max id + 1] or null
    int32_t block = 0;                 // threads per block, 0 = default choice
    int32_t kernel = 0;                // FV_KERNEL_* of include/fvpatch.h, 0 = default choice
    int32_t prefetch = 0;              // rows in flight per lane (2D wave kernel), 0 = default
    bool vec2 = false;                 // every patch (and both buffers) 16-byte aligned: 16-byte loads
    int32_t rows = 0;                  // output rows staged per flush (2D wave kernel), 0 = default
    MeshArgs mesh;                     // set: the mesh form (fixed-size kernels only)
    int32_t pde = 0;                   // kPde*: 0 = Euler (every kernel); others: the generic block kernel
    double pde_prm[4] = {0.0, 0.0, 0.0, 0.0};  // the PDE's parameters (Euler: gamma above)
    double dt = 0.0;                   // step size for source terms (with r = dt / h)
};

// PDEs of the generic kernel (the FV_PDE_* values of include/fvpatch.h).
constexpr int32_t kPdeEuler = 0;
constexpr int32_t kPdeShallowWater = 1;
constexpr int32_t kPdeAdvection = 2;
constexpr int32_t kPdeAcoustics = 3;
constexpr int32_t kPdeAcousticsNcp = 4;

// One wave's work in a task-list launch: `count` (<= 64 / (p + 2)) patches of
// size p, at entries first .. first + count - 1 of the offsets / ids lists;
// `rows` output rows are staged per flush, or rows == 0 for the fixed-size
// form (its own rows).
struct WaveTask {
    int32_t p;
    int32_t rows;
    int32_t first;
    int32_t count;
};

// One task-list launch of the 2D wave kernel over mixed patch sizes.
struct TaskLaunch {
    const double *in = nullptr;
    double *out = nullptr;
    const int64_t *offsets = nullptr;  // device, sorted into tasks
    const int64_t *out_offsets = nullptr;  // device, output offsets in the same order (null: same as input)
    const int32_t *ids = nullptr;      // device, lambda index of each entry
    const WaveTask *tasks = nullptr;   // device [num_tasks]
    int32_t num_tasks = 0;
    int32_t nq = 5;
    int32_t ring_words = 0;            // LDS doubles per wave (max over the tasks' sizes)
    int32_t prefetch = 0;
    bool vec2 = false;
    bool persistent = true;            // grid of resident waves looping over the tasks
    double r = 0.0;
    const double *r_dev = nullptr;
    double gamma = 1.4;
    uint32_t flags = 0;
    double *lambda_out = nullptr;
};

// Lanes one patch occupies (its cross-section plane including halo volumes).
inline int plane_lanes(int p, int dim) { return dim == 2 ? (p + 2) : (p + 2) * (p + 2); }

// Default block size: the multiple of 64 in [lanes, 1024] with the best lane
// utilisation, smallest first among equals.
int default_block(int p, int dim);

// Dynamic LDS bytes a block of `block` threads needs.
size_t update_lds_bytes(int dim, int nq, int block);

// Enqueue one update launch; returns hipSuccess or the launch error.
hipError_t launch_update(const UpdateLaunch &L, hipStream_t stream);
// LDS of the generic kernel's smallest block for one patch of size p of a PDE (kPde*).
size_t pde_min_lds_bytes(int pde, int dim, int p);
// The 2D wave form for the PDEs other than Euler (at the fixed sizes p = 3, 5, 9, 16, 17).
bool pde_wave_fits(int pde, int dim, int p);
hipError_t launch_update2d_pde(const UpdateLaunch &L, hipStream_t stream);
// The interior-mapped 3D form for advection and acoustics (built for p = 4, 8).
bool pde3d_fits(int pde, int dim, int p);
hipError_t launch_update3d_pde(const UpdateLaunch &L, hipStream_t stream);

// 2D kernel with each padded patch row inside one wavefront (p + 2 <= 64).
bool wave2d_fits(int p);
size_t wave2d_lds_bytes(int p, int nq, int block, int rows);
int wave2d_ring_words(int p, int nq, int rows);
hipError_t launch_update2d(const UpdateLaunch &L, hipStream_t stream);
hipError_t launch_update2d_tasks(const TaskLaunch &T, hipStream_t stream);
// Fixed-size form of the same kernel (compile-time patch size; N = 5 and
// p in {3, 5, 9, 16, 17}).
bool wave2d_fixed(int p, int nq);
// The 2D fixed-size kernel for p with rows of an odd number of doubles: its vec2 form needs only a
// 16-byte aligned output buffer, whatever the patches' offsets (p = 17 writes whole rows in 16-byte
// pairs; p = 3, 5, 9 ignore vec2).
inline bool fixed_odd_rows(int dim, int p, int nq) { return dim == 2 && wave2d_fixed(p, nq) && ((p + 2) * nq) % 2 == 1; }
// LDS words per wave of a fixed-size body in the task-list launch; whole_rows: the launch writes
// whole output rows (periodic halo or FV_HALO_FROM_IN), else interior-only rows.
int wave2d_fixed_ring_words(int p, bool whole_rows);
void wave2d_fixed_shape(int p, int *prefetch, int *rows);
int wave2d_fixed_block();
// 3D kernel with a patch's cross-section in one wavefront (compile-time
// p in {4, 6, 8}, N = 5; one wave per block).
bool wave3d_fixed(int p, int nq);
void wave3d_fixed_shape(int p, int *prefetch, int *rows);
hipError_t launch_update3d_fixed(const UpdateLaunch &L, hipStream_t stream);
hipError_t launch_update2d_fixed(const UpdateLaunch &L, hipStream_t stream);

// 2D kernel with whole patches per block, one thread per interior volume (p*p <= 1024).
inline bool tile2d_fits(int p) { return p * p <= 1024; }
int tile2d_default_block(int p);
size_t tile2d_lds_bytes(int p, int nq, int G);
int tile2d_patches_per_block(int p, int nq, int block, size_t lds_limit);
hipError_t launch_update2d_tile(const UpdateLaunch &L, hipStream_t stream);

// dt_next = cfl h / (dim max lambda) and r_next = dt_next / h, on the device.
// `slot` (max bits) and `done` (block counter) must be zero before the first launch; each launch
// leaves them zero.
hipError_t launch_next_dt(const double *lambda, int32_t n, double cfl, double h, int32_t dim, double *dt_out,
                          double *r_out, unsigned long long *slot, unsigned int *done, hipStream_t stream);
// r = dt / h on the device.
hipError_t launch_ratio(const double *dt, double h, double *r_out, hipStream_t stream);

}  // namespace fv
