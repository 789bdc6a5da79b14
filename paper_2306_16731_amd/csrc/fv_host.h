// fv_host.h -- library-private host helpers shared by the ABI, plan and
// serving code (validation, error reporting, per-device context).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvpatch.h"

namespace fv {

struct BatchShape {
    bool contiguous = false;  // offsets == NULL
    int32_t uniform_p = -1;   // common interior size, -1 if mixed
    int64_t lo = 0, hi = 0;   // extent of the batch in doubles
};

// Record an error detail for fv_last_error() and return `s`.
fv_status fail(fv_status s, const char *fmt, ...);
void clear_error();

int max_p(int dim);
int64_t patch_doubles(int p, int dim, int nq);

fv_status check_scalars(int32_t dim, int32_t nq, double dt, double h, double gamma, uint32_t flags);
fv_status check_batch(const double *in, const double *out, const int32_t *sizes, const int64_t *offsets,
                      int32_t num_patches, int32_t dim, int32_t nq, const double *lambda_out, BatchShape *shape);
// sizes / offsets only: ranges, bounds, overlaps between patches
fv_status check_layout(const int32_t *sizes, const int64_t *offsets, int32_t num_patches, int32_t dim, int32_t nq,
                       BatchShape *shape);
// device buffers over the extent [lo, hi) of a validated layout
fv_status check_buffers(const double *in, const double *out, const double *lambda_out, int32_t num_patches,
                        int64_t lo, int64_t hi);

struct UpdateLaunch;
// Launch parameters installed for a patch class (or the defaults), and their
// application to a launch.
fv_tuning tuning_for(int dim, int nq, int p);
void apply_tuning(UpdateLaunch &L);

// A PDE other than Euler for the generic block kernel: its FV_PDE_* id and
// parameters as the kernel takes them.
struct PdeArgs {
    int32_t pde = 0;
    double prm[4] = {0.0, 0.0, 0.0, 0.0};
};

// Plain per-batch launch on validated arguments (out_offsets: optional host
// array of output offsets; NULL = output at the input offsets; pde: NULL =
// the Euler equations with `gamma`, else the generic kernel for that PDE).
fv_status plain_update(const double *in, double *out, const int32_t *sizes, const int64_t *offsets, int32_t T,
                       int32_t dim, int32_t nq, double dt, double h, double gamma, uint32_t flags, double *lambda_out,
                       hipStream_t stream, const BatchShape &shape, const int64_t *out_offsets,
                       const PdeArgs *pde = nullptr);

struct DeviceContext;
// Context of the current HIP device; FV_ERR_NO_DEVICE / FV_ERR_UNSUPPORTED
// when there is none or it is not a gfx950.
fv_status current_context(DeviceContext **out);

}  // namespace fv
