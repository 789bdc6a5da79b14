// fv_host.h -- library-private host helpers shared by the ABI, plan and
// serving code (validation, error reporting, per-device context).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

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
// sort_buf (optional, sort_cap entries): where the overlap check of unsorted offsets sorts the
// patch ranges; NULL = a temporary vector.
fv_status check_batch(const double *in, const double *out, const int32_t *sizes, const int64_t *offsets,
                      int32_t num_patches, int32_t dim, int32_t nq, const double *lambda_out, BatchShape *shape,
                      std::pair<int64_t, int64_t> *sort_buf = nullptr, int64_t sort_cap = 0);
// sizes / offsets only: ranges, bounds, overlaps between patches
fv_status check_layout(const int32_t *sizes, const int64_t *offsets, int32_t num_patches, int32_t dim, int32_t nq,
                       BatchShape *shape, std::pair<int64_t, int64_t> *sort_buf = nullptr, int64_t sort_cap = 0);
// device buffers over the extent [lo, hi) of a validated layout
fv_status check_buffers(const double *in, const double *out, const double *lambda_out, int32_t num_patches,
                        int64_t lo, int64_t hi);

struct UpdateLaunch;
// Launch parameters installed for a patch class (or the defaults), and their
// application to a launch.
fv_tuning tuning_for(int dim, int nq, int p);
void apply_tuning(UpdateLaunch &L);
void apply_tuning(UpdateLaunch &L, const fv_tuning &t);
// Validate launch parameters for a class and fill in their defaults (fv_set_tuning's rules).
fv_status resolve_tuning(int32_t dim, int32_t unknowns, int32_t p, const fv_tuning &in, fv_tuning *out);

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

// Descriptor lists of a plain call, grouped by patch size (a counting sort, largest first
// at launch).  Layout of the lists (host staging and its device copy alike): [num] int64
// input offsets, [num] int64 output offsets when with_out, [num] int32 ids.  Fixed-size:
// building them allocates nothing.
struct DescriptorGroups {
    int32_t count[FV_MAX_P_2D + 2];
    int32_t start[FV_MAX_P_2D + 2];
    char odd[FV_MAX_P_2D + 2];  // some patch of this size starts at an odd double
    int32_t num = 0;
    bool with_out = false;
};
size_t descriptor_bytes(int32_t T, bool with_out_offsets);
// Fill `host` (descriptor_bytes(T, out_offsets != NULL) bytes) and `g` for validated sizes / offsets.
void build_descriptors(const int32_t *sizes, const int64_t *offsets, const int64_t *out_offsets, int32_t T,
                       int32_t dim, int32_t nq, void *host, DescriptorGroups *g);
struct UpdateLaunch;
// One launch per size class of `g`, reading the lists from device memory `dev`; `tmpl` holds
// everything else of the launch (buffers, step, flags, lambda, PDE).
fv_status launch_descriptor_groups(const UpdateLaunch &tmpl, const void *dev, const DescriptorGroups &g,
                                   hipStream_t stream);
// Equal sizes at evenly spaced offsets (stride at least one patch), or offsets == NULL: such a
// batch runs as one launch with no descriptors, from offsets[0] (*base) with *stride doubles
// between patches.
bool regular_batch(const int64_t *offsets, int32_t T, int32_t dim, int32_t nq, const BatchShape &shape,
                   int64_t *base, int64_t *stride);
// That launch; *taken = false (and nothing enqueued) when the batch is not regular.
fv_status regular_launch(const UpdateLaunch &tmpl, const int64_t *offsets, int32_t T, const BatchShape &shape,
                         hipStream_t stream, bool *taken);
// Everything of a plain call's launches but the patch selection.
UpdateLaunch launch_template(const double *in, double *out, int32_t dim, int32_t nq, double dt, double h,
                             double gamma, uint32_t flags, double *lambda_out, const PdeArgs *pde);

struct DeviceContext;
// Context of the current HIP device; FV_ERR_NO_DEVICE / FV_ERR_UNSUPPORTED
// when there is none or it is not a gfx950.
fv_status current_context(DeviceContext **out);

}  // namespace fv
