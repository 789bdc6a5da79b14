// fv_step.hip -- device-side time-step size for captured multi-step runs.
//
// The per-patch maximum eigenvalue of the new solution feeds the CFL
// condition and fixes the next time step (end of Sec. 2.2).  Inside a
// captured graph the step size has to be formed on the device:
//     dt_next = cfl * h / (d * max_t lambda_t),   r_next = dt_next / h
// (max NaN-propagating, so a non-physical state yields a NaN step size that
// the caller sees in dt_dev).  `slot` and `done` are device words that must be
// zero before the first launch; every launch leaves them zero again.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "fv_internal.h"
#include "fv_physics.h"

namespace fv {
namespace {

constexpr int kStepThreads = 256;
constexpr int kStepBlocks = 256;

// Many blocks: each folds its part of lambda into one 64-bit maximum on the
// bit pattern (values are >= 0, NaN's pattern sorts above +inf, so the integer
// maximum is the NaN-propagating maximum); the last block to finish turns it
// into the next step size and resets the slot and the counter for the next
// step (so a replayed graph needs no memset nodes).
__global__ void __launch_bounds__(kStepThreads)
next_dt_kernel(const double *__restrict__ lambda, int32_t n, double cfl, double h, int32_t dim,
               double *__restrict__ dt_out, double *__restrict__ r_out, unsigned long long *__restrict__ slot,
               unsigned int *__restrict__ done) {
    __shared__ double part[kStepThreads / 64];
    __shared__ bool last;
    double m = 0.0;
    for (int32_t t = blockIdx.x * kStepThreads + threadIdx.x; t < n; t += gridDim.x * kStepThreads)
        m = nanmax(m, lambda[t]);
    for (int o = 32; o > 0; o >>= 1) m = nanmax(m, __shfl_xor(m, o, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double g = 0.0;
        for (int w = 0; w < kStepThreads / 64; ++w) g = nanmax(g, part[w]);
        atomicMax(slot, __builtin_bit_cast(unsigned long long, g));
        __threadfence();
        last = atomicAdd(done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        const double g = __builtin_bit_cast(double, atomicAdd(slot, 0ull));
        const double dt = cfl * h / ((double)dim * g);
        *dt_out = dt;
        *r_out = dt / h;
        atomicExch(slot, 0ull);
        atomicExch(done, 0u);
    }
}

// dt/h from a caller-provided dt (first step of a captured run).
__global__ void ratio_kernel(const double *__restrict__ dt, double h, double *__restrict__ r_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *r_out = *dt / h;
}

}  // namespace

hipError_t launch_next_dt(const double *lambda, int32_t n, double cfl, double h, int32_t dim, double *dt_out,
                          double *r_out, unsigned long long *slot, unsigned int *done, hipStream_t stream) {
    const int blocks = std::max(1, std::min(kStepBlocks, (n + kStepThreads - 1) / kStepThreads));
    hipLaunchKernelGGL(next_dt_kernel, dim3(blocks), dim3(kStepThreads), 0, stream, lambda, n, cfl, h, dim, dt_out,
                       r_out, slot, done);
    return hipGetLastError();
}

hipError_t launch_ratio(const double *dt, double h, double *r_out, hipStream_t stream) {
    hipLaunchKernelGGL(ratio_kernel, dim3(1), dim3(64), 0, stream, dt, h, r_out);
    return hipGetLastError();
}

}  // namespace fv
