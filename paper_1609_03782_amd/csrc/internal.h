// Library-internal declarations shared by the host code and the kernel
// translation units (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stencil_common.h"

namespace igk {

// Host-side inputs of the parameter kernel.
struct ParamIn {
    float K, tau;
    float C[3];
    int cond;
    int abort_on_nonfinite;
    double rms;        // > 0: given; else estimated from the scan
};

struct NaiveGeom;
struct BlockGeom;

hipError_t launch_sum_partial(int dtype, const void* x, long n, double* part, int nblk, hipStream_t s);
hipError_t launch_params_final(const double* part, int nparts, long n, const ParamIn& in, DevParams* out,
                               hipStream_t s);
hipError_t launch_compare(int dtype, const void* x, const double* ref, long n, double tol, double* part,
                          int nblk, double* out, hipStream_t s);
hipError_t launch_copy(int dtype, const void* a, void* b, long n, const DevParams* dp, hipStream_t s);

// Stencil launchers; one translation unit per (conductance, storage type).
// V in {1,2,4,8}, R in {1,2,4}, T in {1..4}.
struct StencilLaunch {
    hipError_t (*naive)(const void* src, void* dst, int nx, int ny, int nz, const DevParams* dp, hipStream_t s);
    hipError_t (*blocked)(const void* src, void* dst, const BlockGeom& g, int V, int R, int T,
                          const DevParams* dp, hipStream_t s, int nblocks);
};
const StencilLaunch* stencil_table(int cond, int dtype);

constexpr int kPartBlocks = 1024;   // partials of the FP64 reductions

}  // namespace igk
