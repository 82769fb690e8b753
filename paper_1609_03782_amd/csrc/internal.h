// Library-internal declarations shared by the host code and the kernel
// translation units (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "igfilter.h"
#include "plan.h"
#include "stencil_common.h"
#include "stencil_kernels.h"

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


hipError_t launch_sum_partial(int dtype, const void* x, long n, double* part, int nblk, hipStream_t s);
hipError_t launch_params_final(const double* part, int nparts, long n, const ParamIn& in, DevParams* out,
                               hipStream_t s);
hipError_t launch_compare(int dtype, const void* x, const double* ref, long n, double tol, double* part,
                          int nblk, double* out, hipStream_t s);
hipError_t launch_copy(int dtype, const void* a, void* b, long n, const DevParams* dp, hipStream_t s);
// Writes NaN over all n elements of x if dp->abort is set; otherwise every
// workgroup returns at once.
hipError_t launch_nan_if_abort(int dtype, void* x, long n, const DevParams* dp, hipStream_t s);

// Stencil launchers; one translation unit per (conductance, storage type).
// V in {1,2,4,8}, T in {1..4}.
struct StencilLaunch {
    hipError_t (*naive)(const void* src, void* dst, int nx, int ny, int nz, const DevParams* dp, hipStream_t s);
    // one workgroup per piece, or (g.grouped) nwg workgroups each running its
    // range of the table
    hipError_t (*blocked)(const void* src, void* dst, const BlockGeom& g, int V, int T, const Piece* pieces,
                          int nwg, const DevParams* dp, hipStream_t s);
};
const StencilLaunch* stencil_table(int cond, int dtype);

constexpr int kPartBlocks = 2048;   // partials of the FP64 reductions

}  // namespace igk

// A buffer a kernel will touch: device (or managed) memory of `device` whose
// allocation covers [p, p + bytes).  A host pointer or a short allocation is
// reported as IG_ERR_INVALID_ARG (naming `what`) instead of faulting on the GPU.
ig_status igk_check_buffer(const void* p, size_t bytes, int device, const char* what);
// The calling thread's current device (0 if it cannot be read).
int igk_current_device();
// The library's device / pinned-host allocations (counted, and failed on
// purpose when a test asks for it; see ig_debug_fail_alloc).  free(NULL) is a no-op.
hipError_t igk_malloc(void** p, size_t bytes);
void igk_free(void* p);
hipError_t igk_host_malloc(void** p, size_t bytes);
void igk_host_free(void* p);
// What one filter run needs besides its input and output: the ping-pong
// scratch cube, the run's constants, the reduction partials, and the piece
// table of each pass depth.  A handle provides its own allocations; the
// no-allocation entry point provides carved-out parts of a static array.
struct RunCtx {
    const ig_params* p;
    void* scratch;               // nx*ny*nz elements of p->dtype
    igk::DevParams* dparams;
    double* parts;               // kPartBlocks * 6 doubles
    double* results;             // 8 doubles
    // the plan of the pass of depth T and its piece table on the device
    ig_status (*plan)(void* self, const ig_schedule& s, int T, const PassPlan** out, const igk::Piece** dev);
    void* plan_self;
    hipError_t (*hook)(void* self, hipStream_t s);   // timing event before/after each pass (nullable)
    void* hook_self;
};
// Enqueue rho (scan when `scan`), the passes and the NaN-on-abort fill.
ig_status igk_enqueue_run(const RunCtx& c, const ig_schedule& sched, const void* d_in, void* d_out, bool scan,
                          hipStream_t stream, int* passes_out);
// Wait for the stream and fill *stats (second scan of d_out for sum_out).
ig_status igk_finish_stats(const RunCtx& c, const ig_schedule& sched, int passes, const void* d_out,
                           hipStream_t s, ig_stats* stats);

