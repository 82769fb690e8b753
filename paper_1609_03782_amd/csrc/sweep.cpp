// Parameter sweep scored by the quality diagnostics (Section 6's tuning of
// the filter over a grid of K, tau, n and C).  See ig_filter_sweep in
// include/igquality.h.  Host orchestration only: every run and every score
// is a device call of the library (ig_filter_run, ig_quality); one filter
// handle is re-parameterised per point, so the sweep allocates two cubes in
// all.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "igquality.h"
#include "internal.h"

#define fail igk_fail

namespace {

ig_params point_params(const ig_params& base, const ig_sweep_point& pt, double rho) {
    ig_params p = base;
    p.K = pt.K;
    p.tau = pt.tau;
    p.n_iter = pt.n_iter;
    for (int a = 0; a < 3; ++a) p.C[a] = pt.C[a];
    p.rms = rho;
    return p;
}

}  // namespace

extern "C" ig_status ig_filter_sweep(const ig_params* base, const ig_sweep_point* points, int32_t count,
                                     const float* d_in, const float* d_model, const ig_quality_params* q,
                                     int device, void* hip_stream, ig_quality_result* results, int32_t* best,
                                     float* d_best) {
    if (!points || count < 1 || !d_in || !q || !results || !best) return fail(IG_ERR_INVALID_ARG, "bad argument");
    ig_status st = igk_validate_params(base);
    if (st != IG_OK) return st;
    if (base->dtype != IG_F32) return fail(IG_ERR_UNSUPPORTED, "the sweep takes FP32 cubes");
    for (int i = 0; i < count; ++i) {
        const ig_params p = point_params(*base, points[i], 1.0);
        st = igk_validate_params(&p);
        if (st != IG_OK) {
            const std::string why = ig_last_error();
            return fail(st, "point %d: %s", i, why.c_str());
        }
    }
    if (q->struct_size != (int32_t)sizeof(ig_quality_params)) return fail(IG_ERR_INVALID_ARG, "q.struct_size");
    *best = -1;
    const long n = (long)(base->nx * base->ny * base->nz);
    st = igk_check_buffer(d_in, (size_t)n * 4, device, "d_in");
    if (st == IG_OK && d_model) st = igk_check_buffer(d_model, (size_t)n * 4, device, "d_model");
    if (st == IG_OK && d_best) st = igk_check_buffer(d_best, (size_t)n * 4, device, "d_best");
    if (st != IG_OK) return st;
    double rho = base->rms;
    if (!(rho > 0.0)) {
        double sum = 0.0, sumsq = 0.0;
        int64_t bad = 0;
        st = ig_reduce(d_in, IG_F32, n, device, hip_stream, &sum, &sumsq, &bad);
        if (st != IG_OK) return st;
        if (bad) return fail(IG_ERR_NONFINITE, "the input holds %lld non-finite voxels", (long long)bad);
        rho = std::sqrt(sumsq / (double)n);
    }
    ig_quality_params qq = *q;
    if (!(qq.rms_o > 0.0)) qq.rms_o = rho > 0.0 ? rho : 1.0;
    const ig_params p0 = point_params(*base, points[0], rho > 0.0 ? rho : 1.0);
    ig_filter* f = nullptr;
    st = ig_filter_create(&p0, device, &f);
    if (st != IG_OK) return st;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    float* work = nullptr;
    hipError_t he = igk_malloc((void**)&work, (size_t)n * sizeof(float));
    (void)hipSetDevice(prev >= 0 ? prev : device);
    if (he != hipSuccess) {
        ig_filter_destroy(f);
        return fail(he == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "work cube: %s",
                    hipGetErrorString(he));
    }
    hipStream_t s = (hipStream_t)hip_stream;
    double bestF = -INFINITY;
    for (int i = 0; i < count && st == IG_OK; ++i) {
        const ig_params p = point_params(*base, points[i], rho > 0.0 ? rho : 1.0);
        st = ig_filter_set_params(f, &p);
        if (st == IG_OK) st = ig_filter_run(f, d_in, work, hip_stream, nullptr);
        if (st == IG_OK)
            st = ig_quality(&qq, d_in, work, d_model, base->nx, base->ny, base->nz, device, hip_stream, &results[i]);
        if (st != IG_OK) break;
        const double F = results[i].F[0];
        if (F == F && F > bestF) {
            bestF = F;
            *best = i;
            if (d_best) {
                he = hipMemcpyAsync(d_best, work, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, s);
                if (he != hipSuccess) st = fail(IG_ERR_DEVICE, "copy of the best output: %s", hipGetErrorString(he));
            }
        }
    }
    if (st == IG_OK && (he = hipStreamSynchronize(s)) != hipSuccess)
        st = fail(IG_ERR_DEVICE, "sync: %s", hipGetErrorString(he));
    (void)hipStreamSynchronize(s);   // the work cube is in use until the stream drains
    (void)hipSetDevice(device);
    igk_free(work);
    (void)hipSetDevice(prev >= 0 ? prev : device);
    ig_filter_destroy(f);
    return st;
}
