/* Filtering-quality diagnostics on the GPU (part of libigfilter.so).
 *
 * Section 6 of Punzo, van der Hulst & Roerdink (arXiv 1609.03782) scores a
 * filtered cube I_f against the original I_o inside a region of interest
 * (ROI) with masks M_i = [I_i >= t rms_i]:
 *   S_oo = sum I_o M_o,  S_of = sum I_o M_f,  F = |S_of| / |S_oo|,
 *   sigma_S(o,i) = sqrt(N_i) rms_i (N_i independent voxels in M_i),
 *   sigma_F^2 = sigma_Sof^2 / S_oo^2 + S_of^2 sigma_Soo^2 / S_oo^4,
 * and, for a cube with a known noiseless model I_m, the recovered fraction
 *   F_M = |S_mf| / |S_m|,  S_mf = sum I_m M_f,  S_m = sum I_m,
 * with F evaluated over a sweep of M_f thresholds (0 to 4.5 rms in the paper).
 *
 * Readings where the paper is silent: rms_i defaults to the plain root mean
 * square of the whole cube i; the mask test is float(I) >= t * rms in FP64;
 * N_i = mask count / indep; sigma_FM = sqrt(N_f) rms_f / |S_m|.
 *
 * All sums are FP64, two-stage with a fixed work split and a fold in index
 * order: results are bitwise reproducible run to run.
 */
#ifndef IGQUALITY_H
#define IGQUALITY_H

#include <stdint.h>

#include "igfilter.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IG_QUALITY_MAX_THR 63

typedef struct {
    int32_t struct_size;                 /* sizeof(ig_quality_params) */
    int32_t n_thr;                       /* M_f thresholds in thr_f: 1..IG_QUALITY_MAX_THR */
    int64_t roi[6];                      /* x0, x1, y0, y1, z0, z1, half-open; all zero: the whole cube */
    double thr_f[IG_QUALITY_MAX_THR];    /* M_f thresholds, units of rms_f (any order) */
    double thr_o;                        /* M_o threshold, units of rms_o (3 in the paper) */
    double rms_o, rms_f;                 /* > 0: used as given; else the plain rms of the whole cube */
    double indep;                        /* voxels per independent element (> 0; 1: uncorrelated noise) */
} ig_quality_params;

typedef struct {
    double rms_o, rms_f;                 /* noise levels used */
    double S_oo, S_m;                    /* S_m = 0 without a model */
    int64_t N_o, n_roi;                  /* voxels in M_o, voxels in the ROI */
    double S_of[IG_QUALITY_MAX_THR];
    double S_mf[IG_QUALITY_MAX_THR];     /* 0 without a model */
    int64_t N_f[IG_QUALITY_MAX_THR];
    double F[IG_QUALITY_MAX_THR];        /* NaN when S_oo == 0 */
    double sigma_F[IG_QUALITY_MAX_THR];
    double F_M[IG_QUALITY_MAX_THR];      /* NaN without a model or when S_m == 0 */
    double sigma_FM[IG_QUALITY_MAX_THR];
} ig_quality_result;

/* F, sigma_F, F_M and sigma_FM for every M_f threshold of q.  d_orig, d_filt
 * and d_model (nullable) are FP32 device cubes of nx*ny*nz voxels, [z][y][x]
 * with x fastest, on `device`; they are only read.  Runs on hip_stream and
 * waits for it (the result is host memory).  Errors: IG_ERR_INVALID_ARG for a
 * NULL cube or result, bad sizes, an empty or out-of-range ROI, n_thr out of
 * range, non-finite thresholds or indep <= 0; IG_ERR_NONFINITE when a cube
 * whose rms is to be estimated holds NaN or Inf; IG_ERR_DEVICE for HIP
 * failures. */
ig_status ig_quality(const ig_quality_params* q, const float* d_orig, const float* d_filt, const float* d_model,
                     int64_t nx, int64_t ny, int64_t nz, int device, void* hip_stream, ig_quality_result* out);

/* One point of a parameter sweep. */
typedef struct {
    float K, tau;          /* K in units of the noise level rho */
    int32_t n_iter;
    float C[3];            /* per axis x, y, z */
} ig_sweep_point;

/* Parameter sweep, the tuning procedure of Section 6: filter d_in once per
 * point, with base's conductance and shape and the point's K, tau, n_iter and
 * C, and score each output with ig_quality(q, d_in, output, d_model).  The
 * input's noise level rho (base->rms > 0: as given; else the plain rms of
 * d_in, computed once) is used by every run and, unless q->rms_o > 0, as
 * rms_o.  results[i] receives point i's diagnostics; *best the index of the
 * largest F[0] (the lowest index among equal values; -1 if every F[0] is
 * NaN); d_best (nullable, nx*ny*nz FP32 device memory) the output of that
 * point.  FP32 storage only; d_in and d_model are only read.  Device memory:
 * one filter scratch cube and one work cube for the whole sweep.  Every point
 * is validated before any work starts.  Waits for the stream. */
ig_status ig_filter_sweep(const ig_params* base, const ig_sweep_point* points, int32_t count, const float* d_in,
                          const float* d_model, const ig_quality_params* q, int device, void* hip_stream,
                          ig_quality_result* results, int32_t* best, float* d_best);

#ifdef __cplusplus
}
#endif

#endif /* IGQUALITY_H */
