/* Wavelet-lifting denoiser on the GPU (part of libigfilter.so): Section 3.4
 * of Punzo, van der Hulst & Roerdink (arXiv 1609.03782).
 *
 * One line x of length n is lifted in three steps: split into even_i = x_2i
 * and odd_i = x_2i+1, predict d_i = odd_i - P(even), update c_i = even_i +
 * U(d), and stored back as [c_0 .. c_ceil(n/2)-1, d_0 .. d_floor(n/2)-1].
 *   Haar:        P = even_i,                    U = d_i / 2;
 *   Le Gall 5/3: P = (even_i + even_i+1) / 2,   U = (d_i-1 + d_i) / 4,
 * with symmetric extension at the ends of the line.  A level lifts the
 * current approximation box along x, then y, then z (an axis of length 1 is
 * left alone); the next level works on the box of the first ceil(n/2) entries
 * of each axis.  Denoising thresholds the detail coefficients of level l at
 * t[l-1] * rms and the final approximation box at t[levels-1] * rms (hard:
 * |w| < threshold -> 0; the paper thresholds the approximation too, Section
 * 3.4), then reconstructs.
 *
 * Arithmetic: FP32, each step in the order written above with no fused
 * multiply-add (the constants 1/2 and 1/4 are exact), so the results are
 * reproducible bit for bit; the threshold test compares |w| with t * rms in
 * FP64.
 */
#ifndef IGWAVELET_H
#define IGWAVELET_H

#include <stdint.h>

#include "igfilter.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { IG_WAVELET_HAAR = 0, IG_WAVELET_LEGALL53 = 1 } ig_wavelet_kind;

#define IG_WAVELET_MAX_LEVELS 8

typedef struct {
    int32_t struct_size;                   /* sizeof(ig_wavelet_params) */
    int32_t kind;                          /* ig_wavelet_kind */
    int32_t levels;                        /* 1..IG_WAVELET_MAX_LEVELS (the paper: 1..3) */
    int32_t reserved;                      /* must be 0 */
    double t[IG_WAVELET_MAX_LEVELS];       /* denoise: threshold of level l's details in units of rms (>= 0);
                                              t[levels-1] also for the final approximation box */
    double rms;                            /* denoise: > 0 as given; else the plain rms of the input */
} ig_wavelet_params;

/* Forward transform of the FP32 cube d_in (nx*ny*nz, x fastest) into d_coef
 * (d_coef == d_in allowed; otherwise they must not overlap).  Asynchronous on
 * hip_stream; buffers and stream belong to the calling thread's current device
 * (as for every entry point of this header).  Errors: IG_ERR_INVALID_ARG (NULL, partial overlap, bad sizes,
 * kind, levels or reserved), IG_ERR_UNSUPPORTED (a line along y or z longer
 * than 2560, or along x longer than 10240: it must fit one compute unit's
 * LDS), IG_ERR_DEVICE. */
ig_status ig_wavelet_forward(const ig_wavelet_params* p, const float* d_in, float* d_coef, int64_t nx, int64_t ny,
                             int64_t nz, void* hip_stream);

/* Inverse transform of d_coef into d_out (d_out == d_coef allowed).
 * Asynchronous.  Errors as for ig_wavelet_forward. */
ig_status ig_wavelet_inverse(const ig_wavelet_params* p, const float* d_coef, float* d_out, int64_t nx, int64_t ny,
                             int64_t nz, void* hip_stream);

/* Denoise d_in into d_out (d_out == d_in allowed): forward transform, hard
 * thresholds, inverse.  *rms_used (nullable) receives the noise level used.
 * Waits for the stream only when rms must be estimated (it is a host value
 * the thresholds need).  Errors as above, plus IG_ERR_INVALID_ARG for negative
 * or non-finite thresholds and IG_ERR_NONFINITE when an estimated rms meets NaN
 * or Inf in the input. */
ig_status ig_wavelet_denoise(const ig_wavelet_params* p, const float* d_in, float* d_out, int64_t nx, int64_t ny,
                             int64_t nz, void* hip_stream, double* rms_used);

#ifdef __cplusplus
}
#endif

#endif /* IGWAVELET_H */
