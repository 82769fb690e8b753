/* Box and Gaussian smoothing of a data cube on the GPU (part of
 * libigfilter.so): the comparison filters of Section 3 of Punzo, van der
 * Hulst & Roerdink (arXiv 1609.03782).
 *
 *  box      the mean of the N_x x N_y x N_z neighbourhood (odd N) centred on
 *           each voxel, the voxel included (Section 3.1);
 *  Gaussian the weighted mean with weights exp(-sum_j u_j^2 / (2 sigma_j^2)),
 *           u = R^T d for the offset d, R = R_z(theta_z) R_y(theta_y)
 *           R_x(theta_x) (right-handed Euler rotations, degrees) and
 *           sigma_j = FWHM_j / (2 sqrt(2 ln 2)) (Section 3.2).
 *
 * Readings where the paper is silent: the kernel box has half-width
 * r_i = floor(truncate * s_i + 0.5) (s_i = sigma_i for an axis-aligned
 * kernel, sqrt(sum_j R_ij^2 sigma_j^2) for a rotated one); at the cube faces
 * the weighted mean runs over the neighbours inside the cube (weights
 * renormalised over them).
 *
 * The box and the axis-aligned Gaussian are separable: 1-D sums along x, y
 * and z, each renormalised over its in-cube taps, give the 3-D definition
 * exactly (up to rounding).  For half-widths up to 8 one fused pass computes
 * all three sums while streaming the cube along z (each voxel read and
 * written once); larger half-widths, or rows longer than 5,592,405 voxels,
 * run three passes (x, y, z) through d_work.  Both routes compute the same
 * sums in the same order, so they give the same values.  A rotated Gaussian
 * runs as one dense 3-D pass.  Weights are computed on the device in FP64 and
 * stored as FP32; sums are FP32.
 */
#ifndef IGSMOOTH_H
#define IGSMOOTH_H

#include <stdint.h>

#include "igfilter.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { IG_SMOOTH_BOX = 0, IG_SMOOTH_GAUSS = 1 } ig_smooth_kind;

typedef struct {
    int32_t struct_size;   /* sizeof(ig_smooth_params) */
    int32_t kind;          /* ig_smooth_kind */
    float size[3];         /* box: N_x, N_y, N_z (odd integers >= 1); Gaussian: FWHM_x, y, z in voxels (> 0) */
    float theta[3];        /* Gaussian: Euler angles theta_x, theta_y, theta_z in degrees; box: must be 0 */
    float truncate;        /* Gaussian: kernel half-width in units of sigma (0: 3) */
    int32_t reserved;      /* must be 0 */
} ig_smooth_params;

/* Kernel half-widths (r_x, r_y, r_z) that s implies, and whether it runs as
 * separable 1-D sums (1: the fused pass or three passes) or one dense pass
 * (0).  Host only. */
ig_status ig_smooth_geometry(const ig_smooth_params* s, int32_t* radius, int32_t* separable);

/* Smooth d_in (FP32, nx*ny*nz voxels, x fastest) into d_out on hip_stream;
 * the buffers and the stream belong to the calling thread's current device.
 * d_work: nx*ny*nz FP32 device scratch, required by the separable kernels (the
 * three-pass route holds its middle pass there; the fused pass leaves it
 * untouched), ignored (may be NULL) by the dense one.  d_in is only
 * read; d_in, d_out and d_work must not overlap.  Asynchronous.  Errors:
 * IG_ERR_INVALID_ARG (NULL or overlapping buffers, bad sizes, even or
 * non-integer box sizes, FWHM <= 0, non-finite values, non-zero reserved or box
 * angles), IG_ERR_UNSUPPORTED (a half-width above 31 for the separable path,
 * or a dense kernel too large for one compute unit's LDS: its
 * (2 r_x + 1)(2 r_y + 1)(2 r_z + 1) weights plus an input tile of at least
 * (64 + 2 r_x)(4 + 2 r_y)(1 + 2 r_z) voxels, x 4 B, above 160 KiB),
 * IG_ERR_DEVICE. */
ig_status ig_smooth(const ig_smooth_params* s, const float* d_in, float* d_out, float* d_work, int64_t nx,
                    int64_t ny, int64_t nz, void* hip_stream);

/* Route of the separable kernels for later ig_smooth calls, process-wide:
 * 0 (the default) the fused pass wherever it applies, 1 always the three
 * passes (for comparisons and measurements; the values are the same).  Not
 * synchronised with ig_smooth calls running in other threads.  Errors:
 * IG_ERR_INVALID_ARG for any other value.  Host only. */
ig_status ig_smooth_set_path(int32_t path);

#ifdef __cplusplus
}
#endif

#endif /* IGSMOOTH_H */
