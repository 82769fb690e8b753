/*
 * igsurrogate.h - C ABI of the learned surrogate of the intensity-driven
 * gradient filter (MI355X / gfx950).
 *
 * The surrogate is not part of the paper: it is a small 3-D CNN trained on
 * pairs (cube, n-step filtered cube) that the filter of Section 3.3 itself
 * produces, and predicts the filtered cube in one pass:
 *     a_0 = x,  z_l = conv3x3x3(a_{l-1}) + b_l,  a_l = gelu(z_l)  (l < depth),
 *     y = x + z_depth  (one output channel, residual to the input),
 * with zero padding outside the cube and gelu(z) = z/2 (1 + erf(z/sqrt 2)).
 * Weights and activations are bf16, accumulation FP32 on the matrix cores,
 * master weights FP32 with Adam.  The filter keeps the last word: a residual
 * check runs two plain filter steps on the prediction and falls back to the
 * full filter when the predicted error is too large.
 *
 * Conventions are those of igfilter.h (device pointers, caller-owned
 * buffers, hip_stream, ig_status, ig_last_error).  Cubes are FP32
 * [nz][ny][nx], x fastest; activations are bf16 channels-last
 * [(z*ny + y)*nx + x][C] passed as raw 16-bit words.  A weight tensor is FP32
 * [27][c_in][c_out] with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1): output voxel v
 * reads input voxel v + (dz, dy, dx).
 */
#ifndef IGSURROGATE_H
#define IGSURROGATE_H

#include <stdint.h>

#include "igfilter.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t struct_size;   /* = sizeof(ig_surrogate_params) */
    int32_t depth;          /* convolution layers, >= 2 (8 for the reference network) */
    int32_t width;          /* hidden channels: must be 32 */
    int32_t reserved;       /* must be 0 */
    float lr, beta1, beta2, eps;   /* Adam */
    uint64_t seed;          /* weight initialisation (last layer starts at 0: y = x) */
} ig_surrogate_params;

typedef struct ig_surrogate ig_surrogate;

ig_status ig_surrogate_create(const ig_surrogate_params* p, int device, ig_surrogate** out);
void ig_surrogate_destroy(ig_surrogate* s);

/* Number of FP32 parameters: per layer W (27*c_in*c_out) then b (c_out). */
int64_t ig_surrogate_param_count(const ig_surrogate* s);
/* Copy all FP32 master parameters from / to host memory (count entries).
 * set resets the Adam state. */
ig_status ig_surrogate_set_weights(ig_surrogate* s, const float* host, int64_t count);
ig_status ig_surrogate_get_weights(const ig_surrogate* s, float* host, int64_t count);
/* Gradient of the last training step's loss (same layout as the weights). */
ig_status ig_surrogate_get_grads(const ig_surrogate* s, float* host, int64_t count);

/* Checkpoints of the training state: FP32 master weights, Adam m and v, the
 * step count and the initialisation seed, with the Adam hyper-parameters the
 * handle was created with recorded beside them.  Layout (little-endian): a
 * 64-byte header {char magic[8] = "IGSURR\0\1"; uint32 header_bytes = 64;
 * uint32 version = 1; int32 depth; int32 width; int64 nparam; int64 step;
 * uint64 seed; float lr, beta1, beta2, eps}, then FP32 params[nparam],
 * m[nparam], v[nparam], then the 64-bit FNV-1a hash of every byte before it.
 * save waits for the device and writes `path` through a temporary file
 * renamed into place.  load checks magic, version, sizes and hash, and that
 * the network's depth and width match the handle's (else
 * IG_ERR_INVALID_ARG with nothing changed); it restores weights, m, v, step
 * and seed (the handle keeps its own lr, betas and eps), so training resumes
 * exactly where the saved run stood.  checkpoint_info reads and checks a
 * file on the host only (no device, no handle); outputs are nullable. */
ig_status ig_surrogate_save(const ig_surrogate* s, const char* path);
ig_status ig_surrogate_load(ig_surrogate* s, const char* path);
ig_status ig_surrogate_checkpoint_info(const char* path, int32_t* depth, int32_t* width, int64_t* nparam,
                                       int64_t* step, uint64_t* seed);

/* Learning rate of later training steps (a schedule is the caller's: e.g.
 * cosine decay over the planned steps); IG_ERR_INVALID_ARG unless finite > 0.
 * get_step: Adam steps taken so far (-1 for NULL). */
ig_status ig_surrogate_set_lr(ig_surrogate* s, float lr);
int64_t ig_surrogate_get_step(const ig_surrogate* s);

/* Clipping of later training steps by the global gradient norm: when
 * ||g||_2 (FP64, over every parameter) exceeds max_norm, the step uses
 * g * max_norm / ||g||; 0 (the default) turns it off.  The factor is computed
 * and applied on the device.  last_grad_norm waits and returns ||g|| of the
 * last step (before clipping); IG_ERR_INVALID_ARG before the first step. */
ig_status ig_surrogate_set_clip(ig_surrogate* s, float max_norm);
ig_status ig_surrogate_last_grad_norm(const ig_surrogate* s, double* norm);

/* One Adam step on the mean squared error over `batch` cubes of one shape:
 * d_x[k], d_t[k] are device FP32 cubes (input, target).  loss (nullable)
 * receives the mean squared error before the step (the call then waits). */
ig_status ig_surrogate_train_step(ig_surrogate* s, const float* const* d_x, const float* const* d_t, int32_t batch,
                                  int64_t nx, int64_t ny, int64_t nz, void* hip_stream, double* loss);

/* Predict y from x.  tile > 0: cubes of tile^3 outputs, each computed with a
 * halo of `depth` voxels (the network's receptive radius), which gives the
 * same result as one piece; a piece with its halo must stay below the piece
 * limit, 2^28 voxels (its two 32-channel bf16 activation buffers take 128
 * bytes per voxel: 32 GiB at the limit).  tile == 0: the whole cube in one
 * piece below that limit (a 512^3 cube: 17 GiB of buffers), otherwise slabs
 * of the whole x-y extent: the fewest equal runs of planes whose slab with
 * its halo planes stays below it.  The buffers are kept by the handle for the
 * next call. */
ig_status ig_surrogate_infer(ig_surrogate* s, const float* d_x, float* d_y, int64_t nx, int64_t ny, int64_t nz,
                             int32_t tile, void* hip_stream);

typedef struct {
    double residual;        /* rms of (2 plain steps of y) - y, in units of rho */
    double predicted_rmse;  /* slope * residual */
    double rho;             /* noise level of x used by the check */
    int32_t fell_back;      /* 1: y is the plain filter's result */
    int32_t reserved;
} ig_surrogate_report;

/* Checked prediction: y = surrogate(x); r = rms(F_2(y) - y) / rho with F_2
 * two steps of the filter described by p (same K, tau, C; rho of x); if
 * slope * r > threshold, y is replaced by the plain filter (p->n_iter steps).
 * p->dtype must be IG_F32.  Waits for the stream. */
ig_status ig_surrogate_infer_checked(ig_surrogate* s, const ig_params* p, const float* d_x, float* d_y,
                                     int32_t tile, double slope, double threshold, void* hip_stream,
                                     ig_surrogate_report* rep);

/* Building blocks, for checking the kernels one by one.
 * ig_conv3d_forward: d_in bf16 [v][c_in] (c_in 1 or 32), d_w/d_b FP32,
 *   c_out 1..32.  epilogue 0: FP32 out [v][16*ceil(c_out/16)] = conv + b;
 *   1: bf16 out [v][32] = gelu(conv + b) and, if d_aux != NULL, bf16 d_aux
 *   [v][32] = conv + b; 3: FP32 out [v] = d_aux[v] (FP32) + conv + b, c_out 1.
 * ig_conv3d_input_grad: gradient w.r.t. the input of a conv with weights d_w
 *   [27][c_in][c_out] given d_dz bf16 [v][c_out] (c_out 1 or 32, c_in 1..32):
 *   d_aux == NULL: FP32 out [v][16*ceil(c_in/16)]; else bf16 out [v][32] =
 *   grad * gelu'(d_aux) with d_aux the bf16 pre-activation [v][32].
 * ig_conv3d_weight_grad: FP32 d_dw [27][c_in][c_out] and d_db [c_out] of a
 *   conv with input d_a bf16 [v][c_in] (1 or 32) and output gradient d_dz
 *   bf16 [v][c_out] (1 or 32); partial sums in a fixed order (deterministic).
 * All three allocate temporaries and wait for the stream, and return
 * IG_ERR_INVALID_ARG for cubes of 2^31 / 32 voxels or more (these entry points
 * are for checking the kernels on small cubes; each allocates a whole-cube
 * 32-channel temporary per call). */
ig_status ig_conv3d_forward(const void* d_in, int32_t c_in, const float* d_w, const float* d_b, int32_t c_out,
                            int32_t epilogue, void* d_aux, void* d_out, int64_t nx, int64_t ny, int64_t nz,
                            void* hip_stream);
ig_status ig_conv3d_input_grad(const void* d_dz, int32_t c_out, const float* d_w, int32_t c_in, const void* d_aux,
                               void* d_out, int64_t nx, int64_t ny, int64_t nz, void* hip_stream);
ig_status ig_conv3d_weight_grad(const void* d_a, int32_t c_in, const void* d_dz, int32_t c_out, float* d_dw,
                                float* d_db, int64_t nx, int64_t ny, int64_t nz, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* IGSURROGATE_H */
