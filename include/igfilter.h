/*
 * igfilter.h - C ABI of the MI355X (gfx950) intensity-driven gradient filter.
 *
 * The filter (Punzo, van der Hulst & Roerdink, "Finding faint H I structure
 * in and around galaxies: scraping the barrel", Section 3.3, Eqs. 5-7) runs
 * n explicit, synchronous (Jacobi) steps of anisotropic diffusion on a 3-D
 * data cube:
 *
 *   I_{i+1}(v) = I_i(v) + tau * sum_{a in x,y,z} C_a * sum_{s=+-1} w(v,u) (I_i(u) - I_i(v)),
 *
 * with u = v + s e_a and the weight w chosen by ig_conductance.  A neighbour
 * outside the cube takes the voxel's own value (no flux through the faces).
 * rho, the cube's noise level, scales K: it is the caller's value, or the
 * root mean square of the input over all voxels, computed once (FP64).
 *
 * Conventions shared by every entry point
 *   - Layout: a cube is nz planes of ny rows of nx voxels, x fastest
 *     (right ascension, declination, velocity channel: Section 2 of the
 *     paper), index x + nx * (y + ny * z), densely packed.
 *   - Pointers named d_* are device pointers on the handle's device (e.g.
 *     torch tensors' data_ptr()).  The caller owns them; the library never
 *     frees them.  Handles own their scratch memory.  Before any work is
 *     enqueued, each such buffer is checked with the runtime: host memory
 *     (pinned or not), memory of another device, or an allocation that ends
 *     before the bytes the call uses gives IG_ERR_INVALID_ARG.  (The size
 *     check sees whole runtime allocations: a tensor carved out of a larger
 *     allocation by a caching allocator is checked against that allocation.)
 *   - hip_stream is a hipStream_t cast to void*; NULL means the null stream.
 *     Work is enqueued on that stream and the call returns without waiting,
 *     unless an output argument that lives on the host (stats, latency) is
 *     requested: then the call waits for the stream.
 *   - Errors: every entry point returns an ig_status; no exception crosses
 *     the ABI.  Arguments are validated before any device work is enqueued.
 *     ig_last_error() gives a thread-local message for the last failure.
 *   - Threads: a handle is not re-entrant; distinct handles may be used from
 *     distinct threads.
 */
#ifndef IGFILTER_H
#define IGFILTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IG_OK = 0,
    IG_ERR_INVALID_ARG = 1,    /* bad size, parameter, enum, pointer or overlap */
    IG_ERR_OUT_OF_MEMORY = 2,  /* device allocation failed */
    IG_ERR_DEVICE = 3,         /* a HIP call failed */
    IG_ERR_NONFINITE = 4,      /* the input holds NaN or Inf; the output is set to NaN */
    IG_ERR_UNSUPPORTED = 5     /* valid request this build cannot serve */
} ig_status;

/* Storage type of the cube in device memory.  Arithmetic is FP32 for every
 * storage type; 16-bit storage rounds (to nearest, ties to even) after every
 * step, including steps kept on chip. */
typedef enum { IG_F32 = 0, IG_BF16 = 1, IG_F16 = 2 } ig_dtype;

/* The weight w of the update (Section 3.3):
 *   IG_COND_INTENSITY   : w = 1 / (1 + I_i(v)^2 / (K rho)^2), the paper's
 *                         intensity-driven conductance (Eq. 6), evaluated at
 *                         the centre voxel, i.e. the discretised filter of Eq. 7.
 *   IG_COND_PM_EXP      : w = exp(-((I_i(u) - I_i(v)) / (K rho))^2) per edge,
 *                         the exponential Perona-Malik edge-stopping function.
 *   IG_COND_PM_RATIONAL : w = 1 / (1 + ((I_i(u) - I_i(v)) / (K rho))^2) per
 *                         edge, Eq. 5 with K in rms units. */
typedef enum { IG_COND_INTENSITY = 0, IG_COND_PM_EXP = 1, IG_COND_PM_RATIONAL = 2 } ig_conductance;

/* Filter parameters (Section 3.3: K, tau, n, C_x, C_y, C_z and rms).
 * The paper's slider ranges (tau in [0.0025, 0.0625], C in [0, 10],
 * K in [0.5, 10]) are not enforced; only mathematical validity is. */
typedef struct {
    uint32_t struct_size;   /* = sizeof(ig_params); guards against ABI skew */
    int32_t dtype;          /* ig_dtype */
    int32_t cond;           /* ig_conductance */
    int32_t n_iter;         /* number of steps n >= 0 */
    int64_t nx, ny, nz;     /* >= 1 each; nx*ny*nz < 2^31 */
    float K;                /* > 0 and finite, in units of rho */
    float tau;              /* >= 0 and finite */
    float C[3];             /* C_x, C_y, C_z >= 0 and finite */
    float reserved0;        /* must be 0 */
    double rms;             /* > 0 (finite): use as rho; <= 0: estimate from the input */
} ig_params;

/* How the steps are scheduled on the GPU.  The result is bitwise the same
 * for every schedule: each voxel's arithmetic does not depend on it. */
typedef enum {
    IG_SCHED_AUTO = 0,      /* library choice (tuned table, else heuristic) */
    IG_SCHED_NAIVE = 1,     /* one step per launch, one voxel per thread */
    IG_SCHED_BLOCKED = 2    /* t_block steps per launch, z-streaming tiles */
} ig_sched_kind;

typedef struct {
    int32_t kind;      /* ig_sched_kind */
    int32_t t_block;   /* steps per pass, 1..4 (BLOCKED) */
    int32_t waves;     /* wavefronts per workgroup, 1..16 (BLOCKED) */
    int32_t zchunk;    /* 0: split the cube into pieces of equal work, a whole number of
                          rounds of the workgroups the GPU holds at once; > 0: pieces
                          of zchunk output planes (BLOCKED) */
    int32_t vec;       /* x voxels per lane: 1, 2, 4 or 8; 0 = automatic (8 for
                          256 < nx <= 512, 4 above 512 (256-voxel x tiles), else 4 with
                          `rows` chosen to cover nx).  Cubes wider than one tile
                          (64 vec voxels) are cut into x tiles whose halo is t_block
                          rounded up to a multiple of vec */
    int32_t rounds;    /* zchunk == 0: rounds of resident workgroups; 0 = as few as possible */
    int32_t rows;      /* rows per wavefront: 1, 2 or 4 (a tile has waves * rows rows); more
                          than 1 needs vec 4 and nx <= 256 / rows (one x tile); 0 = automatic
                          with vec 0, else 1 */
} ig_schedule;

typedef struct {
    uint32_t struct_size;   /* = sizeof(ig_stats), set by the caller */
    int32_t passes;         /* kernel launches of the step loop */
    double rms_used;        /* rho */
    double sum_in;          /* sum of the input voxels (FP64) */
    double sum_out;         /* sum of the output voxels (FP64) */
    int64_t nonfinite;      /* NaN / Inf voxels found in the input */
    int32_t monotone;       /* 1 if 2 tau (C_x + C_y + C_z) <= 1 (maximum principle) */
    int32_t reserved;
    ig_schedule schedule;   /* schedule used */
} ig_stats;

typedef struct ig_filter ig_filter;

/* Create a handle for cubes of the given parameters on `device`.  Allocates
 * one scratch cube (ping-pong partner) and small reduction buffers.
 * On error *out is set to NULL. */
ig_status ig_filter_create(const ig_params* p, int device, ig_filter** out);

/* Filter d_in into d_out (both nx*ny*nz elements of p->dtype).  d_in == d_out
 * is allowed (2 cubes of device memory in total, the paper's two-buffer GPU
 * model of Section 5); any other overlap is IG_ERR_INVALID_ARG.  d_in is not
 * modified unless it equals d_out.  If stats != NULL the call waits for the
 * stream and fills it.  The scan of the input runs whenever the rms is
 * estimated or stats are requested; if it finds a NaN or Inf voxel, no step
 * runs and every voxel of d_out is set to NaN (in place, the input is
 * overwritten), and with stats != NULL the call returns IG_ERR_NONFINITE.
 * (With rms given and no stats there is no scan: a non-finite voxel then
 * spreads through the steps as IEEE arithmetic carries it.) */
ig_status ig_filter_run(ig_filter* f, const void* d_in, void* d_out, void* hip_stream,
                        ig_stats* stats);

/* Largest cube, in bytes of its storage type, that ig_filter_run_static
 * serves: 64 MiB (16,777,216 FP32 or 33,554,432 16-bit voxels, e.g. a
 * 256^3 FP32 cube). */
#define IG_STATIC_MAX_CUBE_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the filter
 * of ig_filter_run without a handle and without any device allocation.  The
 * ping-pong cube, the noise-level partials and the piece tables live in one
 * static device array of the library (IG_STATIC_MAX_CUBE_BYTES plus about
 * 1.1 MiB, held on each GPU the library runs on until the process ends).
 * Arguments: p as for ig_filter_create (cubes of at most
 * IG_STATIC_MAX_CUBE_BYTES; larger ones give IG_ERR_INVALID_ARG before any
 * work), `device` the GPU of d_in and d_out, the rest as for ig_filter_run
 * (d_in == d_out allowed; stats nullable, when given the call waits).  The
 * result is bitwise the one ig_filter_run gives for the same parameters.
 * The schedule is the library's automatic one with z chunks sized to one
 * round of workgroups.  Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (concurrent streams or threads) race and
 * must be serialised by the caller; consecutive calls on one stream are
 * ordered by the stream. */
ig_status ig_filter_run_static(const ig_params* p, int device, const void* d_in, void* d_out, void* hip_stream,
                               ig_stats* stats);

/* IG_STATIC_MAX_CUBE_BYTES as the library was built. */
int64_t ig_filter_static_max_bytes(void);

/* Override the schedule (NULL restores IG_SCHED_AUTO).  Rejects shapes the
 * schedule cannot serve with IG_ERR_INVALID_ARG. */
ig_status ig_filter_set_schedule(ig_filter* f, const ig_schedule* s);
ig_status ig_filter_get_schedule(const ig_filter* f, ig_schedule* s);

/* Host-only check (no device work, no handle): IG_OK if schedule s can serve
 * cubes described by p, else IG_ERR_INVALID_ARG with the reason in
 * ig_last_error(). */
ig_status ig_schedule_check(const ig_params* p, const ig_schedule* s);

/* Autotuner: times the filter with each candidate schedule (t_block 1..4,
 * waves 8/12/16, 1 or 2 rounds of pieces; those the shape and the LDS allow)
 * on d_in -> d_work (distinct buffers of the handle's shape and type; d_work
 * is overwritten), sets the fastest on the handle and returns it in *best
 * (and its run time in *best_ms, nullable).  If the environment variable
 * IG_TUNE_CACHE names a file, a result stored there for the same device
 * architecture, storage type, conductance, shape and n is used without
 * timing, and new results are appended to it (one JSON object per line).
 * Waits for the stream. */
ig_status ig_filter_autotune(ig_filter* f, const void* d_in, void* d_work, void* hip_stream, ig_schedule* best,
                             double* best_ms);

/* Kernel timing: while enabled, every launch of the step loop (the passes of
 * ig_filter_run) is bracketed by HIP events recorded on the run's stream.
 * ig_filter_get_timing waits for those events and returns the summed device
 * time in ms and the number of timed launches since the last reset. */
ig_status ig_filter_set_timing(ig_filter* f, int enable);
ig_status ig_filter_get_timing(ig_filter* f, double* total_ms, int64_t* launches, int reset);

/* Host-only: the work split of one pass of depth t_block under schedule s
 * (BLOCKED) on a GPU with ncu compute units.  geom[9] receives
 * {ntx, nty, ox, oy, waves, vec_io, V, pieces, rows per wavefront}; if
 * pieces != NULL, up to cap
 * pieces as {tile_x, tile_y, z0, z1} (outputs in planes [z0, z1) of tile
 * (tile_x, tile_y)).  Tiles split the cube evenly: tile j outputs rows
 * [j*ny/nty, (j+1)*ny/nty) and tile i columns [c(i), c(i+1)), where c(i) is
 * i*nx/ntx rounded up to a multiple of V and c(ntx) = nx (integer division
 * throughout); no tile exceeds ox columns or oy rows.  *count receives the
 * number. */
ig_status ig_schedule_plan(const ig_params* p, const ig_schedule* s, int32_t t_block, int32_t ncu,
                           int32_t* geom, int32_t* pieces, int64_t cap, int64_t* count);

/* Host-only: the schedule a filter created with p and no schedule runs
 * (kind BLOCKED or NAIVE, all fields resolved). */
ig_status ig_schedule_auto(const ig_params* p, ig_schedule* out);

/* Host-only: the workgroups of the same pass.  When the balanced split would
 * leave workgroups unequal (the tile count does not divide the workgroups),
 * each workgroup instead runs a contiguous share of the pieces in turn:
 * *nwg receives the number of workgroups and, if first != NULL, up to cap
 * entries of first[0..nwg] (workgroup b runs pieces [first[b], first[b+1])
 * of ig_schedule_plan's list).  *nwg = 0: one piece per workgroup. */
ig_status ig_schedule_plan_groups(const ig_params* p, const ig_schedule* s, int32_t t_block, int32_t ncu,
                                  int32_t* first, int64_t cap, int64_t* nwg);

/* Replace the filter parameters of f (conductance, K, tau, n_iter, C, rms) in
 * place.  The shape and storage type must stay those f was created with
 * (else IG_ERR_INVALID_ARG); the scratch cube, the schedule and its piece
 * tables are kept, so a series of runs with different parameters on one cube
 * (a parameter sweep) allocates nothing.  Host only; not to be called while
 * a run of f is being enqueued from another thread. */
ig_status ig_filter_set_params(ig_filter* f, const ig_params* p);

/* Release the handle and its device memory (NULL is a no-op). */
void ig_filter_destroy(ig_filter* f);

/* One cube of a batch: its own parameters and caller-owned buffers.
 * d_in == d_out is allowed; items must not share buffers otherwise. */
typedef struct {
    ig_params p;
    const void* d_in;
    void* d_out;
} ig_batch_item;

/* Filter `count` independent cubes of uneven sizes and parameters with one
 * graph launch (all items: FP32 storage, same device).  The graph holds the
 * per-cube noise-level scans, one launch for the LDS-resident cubes (below)
 * and either one kernel launch per pass round (round r: pass r of every other
 * cube that has one) or, with ig_batch_set_launch(1), one persistent launch
 * that runs every pass of every cube: its workgroups take (cube, pass, piece)
 * items in pass-major order from a device counter and start a piece once the
 * cube's previous pass is done.  A dependency wait that lasts more than 2 s
 * marks every item failed, sets every output to NaN and makes a waiting call
 * return IG_ERR_DEVICE.  The graph is built once per batch signature (item shapes and
 * parameters, whether each item runs in place, the buffers' alignment within
 * 16 bytes, and the batch settings) and replayed on later calls with the same
 * signature; a call with other buffers of the same signature rewrites the
 * plan's table of buffer addresses (an asynchronous copy on the stream, after
 * the plan's previous launch has finished) before the launch.  At most 8
 * plans are cached; building a ninth drops the least recently used one (after
 * its last launch has finished).  Scratch cubes for the ping-pong are owned by
 * the cached plan (ig_batch_cache_clear frees them).  A cube of at most the
 * resident limit of voxels (ig_batch_set_resident; default 32768, 128 KiB)
 * with n_iter > 0 runs LDS-resident: one workgroup loads it into LDS, runs all
 * n_iter steps there and writes the result, bitwise what the passes give; its
 * stats report passes = 1, schedule.t_block = n_iter and schedule.waves = the
 * wavefronts of its workgroup (sized to the cube: 1 to 16).  An item whose
 * input holds NaN or Inf runs no step and its output is set to NaN; the call
 * then returns IG_ERR_NONFINITE if it waits (per_item or latency_ms given).
 * per_item (nullable, `count` entries) receives each item's stats; latency_ms
 * (nullable, `count` entries) receives each cube's completion time measured
 * on the GPU clock from the start of the launch.  Either makes the call wait
 * for the stream. */
ig_status ig_filter_batch(const ig_batch_item* items, int32_t count, int device, void* hip_stream,
                          ig_stats* per_item, double* latency_ms);

/* Free every cached batch plan (graphs and scratch) on every device, after
 * each plan's last launch has finished. */
void ig_batch_cache_clear(void);

/* Number of batch plans cached (at most 8). */
int32_t ig_batch_cache_size(void);

/* Schedule of later ig_filter_batch plans: steps per pass t_block (1..4; 0 =
 * library default), wavefronts per workgroup (1..16, > 2 t_block) and planes
 * per z-chunk of a piece (1..4096; default 32).  All items of a batch must
 * share one conductance, and those not run LDS-resident need nx <= 256. */
ig_status ig_batch_set_schedule(int32_t t_block, int32_t waves, int32_t zchunk);

/* Launch mode of later ig_filter_batch plans: 0 (default) one launch per
 * pass round, 1 one persistent launch (see ig_filter_batch); results are
 * bitwise the same.  Host only.  Errors: IG_ERR_INVALID_ARG for other
 * values.  ig_batch_get_launch returns the current mode. */
ig_status ig_batch_set_launch(int32_t persistent);
int32_t ig_batch_get_launch(void);

/* Resident limit of later ig_filter_batch plans: cubes of at most max_voxels
 * voxels (0..32768; 0 = none) run LDS-resident.  Host only.  Errors:
 * IG_ERR_INVALID_ARG outside that range. */
ig_status ig_batch_set_resident(int32_t max_voxels);

/* The current resident limit (IG_ERR_INVALID_ARG for NULL). */
ig_status ig_batch_get_resident(int32_t* max_voxels);

/* Batch autotuner: runs the batch with t_block 1..4, waves 8, 12 and 16,
 * z-chunks of 16, 32 and 64 planes, both launch modes, and, when some cube is
 * small enough, with the resident limit at 32768 and at 0; keeps the fastest
 * (sets it as by ig_batch_set_schedule, ig_batch_set_launch and
 * ig_batch_set_resident, and keeps only that plan cached) and returns the
 * schedule (the launch mode through ig_batch_get_launch, the resident limit
 * through ig_batch_get_resident).  Every item must have d_in != d_out (outputs are
 * overwritten; inputs are read only).  Waits for the stream. */
ig_status ig_batch_autotune(const ig_batch_item* items, int32_t count, int device, void* hip_stream,
                            int32_t* best_t_block, int32_t* best_waves, int32_t* best_zchunk, double* best_ms);

/* Comparison of a device cube with an FP64 device reference (both n
 * elements): maximum |x - ref|, root mean square of x - ref, count of
 * |x - ref| > tol, maximum |ref|, sum of x and of ref; FP64 accumulation in
 * a fixed order.  Waits for the stream. */
typedef struct {
    double max_abs;
    double rms;
    double max_ref;
    double sum_x;
    double sum_ref;
    int64_t n_over;
} ig_compare_result;

ig_status ig_compare(const void* d_x, int32_t x_dtype, const double* d_ref, int64_t n, double tol,
                     int device, void* hip_stream, ig_compare_result* res);

/* FP64 sum, sum of squares and non-finite count of a device cube (the
 * reductions behind the rms estimate and the conservation check).  Waits. */
ig_status ig_reduce(const void* d_x, int32_t x_dtype, int64_t n, int device, void* hip_stream,
                    double* sum, double* sumsq, int64_t* nonfinite);

const char* ig_status_string(ig_status s);
const char* ig_last_error(void);
/* Library version as "major.minor.patch". */
const char* ig_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IGFILTER_H */
