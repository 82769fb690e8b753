// Filtering-quality diagnostics (Section 6): masked FP64 sums over a region
// of interest for a sweep of mask thresholds, then F, sigma_F, F_M, sigma_FM.
// See include/igquality.h.
//
// Partial sums live in 192 FP64 slots per partial: slot 3j + {0, 1, 2} holds
// (sum of original values, sum of model values, voxel count) under mask j,
// j < n_thr for the M_f thresholds and j = 63 for M_o (whose model slot is the
// unmasked model sum).  Two ways to produce the partials, both with a fixed
// work split and fixed-order sums, so results are bitwise reproducible run to
// run (no atomics):
//
//  * up to 8 thresholds (the sweep's case): voxel-parallel.  Each thread keeps
//    every mask's sums in registers and walks its voxels in a fixed order
//    (a contiguous range of ROI rows per workgroup, four loads in flight per
//    thread); a fixed shuffle tree and the wavefronts in order make one
//    partial per workgroup.  Bound by HBM.
//  * more thresholds: lane j of every wavefront owns mask j.  A wavefront
//    takes 64-voxel chunks in a fixed order, parks each chunk's three values
//    as FP64 in its LDS slice, and every lane walks the 64 voxels in order
//    (a uniform-address LDS read is a broadcast).  One partial per wavefront.
//
// k_quality_fold folds each slot over the partials (block b folds slot b:
// strided per-thread sums, then a fixed tree); k_quality_derive turns the 192
// sums into the diagnostics.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "igquality.h"
#include "internal.h"

namespace igk {

struct QGeom {
    long nx, ny;          // row and plane strides of the cube
    long x0, y0, z0;      // ROI origin
    long rx, ry;          // ROI extents in x and y
    long nroi;            // voxels in the ROI
    long nrows;           // ROI rows (ry * rz)
    int has_model;
    int pad;
    double thr[64];       // absolute threshold per mask (+inf: unused)
};

constexpr int kQWaves = 4;          // wavefronts per workgroup
constexpr int kQMaxBlocks = 1024;
constexpr int kQSlots = 192;        // 64 masks x (orig sum, model sum, count)
constexpr int kQSeg = 256;          // row-segment length of the voxel-parallel kernel

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int K>
__global__ void __launch_bounds__(256)
k_quality_vox(const float* __restrict__ orig, const float* __restrict__ filt, const float* __restrict__ model,
              QGeom g, double* __restrict__ part) {
    constexpr int NA = 3 * (K + 1);
    double acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = 0.0;
    double thr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) thr[k] = g.thr[k];
    const double thr_o = g.thr[63];
    // workgroup b takes a contiguous range of ROI rows (sequential memory),
    // (y, z) carried from row to row; within a row, thread t takes voxels
    // t, t + kQSeg, ... (kQUnroll loads of each cube in flight: every lane
    // loads, at x clamped into the row, and lanes past the row skip the sums;
    // loads under a branch made the compiler wait for each one in turn)
    constexpr int kQUnroll = 4;
    const float* mp = g.has_model ? model : orig;   // any readable cube when there is no model
    const long per = (g.nrows + gridDim.x - 1) / gridDim.x;
    const long r0 = (long)blockIdx.x * per, r1 = min(g.nrows, r0 + per);
    long y = r0 % g.ry, z = r0 / g.ry;
    for (long row = r0; row < r1; ++row) {
        const long base = g.x0 + g.nx * ((g.y0 + y) + g.ny * (g.z0 + z));
        for (long x0 = 0; x0 < g.rx; x0 += (long)kQSeg * kQUnroll) {
            float fo[kQUnroll], ff[kQUnroll], fm[kQUnroll];
            bool in[kQUnroll];
#pragma unroll
            for (int u = 0; u < kQUnroll; ++u) {
                const long x = x0 + u * kQSeg + threadIdx.x;
                const long xc = min(x, g.rx - 1);
                in[u] = x < g.rx;
                fo[u] = orig[base + xc];
                ff[u] = filt[base + xc];
                fm[u] = mp[base + xc];
            }
#pragma unroll
            for (int u = 0; u < kQUnroll; ++u) {
                if (!in[u]) continue;
                const double o = (double)fo[u], f = (double)ff[u], m = g.has_model ? (double)fm[u] : 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const bool p = f >= thr[k];
                    acc[3 * k] += p ? o : 0.0;
                    acc[3 * k + 1] += p ? m : 0.0;
                    acc[3 * k + 2] += p ? 1.0 : 0.0;
                }
                const bool po = o >= thr_o;
                acc[3 * K] += po ? o : 0.0;
                acc[3 * K + 1] += m;
                acc[3 * K + 2] += po ? 1.0 : 0.0;
            }
        }
        if (++y == g.ry) {
            y = 0;
            ++z;
        }
    }
    __shared__ double red[kQWaves][NA];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        const double v = wsum(acc[a]);
        if (lane == 0) red[wid][a] = v;
    }
    __syncthreads();
    double* out = part + (long)blockIdx.x * kQSlots;
    for (int sl = threadIdx.x; sl < kQSlots; sl += 256) {
        const int j = sl / 3, c = sl % 3;
        const int a = j < K ? 3 * j + c : (j == 63 ? 3 * K + c : -1);
        double v = 0.0;
        if (a >= 0)
            for (int w = 0; w < kQWaves; ++w) v += red[w][a];
        out[sl] = v;
    }
}

__global__ void __launch_bounds__(256)
k_quality_lanes(const float* __restrict__ orig, const float* __restrict__ filt, const float* __restrict__ model,
                QGeom g, double* __restrict__ part) {
    __shared__ double vals[kQWaves][64][3];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const long nw = (long)gridDim.x * kQWaves;
    const long gw = (long)blockIdx.x * kQWaves + wid;
    const double thr = g.thr[lane];
    const bool mo = lane == 63;
    double a1 = 0.0, a2 = 0.0, c = 0.0;
    for (long ch = gw; ch * 64 < g.nroi; ch += nw) {
        const long r = ch * 64 + lane;
        double vo = 0.0, vf = 0.0, vm = 0.0;
        if (r < g.nroi) {
            const long x = r % g.rx, t = r / g.rx;
            const long y = t % g.ry, z = t / g.ry;
            const long idx = (g.x0 + x) + g.nx * ((g.y0 + y) + g.ny * (g.z0 + z));
            vo = (double)orig[idx];
            vf = (double)filt[idx];
            if (g.has_model) vm = (double)model[idx];
        }
        vals[wid][lane][0] = vo;
        vals[wid][lane][1] = vf;
        vals[wid][lane][2] = vm;
        __builtin_amdgcn_wave_barrier();
        const int nv = (int)min(64L, g.nroi - ch * 64);
        for (int k = 0; k < nv; ++k) {
            const double so = vals[wid][k][0], sf = vals[wid][k][1], sm = vals[wid][k][2];
            const bool pass = mo ? (so >= thr) : (sf >= thr);
            a1 += pass ? so : 0.0;
            a2 += (pass || mo) ? sm : 0.0;
            c += pass ? 1.0 : 0.0;
        }
        __builtin_amdgcn_wave_barrier();
    }
    double* out = part + gw * kQSlots;
    out[3 * lane] = a1;
    out[3 * lane + 1] = a2;
    out[3 * lane + 2] = c;
}

// Block b folds slot b over `count` partials: thread t sums partials t,
// t + 256, ... in order, then a fixed tree over the threads.
__global__ void __launch_bounds__(256)
k_quality_fold(const double* __restrict__ part, long count, double* __restrict__ sums) {
    const int sl = blockIdx.x;
    double v = 0.0;
    for (long i = threadIdx.x; i < count; i += 256) v += part[i * kQSlots + sl];
    v = wsum(v);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) sums[sl] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// One wavefront: lane j derives the diagnostics of mask j.
__global__ void __launch_bounds__(64)
k_quality_derive(const double* __restrict__ sums, int nthr, int has_model, double rms_o, double rms_f, double indep,
                 long nroi, ig_quality_result* __restrict__ out) {
    const int j = threadIdx.x;
    const double s1 = sums[3 * j], s2 = sums[3 * j + 1];
    const long long n = (long long)sums[3 * j + 2];
    const double S_oo = sums[3 * 63], S_m = sums[3 * 63 + 1];
    const long long N_o = (long long)sums[3 * 63 + 2];
    const double nan = __builtin_nan("");
    if (j == 63) {
        out->rms_o = rms_o;
        out->rms_f = rms_f;
        out->S_oo = S_oo;
        out->S_m = has_model ? S_m : 0.0;
        out->N_o = N_o;
        out->n_roi = nroi;
    }
    if (j < IG_QUALITY_MAX_THR) {
        const bool on = j < nthr;
        const double sig_oo = sqrt((double)N_o / indep) * rms_o;
        const double sig_of = sqrt((double)n / indep) * rms_f;
        double F = nan, sF = nan, FM = nan, sFM = nan;
        if (on && S_oo != 0.0) {
            F = fabs(s1) / fabs(S_oo);
            sF = sqrt(sig_of * sig_of / (S_oo * S_oo) + s1 * s1 * sig_oo * sig_oo / (S_oo * S_oo * S_oo * S_oo));
        }
        if (on && has_model && S_m != 0.0) {
            FM = fabs(s2) / fabs(S_m);
            sFM = sig_of / fabs(S_m);
        }
        out->S_of[j] = on ? s1 : 0.0;
        out->S_mf[j] = on && has_model ? s2 : 0.0;
        out->N_f[j] = on ? n : 0;
        out->F[j] = F;
        out->sigma_F[j] = sF;
        out->F_M[j] = FM;
        out->sigma_FM[j] = sFM;
    }
}

}  // namespace igk

// ====================================================================== host
using namespace igk;
#define fail igk_fail
#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                             \
    } while (0)

namespace {

struct QScratch {   // per-device partials, folded sums and result slot, kept for the process
    double* part = nullptr;
    double* sums = nullptr;
    ig_quality_result* res = nullptr;
};
std::mutex g_qmu;
QScratch g_qs[64];

ig_status noise_level(const float* d, long n, int device, void* stream, double given, double* rms) {
    if (given > 0.0) {
        *rms = given;
        return IG_OK;
    }
    double sum = 0.0, sumsq = 0.0;
    int64_t bad = 0;
    ig_status st = ig_reduce(d, IG_F32, n, device, stream, &sum, &sumsq, &bad);
    if (st != IG_OK) return st;
    if (bad) return fail(IG_ERR_NONFINITE, "a cube whose rms is to be estimated holds %lld non-finite voxels",
                         (long long)bad);
    *rms = n > 0 ? std::sqrt(sumsq / (double)n) : 0.0;
    return IG_OK;
}

}  // namespace

extern "C" ig_status ig_quality(const ig_quality_params* q, const float* d_orig, const float* d_filt,
                                const float* d_model, int64_t nx, int64_t ny, int64_t nz, int device,
                                void* hip_stream, ig_quality_result* out) {
    if (!q || !out || !d_orig || !d_filt) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    if (q->struct_size != (int32_t)sizeof(ig_quality_params)) return fail(IG_ERR_INVALID_ARG, "struct_size");
    if (nx < 1 || ny < 1 || nz < 1) return fail(IG_ERR_INVALID_ARG, "bad cube size");
    if (q->n_thr < 1 || q->n_thr > IG_QUALITY_MAX_THR) return fail(IG_ERR_INVALID_ARG, "n_thr out of range");
    for (int j = 0; j < q->n_thr; ++j)
        if (!std::isfinite(q->thr_f[j])) return fail(IG_ERR_INVALID_ARG, "thr_f[%d] is not finite", j);
    if (!std::isfinite(q->thr_o)) return fail(IG_ERR_INVALID_ARG, "thr_o is not finite");
    if (!(q->indep > 0.0) || !std::isfinite(q->indep)) return fail(IG_ERR_INVALID_ARG, "indep must be > 0");
    if (!std::isfinite(q->rms_o) || !std::isfinite(q->rms_f)) return fail(IG_ERR_INVALID_ARG, "rms not finite");
    int64_t r[6] = {q->roi[0], q->roi[1], q->roi[2], q->roi[3], q->roi[4], q->roi[5]};
    if (!(r[0] | r[1] | r[2] | r[3] | r[4] | r[5])) {
        r[1] = nx; r[3] = ny; r[5] = nz;
    }
    if (r[0] < 0 || r[1] > nx || r[0] >= r[1] || r[2] < 0 || r[3] > ny || r[2] >= r[3] || r[4] < 0 || r[5] > nz ||
        r[4] >= r[5])
        return fail(IG_ERR_INVALID_ARG, "ROI empty or outside the cube");
    if (device < 0 || device >= 64) return fail(IG_ERR_INVALID_ARG, "bad device %d", device);
    {
        const size_t bytes = (size_t)(nx * ny * nz) * 4;
        ig_status cb = igk_check_buffer(d_orig, bytes, device, "d_orig");
        if (cb == IG_OK) cb = igk_check_buffer(d_filt, bytes, device, "d_filt");
        if (cb == IG_OK && d_model) cb = igk_check_buffer(d_model, bytes, device, "d_model");
        if (cb != IG_OK) return cb;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice(%d)", device);
    struct Restore { int d; ~Restore() { if (d >= 0) (void)hipSetDevice(d); } } restore{prev};
    hipStream_t s = (hipStream_t)hip_stream;

    const long n = (long)(nx * ny * nz);
    double rms_o = 0.0, rms_f = 0.0;
    ig_status st = noise_level(d_orig, n, device, hip_stream, q->rms_o, &rms_o);
    if (st != IG_OK) return st;
    st = noise_level(d_filt, n, device, hip_stream, q->rms_f, &rms_f);
    if (st != IG_OK) return st;

    QGeom g{};
    g.nx = nx; g.ny = ny;
    g.x0 = r[0]; g.y0 = r[2]; g.z0 = r[4];
    g.rx = r[1] - r[0]; g.ry = r[3] - r[2];
    g.nroi = g.rx * g.ry * (r[5] - r[4]);
    g.has_model = d_model != nullptr;
    for (int j = 0; j < 64; ++j) g.thr[j] = INFINITY;
    for (int j = 0; j < q->n_thr; ++j) g.thr[j] = q->thr_f[j] * rms_f;
    g.thr[63] = q->thr_o * rms_o;

    g.nrows = g.ry * (r[5] - r[4]);
    std::lock_guard<std::mutex> lk(g_qmu);
    QScratch& qs = g_qs[device];
    if (!qs.part) {   // all three or none: a failure leaves the cache empty
        QScratch fresh{};
        hipError_t e = igk_malloc((void**)&fresh.part, (size_t)kQMaxBlocks * kQWaves * kQSlots * sizeof(double));
        if (e == hipSuccess) e = igk_malloc((void**)&fresh.sums, (size_t)kQSlots * sizeof(double));
        if (e == hipSuccess) e = igk_malloc((void**)&fresh.res, sizeof(ig_quality_result));
        if (e != hipSuccess) {
            igk_free(fresh.part);
            igk_free(fresh.sums);
            igk_free(fresh.res);
            return fail(e == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "quality scratch: %s",
                        hipGetErrorString(e));
        }
        qs = fresh;
    }
    long count;
    if (q->n_thr <= 8) {
        const int K = q->n_thr <= 1 ? 1 : q->n_thr <= 2 ? 2 : q->n_thr <= 4 ? 4 : 8;
        const int blocks = (int)std::min<long>(kQMaxBlocks * 2, g.nrows);
        auto k = K == 1 ? k_quality_vox<1> : K == 2 ? k_quality_vox<2> : K == 4 ? k_quality_vox<4> : k_quality_vox<8>;
        hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, s, d_orig, d_filt, d_model, g, qs.part);
        count = blocks;
    } else {
        const long chunks = (g.nroi + 63) / 64;
        const int blocks = (int)std::min<long>(kQMaxBlocks, (chunks + kQWaves - 1) / kQWaves);
        hipLaunchKernelGGL(k_quality_lanes, dim3(blocks), dim3(64 * kQWaves), 0, s, d_orig, d_filt, d_model, g,
                           qs.part);
        count = (long)blocks * kQWaves;
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_quality_fold, dim3(kQSlots), dim3(256), 0, s, qs.part, count, qs.sums);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_quality_derive, dim3(1), dim3(64), 0, s, qs.sums, q->n_thr, g.has_model, rms_o, rms_f,
                       q->indep, g.nroi, qs.res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, qs.res, sizeof(ig_quality_result), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return IG_OK;
}

// Free the per-device quality scratch (the next ig_quality allocates it again).
void igk_quality_cache_release() {
    std::lock_guard<std::mutex> lk(g_qmu);
    int prev = -1;
    (void)hipGetDevice(&prev);
    for (int d = 0; d < 64; ++d) {
        QScratch& qs = g_qs[d];
        if (!qs.part && !qs.sums && !qs.res) continue;
        (void)hipSetDevice(d);
        igk_free(qs.part);
        igk_free(qs.sums);
        igk_free(qs.res);
        qs = QScratch{};
    }
    if (prev >= 0) (void)hipSetDevice(prev);
}
