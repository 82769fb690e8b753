// Wavelet lifting (Haar, Le Gall 5/3) and the thresholding denoiser of
// Section 3.4; see include/igwavelet.h.
//
// A workgroup lifts whole lines held in LDS in interleaved order: the predict
// step overwrites the odd slots with the details (it reads even slots only),
// the update step overwrites the even slots with the approximations (it reads
// odd slots only), so one LDS line per line suffices and every step is a
// parallel loop over the line.  Lines along x: 4 lines per workgroup, lanes
// along the line (coalesced).  Lines along y or z: W lines of consecutive x
// per workgroup (W = 64, 32 or 16, what LDS allows), lanes across the lines
// (coalesced), rows of threads along the line.  Stores de-interleave into
// [approximations, details].
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>

#include "igwavelet.h"
#include "internal.h"

namespace igk {

constexpr int kWHaar = IG_WAVELET_HAAR;
constexpr int kLinesX = 4;
constexpr int kMaxLineX = 10240;
constexpr int kMaxLineYZ = 2560;

struct LiftGeom {
    long nx, ny;      // cube strides
    long bx, by, bz;  // current box
    // denoiser only, on the first inverse pass of level 1: a coefficient
    // outside the box [0, ax) x [0, ay) x [0, az) (a detail of level 1, not
    // touched since the forward transform) is set to 0 as it is loaded when
    // |c| < athr, the threshold pass's rule for that level
    long ax, ay, az;
    double athr;
    int thr_on;
};

__device__ __forceinline__ float thr_load(float v, long x, long y, long z, const LiftGeom& g) {
    const bool detail1 = x >= g.ax || y >= g.ay || z >= g.az;
    return (detail1 && !(fabs((double)v) >= g.athr)) ? 0.0f : v;
}

// One lifting direction over the LDS line X (element i at X[i * es]), n >= 2;
// this thread handles elements e0, e0 + step, ...  Ends every step with a
// workgroup barrier (all threads call it).
template <int KIND>
__device__ __forceinline__ void lift_forward(float* X, int es, int n, int e0, int step, bool active) {
    const int ne = (n + 1) / 2, no = n / 2;
    if (active)
        for (int i = e0; i < no; i += step) {
            const float ev = X[(2 * i) * es];
            if constexpr (KIND == kWHaar) {
                X[(2 * i + 1) * es] = X[(2 * i + 1) * es] - ev;
            } else {
                const float right = 2 * i + 2 < n ? X[(2 * i + 2) * es] : ev;
                X[(2 * i + 1) * es] = X[(2 * i + 1) * es] - (ev + right) * 0.5f;
            }
        }
    __syncthreads();
    if (active)
        for (int i = e0; i < ne; i += step) {
            if constexpr (KIND == kWHaar) {
                if (i < no) X[(2 * i) * es] = X[(2 * i) * es] + X[(2 * i + 1) * es] * 0.5f;
            } else {
                const float dl = i > 0 ? X[(2 * i - 1) * es] : X[1 * es];
                const float dr = i < no ? X[(2 * i + 1) * es] : X[(2 * i - 1) * es];
                X[(2 * i) * es] = X[(2 * i) * es] + (dl + dr) * 0.25f;
            }
        }
    __syncthreads();
}

template <int KIND>
__device__ __forceinline__ void lift_inverse(float* X, int es, int n, int e0, int step, bool active) {
    const int ne = (n + 1) / 2, no = n / 2;
    if (active)
        for (int i = e0; i < ne; i += step) {
            if constexpr (KIND == kWHaar) {
                if (i < no) X[(2 * i) * es] = X[(2 * i) * es] - X[(2 * i + 1) * es] * 0.5f;
            } else {
                const float dl = i > 0 ? X[(2 * i - 1) * es] : X[1 * es];
                const float dr = i < no ? X[(2 * i + 1) * es] : X[(2 * i - 1) * es];
                X[(2 * i) * es] = X[(2 * i) * es] - (dl + dr) * 0.25f;
            }
        }
    __syncthreads();
    if (active)
        for (int i = e0; i < no; i += step) {
            const float ev = X[(2 * i) * es];
            if constexpr (KIND == kWHaar) {
                X[(2 * i + 1) * es] = X[(2 * i + 1) * es] + ev;
            } else {
                const float right = 2 * i + 2 < n ? X[(2 * i + 2) * es] : ev;
                X[(2 * i + 1) * es] = X[(2 * i + 1) * es] + (ev + right) * 0.5f;
            }
        }
    __syncthreads();
}

// slot in the interleaved line of stored position j (approximations first)
__device__ __forceinline__ int slot_of(int j, int ne) { return j < ne ? 2 * j : 2 * (j - ne) + 1; }

// Lines along x: kLinesX lines per workgroup of 64 x kLinesX threads.
template <bool FWD, int KIND>
__global__ void __launch_bounds__(256)
k_lift_x(const float* __restrict__ src, float* __restrict__ dst, LiftGeom g) {
    extern __shared__ float X[];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int n = (int)g.bx, ne = (n + 1) / 2;
    const long L = (long)blockIdx.x * kLinesX + ty;
    const bool active = L < g.by * g.bz;
    const long y = active ? L % g.by : 0, z = active ? L / g.by : 0;
    const long base = g.nx * (y + g.ny * z);
    float* line = X + ty * n;
    // loads in groups of 8, each group in flight together before its LDS
    // writes: every lane loads, at an index clamped into the line (a lane past
    // the line or the box does not write the value), since loads under a
    // branch made the compiler wait for each pair before issuing the next
    for (int j0 = tx; j0 < n; j0 += 64 * 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + 64 * u;
            v[u] = src[base + min(j, n - 1)];
        }
        if (!FWD && g.thr_on)
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = thr_load(v[u], j0 + 64 * u, y, z, g);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + 64 * u;
            if (active && j < n) line[FWD ? j : slot_of(j, ne)] = v[u];
        }
    }
    __syncthreads();
    if (FWD) lift_forward<KIND>(line, 1, n, tx, 64, active);
    else lift_inverse<KIND>(line, 1, n, tx, 64, active);
    if (active)
        for (int j = tx; j < n; j += 64) dst[base + j] = line[FWD ? slot_of(j, ne) : j];
}

// Lines along y (AXIS 1) or z (AXIS 2): W lines of consecutive x per
// workgroup of W x (256 / W) threads.
template <bool FWD, int KIND, int AXIS>
__global__ void __launch_bounds__(256)
k_lift_yz(const float* __restrict__ src, float* __restrict__ dst, LiftGeom g, int W) {
    extern __shared__ float X[];
    const int tx = threadIdx.x, ty = threadIdx.y, rows = blockDim.y;
    const int n = (int)(AXIS == 1 ? g.by : g.bz), ne = (n + 1) / 2;
    const long x = (long)blockIdx.x * W + tx;
    const bool active = x < g.bx;
    const long other = blockIdx.y;   // z for lines along y, y for lines along z
    const long es = AXIS == 1 ? g.nx : g.nx * g.ny;
    const long base = x + (AXIS == 1 ? other * g.nx * g.ny : other * g.nx);
    const long basec = base - x + (active ? x : g.bx - 1);   // an in-box column for lanes past the box
    float* col = X + tx;
    // loads in groups of 8, each group in flight together before its LDS
    // writes: every lane loads, at indices clamped into the box (a lane past
    // the line or the box does not write the value), since loads under a
    // branch made the compiler wait for each pair before issuing the next
    for (int j0 = ty; j0 < n; j0 += rows * 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + rows * u;
            v[u] = src[basec + (long)min(j, n - 1) * es];
        }
        if (!FWD && g.thr_on)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const long j = j0 + rows * u;
                v[u] = AXIS == 1 ? thr_load(v[u], x, j, other, g) : thr_load(v[u], x, other, j, g);
            }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + rows * u;
            if (active && j < n) col[(FWD ? j : slot_of(j, ne)) * W] = v[u];
        }
    }
    __syncthreads();
    if (FWD) lift_forward<KIND>(col, W, n, ty, rows, active);
    else lift_inverse<KIND>(col, W, n, ty, rows, active);
    if (active)
        for (int j = ty; j < n; j += rows) dst[base + j * es] = col[(FWD ? slot_of(j, ne) : j) * W];
}

struct ThrGeom {
    long nx, ny, nz;
    int levels;
    int pad;
    long sx[IG_WAVELET_MAX_LEVELS + 1], sy[IG_WAVELET_MAX_LEVELS + 1], sz[IG_WAVELET_MAX_LEVELS + 1];
    double thr[IG_WAVELET_MAX_LEVELS + 1];   // level l at [l - 1]; the final approximation at [levels]
};

// one row segment of 256 voxels per workgroup: grid (ceil(nx / 256), ny, nz)
__global__ void __launch_bounds__(256) k_wthresh(float* __restrict__ c, ThrGeom g) {
    const long x = (long)blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x < g.nx) {
        const long i = x + g.nx * (y + g.ny * z);
        int lv = g.levels + 1;
        for (int l = 1; l <= g.levels; ++l)
            if (x >= g.sx[l] || y >= g.sy[l] || z >= g.sz[l]) {
                lv = l;
                break;
            }
        const float w = c[i];
        if (!(fabs((double)w) >= g.thr[lv - 1])) c[i] = 0.0f;
    }
}

}  // namespace igk

// ====================================================================== host
using namespace igk;
#define fail igk_fail

namespace {

ig_status check(const ig_wavelet_params* p, const void* a, const void* b, int64_t nx, int64_t ny, int64_t nz) {
    if (!p || !a || !b) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    if (p->struct_size != (int32_t)sizeof(ig_wavelet_params)) return fail(IG_ERR_INVALID_ARG, "struct_size");
    if (p->reserved != 0) return fail(IG_ERR_INVALID_ARG, "reserved must be 0");
    if (p->kind != IG_WAVELET_HAAR && p->kind != IG_WAVELET_LEGALL53) return fail(IG_ERR_INVALID_ARG, "bad kind");
    if (p->levels < 1 || p->levels > IG_WAVELET_MAX_LEVELS) return fail(IG_ERR_INVALID_ARG, "levels out of range");
    if (nx < 1 || ny < 1 || nz < 1 || nx * ny * nz >= (1LL << 34)) return fail(IG_ERR_INVALID_ARG, "bad cube size");
    if (nx > kMaxLineX) return fail(IG_ERR_UNSUPPORTED, "lines along x longer than %d", kMaxLineX);
    if (ny > kMaxLineYZ || nz > kMaxLineYZ) return fail(IG_ERR_UNSUPPORTED, "lines along y or z longer than %d", kMaxLineYZ);
    const size_t bytes = (size_t)(nx * ny * nz) * sizeof(float);
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    if (x != y && x < y + bytes && y < x + bytes) return fail(IG_ERR_INVALID_ARG, "buffers overlap partially");
    const int dev = igk_current_device();
    ig_status cb = igk_check_buffer(a, bytes, dev, "input cube");
    if (cb == IG_OK) cb = igk_check_buffer(b, bytes, dev, "output cube");
    return cb;
}

// Lines per workgroup along y or z: the widest whose LDS tile stays within
// 64 KiB (two or more workgroups per CU hide the loads of one another), else
// the widest that fits at all.
int lines_per_block(long n) {
    for (int W : {64, 32, 16})
        if ((size_t)n * W * sizeof(float) <= 65536) return W;
    for (int W : {64, 32, 16})
        if ((size_t)n * W * sizeof(float) <= kMaxLds) return W;
    return 0;
}

template <bool FWD, int KIND>
hipError_t pass(int axis, const float* src, float* dst, const LiftGeom& g, hipStream_t s) {
    if (axis == 0) {
        const size_t lds = (size_t)kLinesX * g.bx * sizeof(float);
        auto k = k_lift_x<FWD, KIND>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        const long lines = g.by * g.bz;
        hipLaunchKernelGGL(k, dim3((unsigned)((lines + kLinesX - 1) / kLinesX)), dim3(64, kLinesX), lds, s, src, dst, g);
        return hipGetLastError();
    }
    const long n = axis == 1 ? g.by : g.bz;
    const int W = lines_per_block(n);
    const size_t lds = (size_t)n * W * sizeof(float);
    auto k = axis == 1 ? k_lift_yz<FWD, KIND, 1> : k_lift_yz<FWD, KIND, 2>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const long other = axis == 1 ? g.bz : g.by;
    hipLaunchKernelGGL(k, dim3((unsigned)((g.bx + W - 1) / W), (unsigned)other), dim3(W, 256 / W), lds, s, src, dst, g,
                       W);
    return hipGetLastError();
}

template <bool FWD>
hipError_t run_pass(int kind, int axis, const float* src, float* dst, const LiftGeom& g, hipStream_t s) {
    return kind == IG_WAVELET_HAAR ? pass<FWD, kWHaar>(axis, src, dst, g, s)
                                   : pass<FWD, IG_WAVELET_LEGALL53>(axis, src, dst, g, s);
}

void box_sizes(int64_t nx, int64_t ny, int64_t nz, int levels, long (*sz)[3]) {
    sz[0][0] = nx; sz[0][1] = ny; sz[0][2] = nz;
    for (int l = 1; l <= levels; ++l)
        for (int a = 0; a < 3; ++a) sz[l][a] = (sz[l - 1][a] + 1) / 2;
}

ig_status forward_impl(const ig_wavelet_params* p, const float* d_in, float* d_coef, int64_t nx, int64_t ny,
                       int64_t nz, hipStream_t s) {
    long sz[IG_WAVELET_MAX_LEVELS + 1][3];
    box_sizes(nx, ny, nz, p->levels, sz);
    const float* src = d_in;
    for (int l = 0; l < p->levels; ++l) {
        LiftGeom g{nx, ny, sz[l][0], sz[l][1], sz[l][2]};
        for (int axis = 0; axis < 3; ++axis) {
            if (sz[l][axis] < 2) continue;
            hipError_t e = run_pass<true>(p->kind, axis, src, d_coef, g, s);
            if (e != hipSuccess) return fail(IG_ERR_DEVICE, "forward lifting: %s", hipGetErrorString(e));
            src = d_coef;
        }
    }
    if (src == d_in && d_in != d_coef) {   // nothing to lift (a 1 x 1 x 1 cube)
        hipError_t e = hipMemcpyAsync(d_coef, d_in, (size_t)(nx * ny * nz) * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(IG_ERR_DEVICE, "copy: %s", hipGetErrorString(e));
    }
    return IG_OK;
}

// athr >= 0: the denoiser's level-1 detail threshold, applied as the first
// pass of level 1 loads the coefficients (see LiftGeom)
ig_status inverse_impl(const ig_wavelet_params* p, const float* d_coef, float* d_out, int64_t nx, int64_t ny,
                       int64_t nz, hipStream_t s, double athr = -1.0) {
    if (d_coef != d_out) {
        hipError_t e = hipMemcpyAsync(d_out, d_coef, (size_t)(nx * ny * nz) * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(IG_ERR_DEVICE, "copy: %s", hipGetErrorString(e));
    }
    long sz[IG_WAVELET_MAX_LEVELS + 1][3];
    box_sizes(nx, ny, nz, p->levels, sz);
    for (int l = p->levels - 1; l >= 0; --l) {
        LiftGeom g{nx, ny, sz[l][0], sz[l][1], sz[l][2], sz[1][0], sz[1][1], sz[1][2], athr, 0};
        g.thr_on = l == 0 && athr >= 0.0;
        for (int axis = 2; axis >= 0; --axis) {
            if (sz[l][axis] < 2) continue;
            hipError_t e = run_pass<false>(p->kind, axis, d_out, d_out, g, s);
            if (e != hipSuccess) return fail(IG_ERR_DEVICE, "inverse lifting: %s", hipGetErrorString(e));
            g.thr_on = 0;
        }
    }
    return IG_OK;
}

}  // namespace

extern "C" ig_status ig_wavelet_forward(const ig_wavelet_params* p, const float* d_in, float* d_coef, int64_t nx,
                                        int64_t ny, int64_t nz, void* hip_stream) {
    ig_status st = check(p, d_in, d_coef, nx, ny, nz);
    if (st != IG_OK) return st;
    return forward_impl(p, d_in, d_coef, nx, ny, nz, (hipStream_t)hip_stream);
}

extern "C" ig_status ig_wavelet_inverse(const ig_wavelet_params* p, const float* d_coef, float* d_out, int64_t nx,
                                        int64_t ny, int64_t nz, void* hip_stream) {
    ig_status st = check(p, d_coef, d_out, nx, ny, nz);
    if (st != IG_OK) return st;
    return inverse_impl(p, d_coef, d_out, nx, ny, nz, (hipStream_t)hip_stream);
}

extern "C" ig_status ig_wavelet_denoise(const ig_wavelet_params* p, const float* d_in, float* d_out, int64_t nx,
                                        int64_t ny, int64_t nz, void* hip_stream, double* rms_used) {
    ig_status st = check(p, d_in, d_out, nx, ny, nz);
    if (st != IG_OK) return st;
    for (int l = 0; l < p->levels; ++l)
        if (!std::isfinite(p->t[l]) || p->t[l] < 0.0) return fail(IG_ERR_INVALID_ARG, "bad threshold t[%d]", l);
    if (!std::isfinite(p->rms)) return fail(IG_ERR_INVALID_ARG, "rms not finite");
    hipStream_t s = (hipStream_t)hip_stream;
    double rms = p->rms;
    if (!(rms > 0.0)) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        double sum = 0.0, sumsq = 0.0;
        int64_t bad = 0;
        const long n = (long)(nx * ny * nz);
        st = ig_reduce(d_in, IG_F32, n, dev, hip_stream, &sum, &sumsq, &bad);
        if (st != IG_OK) return st;
        if (bad) return fail(IG_ERR_NONFINITE, "the input holds %lld non-finite voxels", (long long)bad);
        rms = std::sqrt(sumsq / (double)n);
    }
    if (rms_used) *rms_used = rms;
    st = forward_impl(p, d_in, d_out, nx, ny, nz, s);
    if (st != IG_OK) return st;
    ThrGeom g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.levels = p->levels;
    long sz[IG_WAVELET_MAX_LEVELS + 1][3];
    box_sizes(nx, ny, nz, p->levels, sz);
    for (int l = 0; l <= p->levels; ++l) {
        g.sx[l] = sz[l][0]; g.sy[l] = sz[l][1]; g.sz[l] = sz[l][2];
    }
    for (int l = 0; l < p->levels; ++l) g.thr[l] = p->t[l] * rms;
    g.thr[p->levels] = p->t[p->levels - 1] * rms;
    // The threshold pass covers the level-1 approximation box only (the
    // coefficients of levels 2 and up and the final approximation); the
    // level-1 details around it are thresholded by the inverse transform's
    // first level-1 pass as it loads them, so that pass reads the cube once
    // for both.  ny, nz <= kMaxLineYZ and nx <= kMaxLineX keep the grid within
    // its limits.
    hipLaunchKernelGGL(k_wthresh, dim3((unsigned)((sz[1][0] + 255) / 256), (unsigned)sz[1][1], (unsigned)sz[1][2]),
                       dim3(256), 0, s, d_out, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(IG_ERR_DEVICE, "threshold: %s", hipGetErrorString(e));
    return inverse_impl(p, d_out, d_out, nx, ny, nz, s, g.thr[0]);
}
