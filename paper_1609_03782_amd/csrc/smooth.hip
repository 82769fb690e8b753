// Box and Gaussian smoothing (Section 3.1-3.2); see include/igsmooth.h.
//
// Separable kernels (box, axis-aligned Gaussian): 1-D sums along x, y and z,
// each divided by the sum of the weights of its in-cube taps (the product of
// the three per-axis renormalisations is the 3-D one), with the weights
// computed in FP64 at block start.  Half-widths up to 8: one fused pass that
// streams the cube along z (k_sep3_t).  Otherwise three passes x -> out,
// y -> work, z -> out, each staging a segment of its axis plus the halo in LDS
// (coalesced loads along x).
//
// Rotated Gaussian: one dense pass.  A workgroup of 64 x 4 threads owns an
// output tile of 64 x 4 x TZ voxels, stages the input tile plus halo and the
// (2r_z+1)(2r_y+1)(2r_x+1) weights in LDS, and each thread accumulates TZ
// outputs along z, so a weight read from LDS serves TZ products.  Tiles whose
// input window crosses a cube face also accumulate the weights of their
// in-cube taps for the renormalisation; interior tiles divide by the total.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>

#include "igsmooth.h"
#include "internal.h"

namespace igk {

constexpr int kSepMaxR = 31;
constexpr int kSepSeg = 64;     // outputs per column segment (y and z passes)
constexpr int kSepRow = 256;    // outputs per row segment (x pass)

struct SepGeom {
    long nx, ny, nz;
    int r;
    int kind;        // IG_SMOOTH_BOX / IG_SMOOTH_GAUSS
    double sigma;    // Gaussian sigma along this axis
};

__device__ __forceinline__ void sep_weights(const SepGeom& g, float* w) {
    for (int k = threadIdx.x + threadIdx.y * blockDim.x; k <= 2 * g.r; k += blockDim.x * blockDim.y) {
        const double d = (double)(k - g.r);
        w[k] = g.kind == IG_SMOOTH_BOX ? 1.0f : (float)exp(-d * d / (2.0 * g.sigma * g.sigma));
    }
}

// x pass: row segments of kSepRow outputs, kSepRowsX rows per workgroup of
// kSepRow threads (the weights are computed once per workgroup).
constexpr int kSepRowsX = 8;
__global__ void __launch_bounds__(kSepRow)
k_sep_x(const float* __restrict__ src, float* __restrict__ dst, SepGeom g) {
    __shared__ float w[2 * kSepMaxR + 1];
    __shared__ float row[kSepRowsX][kSepRow + 2 * kSepMaxR];
    const int r = g.r;
    const long x0 = (long)blockIdx.x * kSepRow;
    const long nrows = g.ny * g.nz;
    const long row0 = (long)blockIdx.y * kSepRowsX;
    sep_weights(g, w);
    // all loads of the tile first (each thread: up to two per row), then the
    // LDS writes, so the loads are in flight together
    float v[kSepRowsX][2];
#pragma unroll
    for (int k = 0; k < kSepRowsX; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = threadIdx.x + j * kSepRow;
            const long rw = row0 + k, x = x0 - r + i;
            v[k][j] = (i < kSepRow + 2 * r && rw < nrows && x >= 0 && x < g.nx) ? src[rw * g.nx + x] : 0.0f;
        }
#pragma unroll
    for (int k = 0; k < kSepRowsX; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = threadIdx.x + j * kSepRow;
            if (i < kSepRow + 2 * r) row[k][i] = v[k][j];
        }
    __syncthreads();
    const long x = x0 + threadIdx.x;
    if (x >= g.nx) return;
    const int lo = (int)max(-(long)r, -x), hi = (int)min((long)r, g.nx - 1 - x);
    float ws = 0.0f;
    for (int k = lo; k <= hi; ++k) ws += w[k + r];
    for (int j = 0; j < kSepRowsX; ++j) {
        const long rw = row0 + j;
        if (rw >= nrows) break;
        float acc = 0.0f;
        for (int k = lo; k <= hi; ++k) acc = __builtin_fmaf(w[k + r], row[j][threadIdx.x + r + k], acc);
        dst[rw * g.nx + x] = acc / ws;
    }
}

// y (AXIS 1) or z (AXIS 2) pass: kSepCols columns in x (512-byte row pieces),
// kSepSeg outputs along the axis per workgroup of kSepCols x 2 threads; the
// tile with its halo sits in dynamic LDS.
constexpr int kSepCols = 128;
template <int AXIS>
__global__ void __launch_bounds__(256)
k_sep_yz(const float* __restrict__ src, float* __restrict__ dst, SepGeom g) {
    __shared__ float w[2 * kSepMaxR + 1];
    extern __shared__ float tile[];   // [kSepSeg + 2r][kSepCols]
    const int r = g.r;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const long x = (long)blockIdx.x * kSepCols + tx;
    const long a0 = (long)blockIdx.y * kSepSeg;          // first output along the axis
    const long other = blockIdx.z;                        // z for the y pass, y for the z pass
    const long na = AXIS == 1 ? g.ny : g.nz;
    const long sa = AXIS == 1 ? g.nx : g.nx * g.ny;       // stride along the axis
    const long base = x + (AXIS == 1 ? other * g.nx * g.ny : other * g.nx);
    sep_weights(g, w);
    // loads in groups of 8 rows, each group's loads in flight together
    const int nrow = kSepSeg + 2 * r;
    for (int i0 = ty; i0 < nrow; i0 += 16) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 2 * u;
            const long a = a0 - r + i;
            v[u] = (i < nrow && x < g.nx && a >= 0 && a < na) ? src[base + a * sa] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 2 * u;
            if (i < nrow) tile[i * kSepCols + tx] = v[u];
        }
    }
    __syncthreads();
    if (x >= g.nx) return;
    for (int j = ty; j < kSepSeg; j += 2) {
        const long a = a0 + j;
        if (a >= na) break;
        const int lo = (int)max(-(long)r, -a), hi = (int)min((long)r, na - 1 - a);
        float acc = 0.0f, ws = 0.0f;
        for (int k = lo; k <= hi; ++k) {
            acc = __builtin_fmaf(w[k + r], tile[(j + r + k) * kSepCols + tx], acc);
            ws += w[k + r];
        }
        dst[base + a * sa] = acc / ws;
    }
}

// x pass for a half-width R known at compile time (1..8): the same tile of
// kSepRowsX rows (row stride padded to 16 bytes), but thread t computes the 8
// consecutive outputs 8 (t % 32) .. + 7 of row t / 32 from 8 + 2R values read
// once from LDS, with the weights in registers and reciprocal weight sums.
template <int R>
__global__ void __launch_bounds__(kSepRow)
k_sep_x_t(const float* __restrict__ src, float* __restrict__ dst, SepGeom g) {
    __shared__ float w[2 * kSepMaxR + 1];
    constexpr int S = (kSepRow + 2 * R + 3) / 4 * 4;
    __shared__ __attribute__((aligned(16))) float row[kSepRowsX][S];
    const long x0 = (long)blockIdx.x * kSepRow;
    const long nrows = g.ny * g.nz;
    const long row0 = (long)blockIdx.y * kSepRowsX;
    sep_weights(g, w);
    float v[kSepRowsX][2];
#pragma unroll
    for (int k = 0; k < kSepRowsX; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = threadIdx.x + j * kSepRow;
            const long rw = row0 + k, x = x0 - R + i;
            v[k][j] = (i < kSepRow + 2 * R && rw < nrows && x >= 0 && x < g.nx) ? src[rw * g.nx + x] : 0.0f;
        }
#pragma unroll
    for (int k = 0; k < kSepRowsX; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = threadIdx.x + j * kSepRow;
            if (i < kSepRow + 2 * R) row[k][i] = v[k][j];
        }
    __syncthreads();
    const int k = threadIdx.x / 32, i0 = 8 * (threadIdx.x % 32);
    const long rw = row0 + k, xs = x0 + i0;
    if (rw >= nrows || xs >= g.nx) return;
    float wr[2 * R + 1];
    float wsum = 0.0f;
#pragma unroll
    for (int q = 0; q <= 2 * R; ++q) {
        wr[q] = w[q];
        wsum += wr[q];
    }
    const float inv = 1.0f / wsum;
    constexpr int NV = (8 + 2 * R + 3) / 4;   // float4 reads covering the window
    float t[4 * NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const float4 f = *reinterpret_cast<const float4*>(&row[k][i0 + 4 * q]);
        t[4 * q] = f.x; t[4 * q + 1] = f.y; t[4 * q + 2] = f.z; t[4 * q + 3] = f.w;
    }
    float o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const long x = xs + j;
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q <= 2 * R; ++q) acc = __builtin_fmaf(wr[q], t[j + q], acc);
        float scale = inv;
        if (x < R || x + R >= g.nx) {   // taps outside the cube carry no weight
            float ws = 0.0f;
#pragma unroll
            for (int q = 0; q <= 2 * R; ++q)
                if (x + q - R >= 0 && x + q - R < g.nx) ws += wr[q];
            scale = 1.0f / ws;
        }
        o[j] = acc * scale;
    }
    float* d = dst + rw * g.nx + xs;
    if (xs + 8 <= g.nx && ((uintptr_t)d % 16) == 0) {
        reinterpret_cast<float4*>(d)[0] = make_float4(o[0], o[1], o[2], o[3]);
        reinterpret_cast<float4*>(d)[1] = make_float4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (xs + j < g.nx) d[j] = o[j];
    }
}

// y or z pass for a half-width R known at compile time (1..8): the same
// tile, but each thread computes 32 consecutive outputs along the axis from
// 32 + 2R tile values read once into registers, with the weights in
// registers; interior outputs use the reciprocal of the full weight sum, the
// outputs within R of a face the sum of their in-cube taps.
constexpr int kSepTMaxR = 8;
template <int AXIS, int R>
__global__ void __launch_bounds__(256)
k_sep_yz_t(const float* __restrict__ src, float* __restrict__ dst, SepGeom g) {
    __shared__ float w[2 * kSepMaxR + 1];
    extern __shared__ float tile[];   // [kSepSeg + 2R][kSepCols]
    const int tx = threadIdx.x, ty = threadIdx.y;
    const long x = (long)blockIdx.x * kSepCols + tx;
    const long a0 = (long)blockIdx.y * kSepSeg;
    const long other = blockIdx.z;
    const long na = AXIS == 1 ? g.ny : g.nz;
    const long sa = AXIS == 1 ? g.nx : g.nx * g.ny;
    const long base = x + (AXIS == 1 ? other * g.nx * g.ny : other * g.nx);
    sep_weights(g, w);
    constexpr int nrow = kSepSeg + 2 * R;
    for (int i0 = ty; i0 < nrow; i0 += 16) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 2 * u;
            const long a = a0 - R + i;
            v[u] = (i < nrow && x < g.nx && a >= 0 && a < na) ? src[base + a * sa] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 2 * u;
            if (i < nrow) tile[i * kSepCols + tx] = v[u];
        }
    }
    __syncthreads();
    if (x >= g.nx) return;
    float wr[2 * R + 1];
    float wsum = 0.0f;
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) {
        wr[k] = w[k];
        wsum += wr[k];
    }
    const float inv = 1.0f / wsum;
    constexpr int NO = kSepSeg / 2;   // outputs of this thread: rows [NO ty, NO ty + NO)
    float t[NO + 2 * R];
#pragma unroll
    for (int i = 0; i < NO + 2 * R; ++i) t[i] = tile[(NO * ty + i) * kSepCols + tx];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        const long a = a0 + NO * ty + j;
        if (a >= na) break;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k <= 2 * R; ++k) acc = __builtin_fmaf(wr[k], t[j + k], acc);
        float scale = inv;
        if (a < R || a + R >= na) {   // taps outside the cube carry no weight
            float ws = 0.0f;
#pragma unroll
            for (int k = 0; k <= 2 * R; ++k)
                if (a + k - R >= 0 && a + k - R < na) ws += wr[k];
            scale = 1.0f / ws;
        }
        dst[base + a * sa] = acc * scale;
    }
}

// y (AXIS 1) or z (AXIS 2) pass: the register-window kernel for half-widths
// 1..8, the general one otherwise.
template <int AXIS>
static hipError_t launch_yz(dim3 grid, hipStream_t st, const float* src, float* dst, const SepGeom& g) {
    const size_t lds = (size_t)(kSepSeg + 2 * g.r) * kSepCols * sizeof(float);
    const dim3 block(kSepCols, 2);
#define IG_YZ_CASE(RR)                                                                                  \
    case RR:                                                                                            \
        hipLaunchKernelGGL((k_sep_yz_t<AXIS, RR>), grid, block, lds, st, src, dst, g);                  \
        return hipGetLastError();
    switch (g.r) {
        IG_YZ_CASE(1) IG_YZ_CASE(2) IG_YZ_CASE(3) IG_YZ_CASE(4)
        IG_YZ_CASE(5) IG_YZ_CASE(6) IG_YZ_CASE(7) IG_YZ_CASE(8)
        default: break;
    }
#undef IG_YZ_CASE
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_sep_yz<AXIS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sep_yz<AXIS>, grid, block, lds, st, src, dst, g);
    return hipGetLastError();
}

// Fused separable pass for half-widths up to 8: x, y and z in one sweep.
// A workgroup of 64 x 8 threads owns an output tile of 64 (x) x 32 (y) voxels
// and a chunk of g.tz planes along z, and streams its input planes (the chunk
// plus R on each side) through LDS: each plane's tile plus its x and y halos
// is loaded (zeros outside the cube), smoothed along x into a second LDS tile
// (all 32 + 2R rows), then along y in registers; thread (tx, ty) keeps rows
// 4 ty .. 4 ty + 3 of column tx and the last 2R + 1 of its y-smoothed planes,
// from which it forms the z sums.  HBM sees each voxel read once (plus the
// halos) and written once, against three reads and three writes for three
// passes.  R is the largest of the three half-widths; an axis with a smaller
// one gets zero weights at its outer taps, which leaves every sum and every
// renormalisation what the three-pass kernels compute, term by term.  Loads
// and stores go through raw buffers: a lane whose voxel lies outside the cube
// gets an offset past the buffer's end, and a plane outside the cube or the
// chunk a buffer of size 0, so no branch surrounds a memory access.
constexpr int kF3X = 64;              // tile width (one lane per column)
constexpr int kF3Y = 32;              // tile height (four rows per thread)
constexpr int kF3Threads = 512;
constexpr int kF3MaxR = 8;
constexpr int kSmBufWord3 = 0x00020000;   // gfx9 raw buffer: 32-bit format, no swizzle or stride
constexpr int kSmOffNone = 0x40000000;    // past the end of every buffer made here

struct Sep3Geom {
    long nx, ny, nz;
    int r[3];          // per-axis half-widths (<= R)
    int kind;
    int tz;            // output planes per workgroup
    double sigma[3];
};

// renormalisation factor of the output at coordinate c along an axis of n voxels
template <int R>
__device__ __forceinline__ float axis_scale(const float (&w)[2 * R + 1], float inv, long c, long n) {
    if (c >= R && c + R < n) return inv;
    float ws = 0.0f;
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k)
        if (c + k - R >= 0 && c + k - R < n) ws += w[k];
    return ws > 0.0f ? 1.0f / ws : 0.0f;   // 0: a column outside the cube (never stored)
}

template <int R>
__global__ void __launch_bounds__(kF3Threads)
k_sep3_t(const float* __restrict__ src, float* __restrict__ dst, Sep3Geom g) {
    constexpr int W = 2 * R + 1;
    constexpr int NR = kF3Y + 2 * R;                      // tile rows with the y halo
    constexpr int RX = kF3X + 2 * R;                      // tile row length with the x halo
    constexpr int NV = (4 + 2 * R + 3) / 4;               // 16-byte LDS reads per 4 x outputs
    constexpr int RS = 60 + 4 * NV;                       // row stride: the last window ends at it
    static_assert(RS >= RX && RS % 4 == 0, "row stride");
    constexpr int NE = NR * RX;                           // tile elements per plane
    constexpr int NL = (NE + kF3Threads - 1) / kF3Threads;
    constexpr int NXI = (NR * (kF3X / 4) + kF3Threads - 1) / kF3Threads;
    __shared__ float wt[3][W];
    __shared__ __attribute__((aligned(16))) float raw[NR * RS + 4];   // + a slot for lanes with no element
    __shared__ float xs[NR * kF3X];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const long nx = g.nx, ny = g.ny, nz = g.nz;
    // blockIdx.x runs fastest, and workgroups are dealt to the 8 XCDs in turn:
    // with 8 tiles across (512 voxels) a column of tiles shares an XCD and its
    // L2, so y-halo rows are mostly rows a neighbour tile read recently.
    // (Handing each XCD a contiguous run of tiles instead measured slower.)
    const long x0 = (long)blockIdx.x * kF3X, y0 = (long)blockIdx.y * kF3Y;
    for (int k = tid; k < 3 * W; k += kF3Threads) {
        const int a = k / W, d = k % W - R;
        float w = 0.0f;
        if (d >= -g.r[a] && d <= g.r[a])
            w = g.kind == IG_SMOOTH_BOX ? 1.0f : (float)exp(-(double)d * d / (2.0 * g.sigma[a] * g.sigma[a]));
        wt[a][k % W] = w;
    }
    // this thread's tile elements: byte offset from the first input row (or
    // kSmOffNone outside the cube) and LDS slot (the spare slot past the tile)
    const long yb = max(y0 - R, 0L);
    const int in_bytes = (int)((min(y0 + kF3Y + R, ny) - yb) * nx * 4);
    int loff[NL], lidx[NL];
#pragma unroll
    for (int m = 0; m < NL; ++m) {
        const int e = tid + m * kF3Threads;
        const int row = e / RX, col = e - row * RX;
        const long y = y0 - R + row, x = x0 - R + col;
        const bool ok = e < NE && y >= 0 && y < ny && x >= 0 && x < nx;
        loff[m] = ok ? (int)(((y - yb) * nx + x) * 4) : kSmOffNone;
        lidx[m] = e < NE ? row * RS + col : NR * RS;
    }
    // this thread's outputs: rows 4 ty + j of column x0 + tx
    const int rows_out = (int)min((long)kF3Y, ny - y0);
    const int out_bytes = (int)(rows_out * nx * 4);
    int soff[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        soff[j] = (4 * ty + j < rows_out && x0 + tx < nx) ? (int)(((4 * ty + j) * nx + x0 + tx) * 4) : kSmOffNone;
    __syncthreads();
    float wx[W], wy[W], wz[W];
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        wx[k] = wt[0][k];
        wy[k] = wt[1][k];
        wz[k] = wt[2][k];
        sx += wx[k];
        sy += wy[k];
        sz += wz[k];
    }
    const float ix = 1.0f / sx, iy = 1.0f / sy, iz = 1.0f / sz;
    float ys[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) ys[j] = axis_scale<R>(wy, iy, y0 + 4 * ty + j, ny);

    const long plane = nx * ny;
    const long z0 = (long)blockIdx.z * g.tz, z1 = min(z0 + g.tz, nz);
    const long zb = z0 - R, ze = z1 + R;
    // input planes are loaded two steps ahead, into two register sets used in
    // turn (the loop runs an even number of steps: a step past the last input
    // plane loads nothing and stores nothing)
    float pa[NL], pb[NL];
    auto load = [&](long zi, float (&pf)[NL]) {
        const bool on = zi >= 0 && zi < nz && zi < ze;
        const auto rs = __builtin_amdgcn_make_buffer_rsrc((void*)(src + (on ? zi : 0) * plane + yb * nx), 0,
                                                          on ? in_bytes : 0, kSmBufWord3);
#pragma unroll
        for (int m = 0; m < NL; ++m)
            pf[m] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, loff[m], 0, 0));
    };
    float ring[4][W];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < W; ++k) ring[j][k] = 0.0f;
    // the outputs of plane zi - R are stored one step later, after the loads
    // of that step are issued, so waiting for a plane's loads never waits for
    // stores issued after them
    float ob[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    long zs = zb - R - 1;   // plane held in ob (none yet)
    auto store = [&]() {
        const bool zon = zs >= z0 && zs < z1;
        const auto rd = __builtin_amdgcn_make_buffer_rsrc((void*)(dst + (zon ? zs : 0) * plane + y0 * nx), 0,
                                                          zon ? out_bytes : 0, kSmBufWord3);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, ob[j]), rd, soff[j], 0, 0);
    };
    auto step = [&](long zi, float (&pf)[NL]) {
#pragma unroll
        for (int m = 0; m < NL; ++m) raw[lidx[m]] = pf[m];
        load(zi + 2, pf);
        store();
        __syncthreads();
        // x: outputs 4c .. 4c + 3 of tile row `row`, from 4 + 2R values
#pragma unroll
        for (int m = 0; m < NXI; ++m) {
            const int it = tid + m * kF3Threads;
            const int row = it >> 4, c = it & 15;
            if (row < NR) {
                float t[4 * NV];
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    const float4 f = *reinterpret_cast<const float4*>(&raw[row * RS + 4 * c + 4 * q]);
                    t[4 * q] = f.x; t[4 * q + 1] = f.y; t[4 * q + 2] = f.z; t[4 * q + 3] = f.w;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float acc = 0.0f;
#pragma unroll
                    for (int k = 0; k < W; ++k) acc = __builtin_fmaf(wx[k], t[j + k], acc);
                    xs[row * kF3X + 4 * c + j] = acc * axis_scale<R>(wx, ix, x0 + 4 * c + j, nx);
                }
            }
        }
        __syncthreads();
        // y: rows 4 ty .. 4 ty + 3 of column tx, from 4 + 2R values
        float t[4 + 2 * R];
#pragma unroll
        for (int i = 0; i < 4 + 2 * R; ++i) t[i] = xs[(4 * ty + i) * kF3X + tx];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < W; ++k) acc = __builtin_fmaf(wy[k], t[j + k], acc);
#pragma unroll
            for (int k = 0; k + 1 < W; ++k) ring[j][k] = ring[j][k + 1];
            ring[j][W - 1] = acc * ys[j];
        }
        // z: output plane zi - R from the ring (planes zi - 2R .. zi)
        zs = zi - R;
        const float zsc = axis_scale<R>(wz, iz, zs, nz);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < W; ++k) acc = __builtin_fmaf(wz[k], ring[j][k], acc);
            ob[j] = acc * zsc;
        }
    };
    // the stores here write nothing (no plane held yet); they give the loop's
    // entry the same order of outstanding loads and stores as its back edge
    load(zb, pa);
    store();
    load(zb + 1, pb);
    store();
    for (long zi = zb; zi < ze; zi += 2) {
        step(zi, pa);
        step(zi + 1, pb);
    }
    store();
}

struct DenseGeom {
    long nx, ny, nz;
    int rx, ry, rz;
    int pad;
    double sigma[3];
    double theta[3];   // radians
};

// Dense rotated Gaussian; TZ outputs along z per thread.
template <int TZ>
__global__ void __launch_bounds__(256)
k_dense(const float* __restrict__ src, float* __restrict__ dst, DenseGeom g) {
    extern __shared__ float sm[];
    const int rx = g.rx, ry = g.ry, rz = g.rz;
    const int kx = 2 * rx + 1, ky = 2 * ry + 1, kz = 2 * rz + 1;
    const int nw = kx * ky * kz;
    const int TXh = 64 + 2 * rx, TYh = 4 + 2 * ry, TZh = TZ + 2 * rz;
    float* W = sm;
    float* T = sm + nw;
    __shared__ float total_sh;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
    const long x0 = (long)blockIdx.x * 64, y0 = (long)blockIdx.y * 4, z0 = (long)blockIdx.z * TZ;

    // weights: the Gaussian in the frame rotated by R = Rz Ry Rx, at u = R^T d
    {
        const double cx = cos(g.theta[0]), sx = sin(g.theta[0]);
        const double cy = cos(g.theta[1]), sy = sin(g.theta[1]);
        const double cz = cos(g.theta[2]), sz = sin(g.theta[2]);
        // R = Rz * Ry * Rx
        const double R00 = cz * cy, R01 = cz * sy * sx - sz * cx, R02 = cz * sy * cx + sz * sx;
        const double R10 = sz * cy, R11 = sz * sy * sx + cz * cx, R12 = sz * sy * cx - cz * sx;
        const double R20 = -sy, R21 = cy * sx, R22 = cy * cx;
        for (int t = tid; t < nw; t += 256) {
            const int ix = t % kx, iy = (t / kx) % ky, iz = t / (kx * ky);
            const double dx = ix - rx, dy = iy - ry, dz = iz - rz;
            const double u0 = R00 * dx + R10 * dy + R20 * dz;   // (R^T d)_0
            const double u1 = R01 * dx + R11 * dy + R21 * dz;
            const double u2 = R02 * dx + R12 * dy + R22 * dz;
            const double e = u0 * u0 / (2.0 * g.sigma[0] * g.sigma[0]) + u1 * u1 / (2.0 * g.sigma[1] * g.sigma[1]) +
                             u2 * u2 / (2.0 * g.sigma[2] * g.sigma[2]);
            W[t] = (float)exp(-e);
        }
    }
    // input tile with halo (zeros outside the cube)
    const int ntile = TXh * TYh * TZh;
    for (int i = tid; i < ntile; i += 256) {
        const int ix = i % TXh, iy = (i / TXh) % TYh, iz = i / (TXh * TYh);
        const long x = x0 - rx + ix, y = y0 - ry + iy, z = z0 - rz + iz;
        T[i] = (x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz)
                   ? src[x + g.nx * (y + g.ny * z)]
                   : 0.0f;
    }
    __syncthreads();
    if (tid < 64) {   // total weight, fixed order (strided partials, then a tree)
        float s = 0.0f;
        for (int t = tid; t < nw; t += 64) s += W[t];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (tid == 0) total_sh = s;
    }
    const bool edge = x0 - rx < 0 || x0 + 63 + rx >= g.nx || y0 - ry < 0 || y0 + 3 + ry >= g.ny || z0 - rz < 0 ||
                      z0 + TZ - 1 + rz >= g.nz;
    float acc[TZ], ws[TZ];
#pragma unroll
    for (int j = 0; j < TZ; ++j) {
        acc[j] = 0.0f;
        ws[j] = 0.0f;
    }
    for (int dz = -rz; dz <= rz; ++dz) {
        for (int dy = -ry; dy <= ry; ++dy) {
            const float* wrow = W + ((dz + rz) * ky + (dy + ry)) * kx + rx;
            const float* col = T + (long)(ty + ry + dy) * TXh + tx + rx;
            const long yy = y0 + ty + dy;
            for (int dx = -rx; dx <= rx; ++dx) {
                const float wv = wrow[dx];
#pragma unroll
                for (int j = 0; j < TZ; ++j)
                    acc[j] = __builtin_fmaf(wv, col[(j + dz + rz) * TXh * TYh + dx], acc[j]);
                if (edge) {
                    const long xx = x0 + tx + dx;
                    const bool in_xy = xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny;
#pragma unroll
                    for (int j = 0; j < TZ; ++j) {
                        const long zz = z0 + j + dz;
                        ws[j] += (in_xy && zz >= 0 && zz < g.nz) ? wv : 0.0f;
                    }
                }
            }
        }
    }
    __syncthreads();
    const float total = total_sh;
    const long x = x0 + tx, y = y0 + ty;
    if (x >= g.nx || y >= g.ny) return;
#pragma unroll
    for (int j = 0; j < TZ; ++j) {
        const long z = z0 + j;
        if (z < g.nz) dst[x + g.nx * (y + g.ny * z)] = acc[j] / (edge ? ws[j] : total);
    }
}

// Dense pass with 8 outputs along z per thread and the z half-width RZ known
// at compile time (1..8): the loops run over (dy, dx) outside and dz inside,
// so each input column of 8 + 2 RZ values is read from LDS once into
// registers and serves all (2 RZ + 1) x 8 products of that column (about a
// third of the LDS reads of the general loop order).
template <int RZ>
__global__ void __launch_bounds__(256)
k_dense_t(const float* __restrict__ src, float* __restrict__ dst, DenseGeom g) {
    constexpr int TZ = 8, KZ = 2 * RZ + 1, NC = TZ + 2 * RZ;
    extern __shared__ float sm[];
    const int rx = g.rx, ry = g.ry;
    const int kx = 2 * rx + 1, ky = 2 * ry + 1;
    const int nw = kx * ky * KZ;
    const int TXh = 64 + 2 * rx, TYh = 4 + 2 * ry;
    const int plane = TXh * TYh;
    float* W = sm;
    float* T = sm + nw;
    __shared__ float total_sh;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
    const long x0 = (long)blockIdx.x * 64, y0 = (long)blockIdx.y * 4, z0 = (long)blockIdx.z * TZ;
    {
        const double cx = cos(g.theta[0]), sx = sin(g.theta[0]);
        const double cy = cos(g.theta[1]), sy = sin(g.theta[1]);
        const double cz = cos(g.theta[2]), sz = sin(g.theta[2]);
        const double R00 = cz * cy, R01 = cz * sy * sx - sz * cx, R02 = cz * sy * cx + sz * sx;
        const double R10 = sz * cy, R11 = sz * sy * sx + cz * cx, R12 = sz * sy * cx - cz * sx;
        const double R20 = -sy, R21 = cy * sx, R22 = cy * cx;
        for (int t = tid; t < nw; t += 256) {
            const int ix = t % kx, iy = (t / kx) % ky, iz = t / (kx * ky);
            const double dx = ix - rx, dy = iy - ry, dz = iz - RZ;
            const double u0 = R00 * dx + R10 * dy + R20 * dz;
            const double u1 = R01 * dx + R11 * dy + R21 * dz;
            const double u2 = R02 * dx + R12 * dy + R22 * dz;
            const double e = u0 * u0 / (2.0 * g.sigma[0] * g.sigma[0]) + u1 * u1 / (2.0 * g.sigma[1] * g.sigma[1]) +
                             u2 * u2 / (2.0 * g.sigma[2] * g.sigma[2]);
            W[t] = (float)exp(-e);
        }
    }
    const int ntile = plane * NC;
    for (int i0 = tid; i0 < ntile; i0 += 256 * 8) {   // loads in groups of 8
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + 256 * u;
            const int ix = i % TXh, iy = (i / TXh) % TYh, iz = i / plane;
            const long x = x0 - rx + ix, y = y0 - ry + iy, z = z0 - RZ + iz;
            v[u] = (i < ntile && x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz)
                       ? src[x + g.nx * (y + g.ny * z)]
                       : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + 256 * u < ntile) T[i0 + 256 * u] = v[u];
    }
    __syncthreads();
    if (tid < 64) {
        float s = 0.0f;
        for (int t = tid; t < nw; t += 64) s += W[t];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (tid == 0) total_sh = s;
    }
    const bool edge = x0 - rx < 0 || x0 + 63 + rx >= g.nx || y0 - ry < 0 || y0 + 3 + ry >= g.ny || z0 - RZ < 0 ||
                      z0 + TZ - 1 + RZ >= g.nz;
    float acc[TZ], ws[TZ];
#pragma unroll
    for (int j = 0; j < TZ; ++j) {
        acc[j] = 0.0f;
        ws[j] = 0.0f;
    }
    for (int dy = -ry; dy <= ry; ++dy) {
        const long yy = y0 + ty + dy;
        for (int dx = -rx; dx <= rx; ++dx) {
            const float* col = T + (ty + ry + dy) * TXh + tx + rx + dx;
            float c[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) c[i] = col[i * plane];
            const float* wz = W + (dy + ry) * kx + (dx + rx);   // + (dz + RZ) kx ky
#pragma unroll
            for (int k = 0; k < KZ; ++k) {
                const float wv = wz[k * kx * ky];
#pragma unroll
                for (int j = 0; j < TZ; ++j) acc[j] = __builtin_fmaf(wv, c[j + k], acc[j]);
            }
            if (edge) {
                const long xx = x0 + tx + dx;
                const bool in_xy = xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny;
#pragma unroll
                for (int k = 0; k < KZ; ++k) {
                    const float wv = wz[k * kx * ky];
#pragma unroll
                    for (int j = 0; j < TZ; ++j) {
                        const long zz = z0 + j + k - RZ;
                        ws[j] += (in_xy && zz >= 0 && zz < g.nz) ? wv : 0.0f;
                    }
                }
            }
        }
    }
    __syncthreads();
    const float total = total_sh;
    const long x = x0 + tx, y = y0 + ty;
    if (x >= g.nx || y >= g.ny) return;
#pragma unroll
    for (int j = 0; j < TZ; ++j) {
        const long z = z0 + j;
        if (z < g.nz) dst[x + g.nx * (y + g.ny * z)] = acc[j] / (edge ? ws[j] : total);
    }
}

}  // namespace igk

// ====================================================================== host
using namespace igk;
#define fail igk_fail

namespace {

constexpr double kFwhmToSigma = 0.42466090014400953;   // 1 / (2 sqrt(2 ln 2))

int g_smooth_path = 0;   // 0: the fused pass where it applies, 1: always three passes

// the fused separable pass applies for half-widths up to kF3MaxR and rows
// short enough that a tile's rows stay below 2^30 bytes (32-bit buffer offsets)
bool fused_applies(int rmax, long nx) {
    return g_smooth_path == 0 && rmax <= kF3MaxR && (long)(kF3Y + 2 * kF3MaxR) * nx * 4 <= (1L << 30);
}

// One round of workgroups: as many z chunks per (x, y) tile as fill every
// compute unit to the kernel's occupancy once (each chunk at least 8
// planes), so no compute unit runs a second, partial round alone.
template <int R>
hipError_t launch_sep3(hipStream_t st, const float* in, float* out, Sep3Geom g) {
    int dev = 0, ncu = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sep3_t<R>, kF3Threads, 0);
    if (e != hipSuccess) return e;
    const long gx = (g.nx + kF3X - 1) / kF3X, gy = (g.ny + kF3Y - 1) / kF3Y;
    const long slots = (long)std::max(ncu, 1) * std::max(occ, 1);
    const long chunks = std::max(1L, std::min(slots / (gx * gy), (g.nz + 7) / 8));
    const long tz = (g.nz + chunks - 1) / chunks;
    g.tz = (int)tz;
    const dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)((g.nz + tz - 1) / tz));
    hipLaunchKernelGGL(k_sep3_t<R>, grid, dim3(kF3Threads), 0, st, in, out, g);
    return hipGetLastError();
}

hipError_t run_sep3(int rmax, const float* in, float* out, const Sep3Geom& g, hipStream_t st) {
    switch (rmax) {
        case 0: return launch_sep3<0>(st, in, out, g);
        case 1: return launch_sep3<1>(st, in, out, g);
        case 2: return launch_sep3<2>(st, in, out, g);
        case 3: return launch_sep3<3>(st, in, out, g);
        case 4: return launch_sep3<4>(st, in, out, g);
        case 5: return launch_sep3<5>(st, in, out, g);
        case 6: return launch_sep3<6>(st, in, out, g);
        case 7: return launch_sep3<7>(st, in, out, g);
        case 8: return launch_sep3<8>(st, in, out, g);
        default: return hipErrorInvalidValue;
    }
}

struct SmoothPlan {
    int r[3];
    bool separable;
    double sigma[3];
    double theta[3];   // radians
};

ig_status plan(const ig_smooth_params* s, SmoothPlan* p) {
    if (!s) return fail(IG_ERR_INVALID_ARG, "params is NULL");
    if (s->struct_size != (int32_t)sizeof(ig_smooth_params)) return fail(IG_ERR_INVALID_ARG, "struct_size");
    if (s->reserved != 0) return fail(IG_ERR_INVALID_ARG, "reserved must be 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(s->size[a]) || !std::isfinite(s->theta[a]))
            return fail(IG_ERR_INVALID_ARG, "non-finite size or angle");
    if (!std::isfinite(s->truncate) || s->truncate < 0.0f) return fail(IG_ERR_INVALID_ARG, "bad truncate");
    if (s->kind == IG_SMOOTH_BOX) {
        for (int a = 0; a < 3; ++a) {
            const float n = s->size[a];
            if (n < 1.0f || n != std::floor(n) || ((long)n) % 2 == 0)
                return fail(IG_ERR_INVALID_ARG, "box size %g must be an odd integer >= 1", (double)n);
            if (s->theta[a] != 0.0f) return fail(IG_ERR_INVALID_ARG, "box angles must be 0");
            p->r[a] = (int)((long)n / 2);
            p->sigma[a] = 0.0;
            p->theta[a] = 0.0;
        }
        p->separable = true;
        return IG_OK;
    }
    if (s->kind != IG_SMOOTH_GAUSS) return fail(IG_ERR_INVALID_ARG, "bad kind %d", s->kind);
    const double tr = s->truncate > 0.0f ? (double)s->truncate : 3.0;
    bool rot = false;
    for (int a = 0; a < 3; ++a) {
        if (!(s->size[a] > 0.0f)) return fail(IG_ERR_INVALID_ARG, "FWHM must be > 0");
        p->sigma[a] = (double)s->size[a] * kFwhmToSigma;
        p->theta[a] = (double)s->theta[a] * (M_PI / 180.0);
        rot = rot || s->theta[a] != 0.0f;
    }
    p->separable = !rot;
    if (!rot) {
        for (int a = 0; a < 3; ++a) p->r[a] = (int)std::floor(tr * p->sigma[a] + 0.5);
        return IG_OK;
    }
    const double cx = std::cos(p->theta[0]), sx = std::sin(p->theta[0]);
    const double cy = std::cos(p->theta[1]), sy = std::sin(p->theta[1]);
    const double cz = std::cos(p->theta[2]), sz = std::sin(p->theta[2]);
    const double R[3][3] = {{cz * cy, cz * sy * sx - sz * cx, cz * sy * cx + sz * sx},
                            {sz * cy, sz * sy * sx + cz * cx, sz * sy * cx - cz * sx},
                            {-sy, cy * sx, cy * cx}};
    for (int i = 0; i < 3; ++i) {
        double e = 0.0;
        for (int j = 0; j < 3; ++j) e += R[i][j] * R[i][j] * p->sigma[j] * p->sigma[j];
        p->r[i] = (int)std::floor(tr * std::sqrt(e) + 0.5);
    }
    return IG_OK;
}

size_t dense_lds(const SmoothPlan& p, int tz) {
    const size_t nw = (size_t)(2 * p.r[0] + 1) * (2 * p.r[1] + 1) * (2 * p.r[2] + 1);
    const size_t tile = (size_t)(64 + 2 * p.r[0]) * (4 + 2 * p.r[1]) * (tz + 2 * p.r[2]);
    return (nw + tile) * sizeof(float);
}

bool overlaps(const void* a, const void* b, size_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return a && b && x < y + bytes && y < x + bytes;
}

template <int RZ>
void (*dense_t_kernel())(const float*, float*, DenseGeom) { return k_dense_t<RZ>; }

template <int TZ>
hipError_t launch_dense(const float* in, float* out, const DenseGeom& g, size_t lds, hipStream_t st) {
    auto k = k_dense<TZ>;
    if constexpr (TZ == 8) {   // the register-column kernel for z half-widths 1..8
        switch (g.rz) {
            case 1: k = dense_t_kernel<1>(); break;
            case 2: k = dense_t_kernel<2>(); break;
            case 3: k = dense_t_kernel<3>(); break;
            case 4: k = dense_t_kernel<4>(); break;
            case 5: k = dense_t_kernel<5>(); break;
            case 6: k = dense_t_kernel<6>(); break;
            case 7: k = dense_t_kernel<7>(); break;
            case 8: k = dense_t_kernel<8>(); break;
            default: break;
        }
    }
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)((g.nz + TZ - 1) / TZ));
    hipLaunchKernelGGL(k, grid, dim3(64, 4), lds, st, in, out, g);
    return hipGetLastError();
}

}  // namespace

extern "C" ig_status ig_smooth_geometry(const ig_smooth_params* s, int32_t* radius, int32_t* separable) {
    SmoothPlan p{};
    ig_status st = plan(s, &p);
    if (st != IG_OK) return st;
    if (radius)
        for (int a = 0; a < 3; ++a) radius[a] = p.r[a];
    if (separable) *separable = p.separable ? 1 : 0;
    return IG_OK;
}

extern "C" ig_status ig_smooth(const ig_smooth_params* s, const float* d_in, float* d_out, float* d_work, int64_t nx,
                               int64_t ny, int64_t nz, void* hip_stream) {
    SmoothPlan p{};
    ig_status st = plan(s, &p);
    if (st != IG_OK) return st;
    if (!d_in || !d_out) return fail(IG_ERR_INVALID_ARG, "NULL cube");
    if (nx < 1 || ny < 1 || nz < 1 || nx > (1LL << 30) || ny > 65535LL * 64 || nz > 65535LL * 64)
        return fail(IG_ERR_INVALID_ARG, "bad cube size");
    const size_t bytes = (size_t)(nx * ny * nz) * sizeof(float);
    if (overlaps(d_in, d_out, bytes)) return fail(IG_ERR_INVALID_ARG, "d_in and d_out overlap");
    {
        const int dev = igk_current_device();
        ig_status cb = igk_check_buffer(d_in, bytes, dev, "d_in");
        if (cb == IG_OK) cb = igk_check_buffer(d_out, bytes, dev, "d_out");
        if (cb == IG_OK && p.separable && d_work) cb = igk_check_buffer(d_work, bytes, dev, "d_work");
        if (cb != IG_OK) return cb;
    }
    hipStream_t st_ = (hipStream_t)hip_stream;
    if (p.separable) {
        if (!d_work) return fail(IG_ERR_INVALID_ARG, "the separable path needs d_work");
        if (overlaps(d_work, d_in, bytes) || overlaps(d_work, d_out, bytes))
            return fail(IG_ERR_INVALID_ARG, "d_work overlaps a cube");
        for (int a = 0; a < 3; ++a)
            if (p.r[a] > kSepMaxR) return fail(IG_ERR_UNSUPPORTED, "half-width %d above %d", p.r[a], kSepMaxR);
        if (ny > 65535 || nz > 65535) return fail(IG_ERR_UNSUPPORTED, "ny and nz must be <= 65535");
        const int rmax = std::max(p.r[0], std::max(p.r[1], p.r[2]));
        if (fused_applies(rmax, nx)) {
            const Sep3Geom g3{nx, ny, nz, {p.r[0], p.r[1], p.r[2]}, s->kind, 0, {p.sigma[0], p.sigma[1], p.sigma[2]}};
            const hipError_t e = run_sep3(rmax, d_in, d_out, g3, st_);
            if (e != hipSuccess) return fail(IG_ERR_DEVICE, "fused pass: %s", hipGetErrorString(e));
            return IG_OK;
        }
        SepGeom g{nx, ny, nz, 0, s->kind, 0.0};
        g.r = p.r[0];
        g.sigma = p.sigma[0];
        const long xrows = (ny * nz + kSepRowsX - 1) / kSepRowsX;
        if (xrows > 2147483647L) return fail(IG_ERR_UNSUPPORTED, "cube too large");
        const dim3 xgrid((unsigned)((nx + kSepRow - 1) / kSepRow), (unsigned)xrows);
        switch (g.r) {
#define IG_X_CASE(RR) \
            case RR: hipLaunchKernelGGL(k_sep_x_t<RR>, xgrid, dim3(kSepRow), 0, st_, d_in, d_out, g); break;
            IG_X_CASE(1) IG_X_CASE(2) IG_X_CASE(3) IG_X_CASE(4)
            IG_X_CASE(5) IG_X_CASE(6) IG_X_CASE(7) IG_X_CASE(8)
#undef IG_X_CASE
            default: hipLaunchKernelGGL(k_sep_x, xgrid, dim3(kSepRow), 0, st_, d_in, d_out, g); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(IG_ERR_DEVICE, "x pass: %s", hipGetErrorString(e));
        g.r = p.r[1];
        g.sigma = p.sigma[1];
        const unsigned gx = (unsigned)((nx + kSepCols - 1) / kSepCols);
        e = launch_yz<1>(dim3(gx, (unsigned)((ny + kSepSeg - 1) / kSepSeg), (unsigned)nz), st_, d_out, d_work, g);
        if (e != hipSuccess) return fail(IG_ERR_DEVICE, "y pass: %s", hipGetErrorString(e));
        g.r = p.r[2];
        g.sigma = p.sigma[2];
        e = launch_yz<2>(dim3(gx, (unsigned)((nz + kSepSeg - 1) / kSepSeg), (unsigned)ny), st_, d_work, d_out, g);
        if (e != hipSuccess) return fail(IG_ERR_DEVICE, "z pass: %s", hipGetErrorString(e));
        return IG_OK;
    }
    int tz = 0;
    for (int c : {8, 4, 2, 1})
        if (dense_lds(p, c) + 256 <= kMaxLds) {   // + the static total slot
            tz = c;
            break;
        }
    if (!tz) return fail(IG_ERR_UNSUPPORTED, "rotated kernel half-widths %d,%d,%d need more LDS than a CU has",
                         p.r[0], p.r[1], p.r[2]);
    if ((ny + 3) / 4 > 65535 || (nz + tz - 1) / tz > 65535) return fail(IG_ERR_UNSUPPORTED, "cube too tall");
    DenseGeom g{nx, ny, nz, p.r[0], p.r[1], p.r[2], 0, {p.sigma[0], p.sigma[1], p.sigma[2]},
                {p.theta[0], p.theta[1], p.theta[2]}};
    const size_t lds = dense_lds(p, tz);
    hipError_t e = tz == 8   ? launch_dense<8>(d_in, d_out, g, lds, st_)
                   : tz == 4 ? launch_dense<4>(d_in, d_out, g, lds, st_)
                   : tz == 2 ? launch_dense<2>(d_in, d_out, g, lds, st_)
                             : launch_dense<1>(d_in, d_out, g, lds, st_);
    if (e != hipSuccess) return fail(IG_ERR_DEVICE, "dense pass: %s", hipGetErrorString(e));
    return IG_OK;
}

extern "C" ig_status ig_smooth_set_path(int32_t path) {
    if (path != 0 && path != 1) return fail(IG_ERR_INVALID_ARG, "path must be 0 or 1");
    g_smooth_path = path;
    return IG_OK;
}
