// Box and Gaussian smoothing (Section 3.1-3.2); see include/igsmooth.h.
//
// Separable kernels (box, axis-aligned Gaussian): three 1-D passes x -> out,
// y -> work, z -> out.  Each pass stages a segment of its axis plus the halo
// in LDS (coalesced loads along x), computes its weights in FP64 at block
// start, and divides every output by the sum of the weights of its in-cube
// taps: the product of the three per-axis renormalisations is the 3-D one.
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
