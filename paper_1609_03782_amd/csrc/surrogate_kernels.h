// Kernels of the learned surrogate: a 3-D CNN of 3x3x3 convolutions that
// approximates n steps of the filter in one pass.
//
// Data layout.  Activations are bf16, channels-last: a[(z*ny + y)*nx + x][C].
// Convolutions are implicit GEMMs on the gfx950 matrix cores with
// v_mfma_f32_16x16x32_bf16 (D[16x16] += A[16x32] B[32x16], FP32 accumulate):
//   forward:  M = voxels (16 consecutive x), N = output channels,
//             K = 32 input channels of one tap (27 taps = 27 K-steps); for a
//             1-channel input K = the 27 taps themselves (padded to 32).
//   input gradient: the same kernel on the output gradient with the weights
//             mirrored in space and transposed in channels.
//   weight gradient: M = input channels (or taps), N = output channels,
//             K = voxels; per-workgroup partials, folded in a fixed order.
// Operand lane layout (wave64, checked on the device): A[i][k] sits in lane
// i + 16*(k/8), element k%8; B[k][n] in lane n + 16*(k/8), element k%8;
// D[m][n] in lane n + 16*(m/4), element m%4.
//
// Weights are kept packed in that B layout: Wp[t][nb][lane][8] holds
// B[k = 8*(lane/16) + e][n = 16*nb + lane%16] of tap t, so a lane's fragment
// is one 16-byte load.  For a 1-channel input the taps are the K index:
// Wp[nb][lane][8] with k = tap.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace igs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

enum { EPI_RAW = 0, EPI_GELU = 1, EPI_BACK_GELU = 2, EPI_RESID = 3 };

constexpr int TX = 32;   // output tile: 32 voxels in x (two 16-row MFMA tiles) ...
constexpr int TY = 4;    // ... by 4 rows in y (one per wavefront), one plane in z

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ u16 f2bf(float f) {   // round to nearest, ties to even (finite inputs)
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * (0.39894228040143268f * __expf(-0.5f * z * z));
}

// ---------------------------------------------------------------- conv
// Output channels padded to 16*NB.  aux: pre-activation (EPI_GELU, optional,
// bf16 [v][16*NB]), pre-activation of the layer below (EPI_BACK_GELU), or the
// FP32 input cube for the residual (EPI_RESID, output channel 0 only).
template <int CIN, int NB, int EPI>
__global__ void __launch_bounds__(256)
k_conv(const u16* __restrict__ in, const bf16x8* __restrict__ wp, const float* __restrict__ bias,
       void* __restrict__ out, const void* __restrict__ aux, int nx, int ny, int nz) {
    constexpr int COUTP = 16 * NB;
    constexpr int LX = TX + 2, LY = TY + 2;
    __shared__ __attribute__((aligned(16))) u16 tile[3 * LY * LX * CIN];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z;

    // stage the input region (with a one-voxel margin; zero outside the cube)
    if constexpr (CIN % 8 == 0) {
        constexpr int CH = CIN / 8;   // 16-byte chunks per voxel
        for (int q = threadIdx.x; q < 3 * LY * LX * CH; q += 256) {
            const int c = q % CH, vox = q / CH;
            const int xx = vox % LX, yy = (vox / LX) % LY, zz = vox / (LX * LY);
            const int x = x0 + xx - 1, y = y0 + yy - 1, z = z0 + zz - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
                v = *reinterpret_cast<const uint4*>(in + ((long)(z * ny + y) * nx + x) * CIN + 8 * c);
            *reinterpret_cast<uint4*>(tile + vox * CIN + 8 * c) = v;
        }
    } else {
        for (int vox = threadIdx.x; vox < 3 * LY * LX; vox += 256) {
            const int xx = vox % LX, yy = (vox / LX) % LY, zz = vox / (LX * LY);
            const int x = x0 + xx - 1, y = y0 + yy - 1, z = z0 + zz - 1;
            tile[vox] = (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
                            ? in[(long)(z * ny + y) * nx + x] : (u16)0;
        }
    }
    __syncthreads();

    f32x4 acc[2][NB];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[s][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int i = lane & 15, kg = lane >> 4;
    if constexpr (CIN == 1) {
        // K = taps: lane holds taps 8*kg .. 8*kg+7 of voxel row i
        bf16x8 b[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[nb] = wp[nb * 64 + lane];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int t = 8 * kg + e;
                u16 h = 0;
                if (t < 27) {
                    const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;   // 0..2 = offset + 1
                    h = tile[(dz * LY + (w + dy)) * LX + (16 * s + i + dx)];
                }
                a[e] = __builtin_bit_cast(__bf16, h);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[s][nb], 0, 0, 0);
        }
    } else {
        static_assert(CIN == 32, "CIN must be 1 or 32");
        for (int t = 0; t < 27; ++t) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            bf16x8 b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[nb] = wp[(t * NB + nb) * 64 + lane];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int vox = (dz * LY + (w + dy)) * LX + (16 * s + i + dx);
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(tile + vox * 32 + 8 * kg);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[s][nb], 0, 0, 0);
            }
        }
    }

    // epilogue: lane holds D[m = 4*kg + e][n = 16*nb + i] of subtile s
    const int y = y0 + w;
    if (y >= ny) return;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int x = x0 + 16 * s + 4 * kg + e;
            if (x >= nx) continue;
            const long v = (long)(z0 * ny + y) * nx + x;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int n = 16 * nb + i;
                const float d = acc[s][nb][e];
                if constexpr (EPI == EPI_RAW) {
                    static_cast<float*>(out)[v * COUTP + n] = d + (bias ? bias[n] : 0.0f);
                } else if constexpr (EPI == EPI_GELU) {
                    const float zpre = d + bias[n];
                    if (aux) const_cast<u16*>(static_cast<const u16*>(aux))[v * COUTP + n] = f2bf(zpre);
                    static_cast<u16*>(out)[v * COUTP + n] = f2bf(gelu(zpre));
                } else if constexpr (EPI == EPI_BACK_GELU) {
                    const float zb = bf2f(static_cast<const u16*>(aux)[v * COUTP + n]);
                    static_cast<u16*>(out)[v * COUTP + n] = f2bf(d * gelu_grad(zb));
                } else {   // EPI_RESID: output channel 0 only
                    if (n == 0) static_cast<float*>(out)[v] = static_cast<const float*>(aux)[v] + (d + bias[0]);
                }
            }
        }
}

// ---------------------------------------------------------- weight grad
// Partial dW of one workgroup: voxels of a 32 x 4 tile over ZC planes.
// CIN == 32: rows = input channels, each wavefront owns taps t = w, w+4, ...
// CIN == 1:  rows = taps (27, padded to 32), one set of accumulators.
// COUT = 32 (NB = 2) or 1 (NB = 1, only column 0 non-zero).
// part[wg][27*CIN][COUTP] in FP32; bias partials in part_b[wg][COUTP].
template <int CIN, int NB, int ZC>
__global__ void __launch_bounds__(256)
k_wgrad(const u16* __restrict__ a, const u16* __restrict__ dz, int cout, float* __restrict__ part,
        float* __restrict__ part_b, int nx, int ny, int nz) {
    constexpr int COUTP = 16 * NB;
    constexpr int LX = TX + 2, LY = TY + 2;
    constexpr int NT = CIN == 32 ? 7 : 1;           // taps per wavefront (CIN == 32)
    __shared__ __attribute__((aligned(16))) u16 at[3 * LY * LX * CIN];
    __shared__ __attribute__((aligned(16))) u16 gt[TY * TX * COUTP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int zb0 = blockIdx.z * ZC;
    const long wg = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;

    // accumulators: CIN == 32 -> [tap slot][channel subtile][nb]; CIN == 1 -> [tap subtile][nb]
    constexpr int MS = 2;
    f32x4 acc[NT][MS][NB];
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int ms = 0; ms < MS; ++ms)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[q][ms][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;   // bias gradient of channel threadIdx.x (< COUTP), this workgroup

    for (int zi = 0; zi < ZC; ++zi) {
        const int z0 = zb0 + zi;
        if (z0 >= nz) break;
        __syncthreads();
        // stage activations (with margin, zero outside) and the output gradient tile
        if constexpr (CIN % 8 == 0) {
            constexpr int CH = CIN / 8;
            for (int q = threadIdx.x; q < 3 * LY * LX * CH; q += 256) {
                const int c = q % CH, vox = q / CH;
                const int xx = vox % LX, yy = (vox / LX) % LY, zz = vox / (LX * LY);
                const int x = x0 + xx - 1, y = y0 + yy - 1, z = z0 + zz - 1;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
                    v = *reinterpret_cast<const uint4*>(a + ((long)(z * ny + y) * nx + x) * CIN + 8 * c);
                *reinterpret_cast<uint4*>(at + vox * CIN + 8 * c) = v;
            }
        } else {
            for (int vox = threadIdx.x; vox < 3 * LY * LX; vox += 256) {
                const int xx = vox % LX, yy = (vox / LX) % LY, zz = vox / (LX * LY);
                const int x = x0 + xx - 1, y = y0 + yy - 1, z = z0 + zz - 1;
                at[vox] = (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
                              ? a[(long)(z * ny + y) * nx + x] : (u16)0;
            }
        }
        for (int q = threadIdx.x; q < TY * TX * COUTP; q += 256) {
            const int n = q % COUTP, vox = q / COUTP;
            const int xx = vox % TX, yy = vox / TX;
            const int x = x0 + xx, y = y0 + yy;
            u16 g = 0;
            if (x < nx && y < ny && n < cout) g = dz[((long)(z0 * ny + y) * nx + x) * cout + n];
            gt[q] = g;
        }
        __syncthreads();
        if (threadIdx.x < COUTP) {
            for (int vox = 0; vox < TY * TX; ++vox) bsum += bf2f(gt[vox * COUTP + threadIdx.x]);
        }
        // K-steps: 32 voxels = one row (yy) of the tile
        for (int yy = 0; yy < TY; ++yy) {
            // B: gradient of voxels 8*kg .. 8*kg+7 of row yy, output channel 16*nb + i
            bf16x8 b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    b[nb][e] = __builtin_bit_cast(__bf16, gt[(yy * TX + 8 * kg + e) * COUTP + 16 * nb + i]);
            if constexpr (CIN == 32) {
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    const int t = w + 4 * q;
                    if (t < 27) {
                        const int dz_ = t / 9, dy = (t / 3) % 3, dx = t % 3;
#pragma unroll
                        for (int ms = 0; ms < MS; ++ms) {
                            bf16x8 av;   // A[c = 16*ms + i][k = voxel 8*kg + e]
#pragma unroll
                            for (int e = 0; e < 8; ++e) {
                                const int vox = (dz_ * LY + (yy + dy)) * LX + (8 * kg + e + dx);
                                av[e] = __builtin_bit_cast(__bf16, at[vox * 32 + 16 * ms + i]);
                            }
#pragma unroll
                            for (int nb = 0; nb < NB; ++nb)
                                acc[q][ms][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[nb], acc[q][ms][nb], 0, 0, 0);
                        }
                    }
                }
            } else {
                if (w == 0) {
#pragma unroll
                    for (int ms = 0; ms < MS; ++ms) {
                        bf16x8 av;   // A[t = 16*ms + i][k = voxel]
                        const int t = 16 * ms + i;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            u16 h = 0;
                            if (t < 27) {
                                const int dz_ = t / 9, dy = (t / 3) % 3, dx = t % 3;
                                h = at[(dz_ * LY + (yy + dy)) * LX + (8 * kg + e + dx)];
                            }
                            av[e] = __builtin_bit_cast(__bf16, h);
                        }
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[0][ms][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[nb], acc[0][ms][nb], 0, 0, 0);
                    }
                }
            }
        }
    }
    // write this workgroup's partials: row r = t*CIN + c (CIN == 32) or t (CIN == 1)
    float* P = part + wg * (27L * CIN * COUTP);
    if constexpr (CIN == 32) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int t = w + 4 * q;
            if (t >= 27) continue;
#pragma unroll
            for (int ms = 0; ms < MS; ++ms)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = 16 * ms + 4 * kg + e, n = 16 * nb + i;
                        P[(t * 32 + c) * COUTP + n] = acc[q][ms][nb][e];
                    }
        }
    } else {
        if (w == 0) {
#pragma unroll
            for (int ms = 0; ms < MS; ++ms)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int t = 16 * ms + 4 * kg + e, n = 16 * nb + i;
                        if (t < 27) P[t * COUTP + n] = acc[0][ms][nb][e];
                    }
        }
    }
    if (threadIdx.x < COUTP) part_b[wg * COUTP + threadIdx.x] = bsum;
}

// dW[j] (+)= sum over workgroups of part[wg][j], in workgroup order.
__global__ void __launch_bounds__(256)
k_wgrad_fold(const float* __restrict__ part, long nwg, long len, float* __restrict__ dst, int accumulate) {
    const long j = (long)blockIdx.x * 256 + threadIdx.x;
    if (j >= len) return;
    float s = 0.0f;
    for (long k = 0; k < nwg; ++k) s += part[k * len + j];
    dst[j] = accumulate ? dst[j] + s : s;
}

// ---------------------------------------------------------- loss, inputs
// x (FP32 cube) -> 1-channel bf16 activation
__global__ void k_to_bf16(const float* __restrict__ x, u16* __restrict__ a, long n) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = f2bf(x[i]);
}

// dy = (2/N_total) (y - t) as bf16 (1 channel); per-workgroup FP64 loss partial
__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ y, const float* __restrict__ t, long n, double scale, u16* __restrict__ dy,
      double* __restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const double r = (double)y[i] - (double)t[i];
        s += r * r;
        if (dy) dy[i] = f2bf((float)(2.0 * scale * r));
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------- optimiser
// Adam on FP32 master parameters (bias-corrected), grads scaled by gscale.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float bc1, float bc2,
                       float gscale) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] * gscale;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Pack FP32 weights W[27][cin][cout] into the B-fragment layout.
//   mode 0 (forward):  B_t[k = c][n = o]               = W[t][c][o]
//   mode 1 (input gradient): B_t[k = o][n = c]         = W[26 - t][c][o]
// For a 1-channel K (cin == 1 in mode 0, cout == 1 in mode 1) the taps are K.
__global__ void k_pack(const float* __restrict__ W, int cin, int cout, int mode, bf16x8* __restrict__ out) {
    const int kin = mode == 0 ? cin : cout, nout = mode == 0 ? cout : cin;
    const int NB = (nout + 15) / 16;
    const int ntap_blocks = kin == 1 ? 1 : 27;
    const int total = ntap_blocks * NB * 64;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= total) return;
    const int lane = q % 64, nb = (q / 64) % NB, tb = q / (64 * NB);
    const int n = 16 * nb + (lane & 15);
    bf16x8 r;
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * (lane >> 4) + e;
        float val = 0.0f;
        if (n < nout) {
            if (kin == 1) {              // k is the tap
                if (k < 27) {
                    const int t = mode == 0 ? k : 26 - k;
                    val = mode == 0 ? W[(t * cin + 0) * cout + n] : W[(t * cin + n) * cout + 0];
                }
            } else if (k < kin) {
                const int t = mode == 0 ? tb : 26 - tb;
                val = mode == 0 ? W[(t * cin + k) * cout + n] : W[(t * cin + n) * cout + k];
            }
        }
        r[e] = __builtin_bit_cast(__bf16, f2bf(val));
    }
    out[q] = r;
}

}  // namespace igs
