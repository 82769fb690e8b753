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

#include <type_traits>

namespace igs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

enum { EPI_RAW = 0, EPI_GELU = 1, EPI_BACK_GELU = 2, EPI_RESID = 3 };

constexpr int TX = 32;   // output tile: 32 voxels in x (two 16-row MFMA tiles) ...
constexpr int TY = 4;    // ... by 4 rows in y (one per wavefront), one plane in z

// LDS stride of one voxel's channels: 32 channels padded to 40 (80 bytes), so
// the 16 lanes of one pass of a 16-byte LDS read (16 consecutive voxels, one
// 8-channel group) start 20 banks apart and cover all 64 banks once; at 64
// bytes they would meet on the same 4 banks (4-way conflicts).
template <int C> constexpr int lds_stride() { return C == 32 ? 40 : C; }

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ u16 f2bf(float f) {   // round to nearest, ties to even (finite inputs)
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

// ------------------------------------------------ conv, z-streaming, 32 in
// Error function by Abramowitz & Stegun, Handbook of Mathematical Functions,
// formula 7.1.26: erf(x) = 1 - (a1 t + ... + a5 t^5) e^{-x^2}, t = 1/(1 + p x)
// for x >= 0, |error| <= 1.5e-7 (far below the bf16 rounding of every value
// it feeds).  e2 returns e^{-x^2}, which GELU' reuses.
__device__ __forceinline__ float erf_as(float x, float* e2) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, ax, 1.0f));
    const float ex = __builtin_amdgcn_exp2f(-(ax * ax) * 1.4426950408889634f);
    float pl = __builtin_fmaf(1.061405429f, t, -1.453152027f);
    pl = __builtin_fmaf(pl, t, 1.421413741f);
    pl = __builtin_fmaf(pl, t, -0.284496736f);
    pl = __builtin_fmaf(pl, t, 0.254829592f);
    const float y = 1.0f - (pl * t) * ex;
    *e2 = ex;
    return x < 0.0f ? -y : y;
}
// gelu(z) = z/2 (1 + erf(z/sqrt2)); gelu'(z) = (1 + erf(z/sqrt2))/2 + z e^{-z^2/2}/sqrt(2 pi)
// GELU through the complementary function the same formula gives directly,
// erfc(x) = (a1 t + ... + a5 t^5) e^{-x^2} for x >= 0: with c = erfc(|z|/sqrt2),
// gelu(z) = max(z, 0) - |z|/2 c on both sides of 0 (12 VALU operations, a
// reciprocal and an exp2).
__device__ __forceinline__ float gelu_fast(float z) {
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f * 0.70710678118654752f, az, 1.0f));
    const float ex = __builtin_amdgcn_exp2f((z * -0.72134752044448170f) * z);   // e^{-z^2/2}
    float pl = __builtin_fmaf(1.061405429f, t, -1.453152027f);
    pl = __builtin_fmaf(pl, t, 1.421413741f);
    pl = __builtin_fmaf(pl, t, -0.284496736f);
    pl = __builtin_fmaf(pl, t, 0.254829592f);
    const float c = (pl * t) * ex;
    return __builtin_fmaf(-0.5f * az, c, fmaxf(z, 0.0f));
}
__device__ __forceinline__ float gelu_grad_fast(float z) {
    float e;
    const float er = erf_as(z * 0.70710678118654752f, &e);
    return 0.5f * (1.0f + er) + z * (0.39894228040143268f * e);
}
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
// four FP32 values to four bf16 (round to nearest, ties to even; the gfx950
// conversion instruction packs two per operation)
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d) {
    const bf16x4 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
    return __builtin_bit_cast(uint2, v);
}

// The convolution of a 32-channel input as a z-stream: a workgroup of 8
// wavefronts owns an output tile of 16*MT voxels in x by 8 rows in y (one
// row per wavefront, MT 16-voxel tiles each) and a chunk of planes [z0, z1),
// computed two planes at a time.  The packed weight fragments of all 27 taps
// are copied to LDS once; input planes z-1 .. z+2 (tile plus a one-voxel
// margin, zeros outside the cube) sit in a ring of four LDS slots, and while
// planes z and z+1 are computed the global loads of planes z+3 and z+4 are in
// flight in registers.  The LDS bandwidth (128 bytes per clock per CU for
// 16-byte reads, whatever the address pattern: measured) bounds this kernel,
// so each weight fragment read from LDS serves both planes: 6 fragment reads
// per tap feed 8 MFMAs instead of 4 reads feeding 4.  The weights are the
// MFMA's A operand and the activations its B operand (the same register
// fragments as the other way round), so each lane ends with four consecutive
// output channels of one voxel and stores them with one 8-byte write.  Per
// output the taps are accumulated in the order 0..26, then the bias is added.
constexpr int kZsRows = 8;
constexpr int kZsAhead = 2;   // taps whose LDS fragments are in flight ahead of the MFMAs
constexpr int kZsCS = 32;     // u16 per staged voxel (32 channels, unpadded)

template <int MT>
constexpr int zs_plane_u16() { return (16 * MT + 2) * (kZsRows + 2) * kZsCS; }
template <int MT, int NB>
constexpr size_t zs_lds_bytes() { return (size_t)27 * NB * 64 * 16 + (size_t)4 * zs_plane_u16<MT>() * 2; }

// Epilogue of the z-stream kernels: lane (i + 16 kg) holds D[m = 4 kg + e][n = i]
// of each (s, nb), output channels 16 nb + 4 kg + e of voxel 16 s + i of row y,
// plane z; four consecutive channels go out in one 8- or 16-byte store.
// Output channels are padded to 16 NB.  aux: the bf16 pre-activation
// [v][16 NB] (EPI_GELU, optional), the pre-activation of the layer below
// (EPI_BACK_GELU), or the FP32 input cube for the residual (EPI_RESID, output
// channel 0 only).
// The four bf16 pre-activations EPI_BACK_GELU multiplies by (0 outside the cube).
template <int NB>
__device__ __forceinline__ uint2 zs_pre(const void* __restrict__ aux, int s, int nb, int x0, int y, int z, int nx,
                                        int ny, int i, int kg) {
    const int x = x0 + 16 * s + i;
    if (y >= ny || x >= nx) return make_uint2(0, 0);
    const long v = (long)(z * ny + y) * nx + x;
    return *reinterpret_cast<const uint2*>(static_cast<const u16*>(aux) + v * 16 * NB + 16 * nb + 4 * kg);
}

// pb: the pre-activations of this fragment (EPI_BACK_GELU only, from zs_pre)
template <int NB, int EPI>
__device__ __forceinline__ void zs_store_one(const f32x4& d, uint2 pb, int s, int nb, const float* __restrict__ bias,
                                             void* __restrict__ out, const void* __restrict__ aux, int x0, int y, int z,
                                             int nx, int ny, int i, int kg) {
    constexpr int COUTP = 16 * NB;
    const int x = x0 + 16 * s + i;
    if (y >= ny || x >= nx) return;
    const long v = (long)(z * ny + y) * nx + x;
    const int n0 = 16 * nb + 4 * kg;
    if constexpr (EPI == EPI_RAW) {
        float4 r;
        r.x = d[0] + (bias ? bias[n0] : 0.0f);
        r.y = d[1] + (bias ? bias[n0 + 1] : 0.0f);
        r.z = d[2] + (bias ? bias[n0 + 2] : 0.0f);
        r.w = d[3] + (bias ? bias[n0 + 3] : 0.0f);
        *reinterpret_cast<float4*>(static_cast<float*>(out) + v * COUTP + n0) = r;
    } else if constexpr (EPI == EPI_GELU) {
        const float z0p = d[0] + bias[n0], z1p = d[1] + bias[n0 + 1];
        const float z2p = d[2] + bias[n0 + 2], z3p = d[3] + bias[n0 + 3];
        if (aux)
            *reinterpret_cast<uint2*>(const_cast<u16*>(static_cast<const u16*>(aux)) + v * COUTP + n0) =
                pack_bf16x4(z0p, z1p, z2p, z3p);
        *reinterpret_cast<uint2*>(static_cast<u16*>(out) + v * COUTP + n0) =
            pack_bf16x4(gelu_fast(z0p), gelu_fast(z1p), gelu_fast(z2p), gelu_fast(z3p));
    } else if constexpr (EPI == EPI_BACK_GELU) {
        const float g0 = gelu_grad_fast(__uint_as_float(pb.x << 16));
        const float g1 = gelu_grad_fast(__uint_as_float(pb.x & 0xffff0000u));
        const float g2 = gelu_grad_fast(__uint_as_float(pb.y << 16));
        const float g3 = gelu_grad_fast(__uint_as_float(pb.y & 0xffff0000u));
        *reinterpret_cast<uint2*>(static_cast<u16*>(out) + v * COUTP + n0) =
            pack_bf16x4(d[0] * g0, d[1] * g1, d[2] * g2, d[3] * g3);
    } else {   // EPI_RESID: output channel 0 only
        if (n0 == 0) static_cast<float*>(out)[v] = static_cast<const float*>(aux)[v] + (d[0] + bias[0]);
    }
}

template <int NB, int EPI, int MT>
__device__ __forceinline__ void zs_store(const f32x4 (&acc)[MT][NB], const float* __restrict__ bias,
                                         void* __restrict__ out, const void* __restrict__ aux, int x0, int y, int z,
                                         int nx, int ny, int i, int kg) {
#pragma unroll
    for (int s = 0; s < MT; ++s)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const uint2 pb = EPI == EPI_BACK_GELU ? zs_pre<NB>(aux, s, nb, x0, y, z, nx, ny, i, kg) : make_uint2(0, 0);
            zs_store_one<NB, EPI>(acc[s][nb], pb, s, nb, bias, out, aux, x0, y, z, nx, ny, i, kg);
        }
}

template <int NB, int EPI, int MT>
__global__ void __launch_bounds__(512)
k_conv_zs(const u16* __restrict__ in, const bf16x8* __restrict__ wp, const float* __restrict__ bias,
          void* __restrict__ out, const void* __restrict__ aux, int nx, int ny, int nz, int ntx, int nty, int zch) {
    constexpr int XW = 16 * MT, LX = XW + 2, LY = kZsRows + 2;
    constexpr int PLU = zs_plane_u16<MT>();
    constexpr int NT = 64 * kZsRows;                // threads
    constexpr int NCH = LX * LY * 4;               // 16-byte chunks of one staged plane
    constexpr int PER = (NCH + NT - 1) / NT;
    extern __shared__ uint4 zs_smem[];
    bf16x8* Bs = reinterpret_cast<bf16x8*>(zs_smem);
    u16* ring = reinterpret_cast<u16*>(zs_smem + 27 * NB * 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const int bt = blockIdx.x;
    const int tx = bt % ntx, ty = (bt / ntx) % nty, tz = bt / (ntx * nty);
    const int x0 = tx * XW, y0 = ty * kZsRows;
    const int z0 = tz * zch, z1 = min(nz, z0 + zch);

    for (int q = threadIdx.x; q < 27 * NB * 64; q += NT) Bs[q] = wp[q];

    uint4 st[2][PER];
    auto fetch = [&](int z, uint4 (&dst)[PER]) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int q = threadIdx.x + NT * k;
            uint4 v = make_uint4(0, 0, 0, 0);
            const int c = q & 3, vox = q >> 2;
            const int x = x0 + vox % LX - 1, y = y0 + vox / LX - 1;
            if (q < NCH && z >= 0 && z < nz && x >= 0 && x < nx && y >= 0 && y < ny)
                v = *reinterpret_cast<const uint4*>(in + ((long)(z * ny + y) * nx + x) * 32 + 8 * c);
            dst[k] = v;
        }
    };
    auto put = [&](int z, const uint4 (&src)[PER]) {   // plane z goes to slot z mod 4
        u16* slot = ring + ((z + 4) & 3) * PLU;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int q = threadIdx.x + NT * k;
            if (q < NCH) *reinterpret_cast<uint4*>(slot + (q >> 2) * kZsCS + 8 * (q & 3)) = src[k];
        }
    };
    fetch(z0 - 1, st[0]);
    put(z0 - 1, st[0]);
    fetch(z0, st[0]);
    put(z0, st[0]);
    fetch(z0 + 1, st[0]);
    fetch(z0 + 2, st[1]);

    const int y = y0 + w;
    // results of the previous pair of planes (zp, zp + 1), stored piecewise
    // during the next pair's tap loop so the epilogue's VALU work (GELU) runs
    // beside the MFMAs and LDS reads instead of between two barriers
    // (EPI_BACK_GELU: the pre-activations they need are loaded before the next
    // planes' staging loads, so their wait does not include those)
    constexpr int NPART = 2 * MT * NB;
    f32x4 prev[2][MT][NB];
    uint2 pre[2][MT][NB];
    int zp = -1;
    bool zp2 = false;   // the previous pair's second plane is an output
    auto store_part = [&](int j) {
        const int pp = j / (MT * NB), s = (j / NB) % MT, nb = j % NB;
        if (zp >= 0 && (pp == 0 || zp2))
            zs_store_one<NB, EPI>(prev[pp][s][nb], pre[pp][s][nb], s, nb, bias, out, aux, x0, y, zp + pp, nx, ny, i, kg);
    };
    for (int z = z0; z < z1; z += 2) {
        put(z + 1, st[0]);
        put(z + 2, st[1]);
        __syncthreads();
        if (z + 2 < z1) {
            fetch(z + 3, st[0]);
            fetch(z + 4, st[1]);
        }

        // planes z and z + 1 (the second is computed but not stored when the
        // chunk ends at z + 1; its inputs are the ring's planes z .. z + 2)
        f32x4 acc[2][MT][NB];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int s = 0; s < MT; ++s)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[p][s][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        // taps in order 0..26, the LDS fragments of tap t + kZsAhead read while
        // tap t's MFMAs run (the scheduling barriers keep the compiler from
        // sinking each read down to its use, which left every pair of MFMAs
        // waiting for the LDS)
        bf16x8 wr[kZsAhead + 1][NB], ar[kZsAhead + 1][2][MT];
        auto load = [&](int t, bf16x8 (&wf)[NB], bf16x8 (&av)[2][MT]) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) wf[nb] = Bs[(t * NB + nb) * 64 + lane];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const u16* slot = ring + ((z + 3 + p + dz) & 3) * PLU;   // plane z + p - 1 + dz
#pragma unroll
                for (int s = 0; s < MT; ++s) {
                    const int vox = (w + dy) * LX + (16 * s + i + dx);
                    av[p][s] = *reinterpret_cast<const bf16x8*>(slot + vox * kZsCS + 8 * kg);
                }
            }
        };
#pragma unroll
        for (int t = 0; t < kZsAhead; ++t) load(t, wr[t], ar[t]);
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            if (t + kZsAhead < 27) load(t + kZsAhead, wr[(t + kZsAhead) % (kZsAhead + 1)], ar[(t + kZsAhead) % (kZsAhead + 1)]);
            __builtin_amdgcn_sched_barrier(0);
            const int r = t % (kZsAhead + 1);
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int s = 0; s < MT; ++s)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[p][s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[r][nb], ar[r][p][s], acc[p][s][nb], 0, 0, 0);
            // one part of the previous pair's epilogue after every third tap
            if (t % 3 == 1 && t / 3 < NPART) store_part(t / 3);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int j = 9; j < NPART; ++j) store_part(j);
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int s = 0; s < MT; ++s)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    prev[p][s][nb] = acc[p][s][nb];
                    pre[p][s][nb] = EPI == EPI_BACK_GELU && (p == 0 || z + 1 < z1)
                                        ? zs_pre<NB>(aux, s, nb, x0, y, z + p, nx, ny, i, kg) : make_uint2(0, 0);
                }
        zp = z;
        zp2 = z + 1 < z1;
        __syncthreads();   // every wavefront is done with slots z - 1 and z before they take planes z + 3, z + 4
    }
#pragma unroll
    for (int j = 0; j < NPART; ++j) store_part(j);
}

// The convolution of a 1-channel input as a z-stream (the network's first
// layer, and the input gradient of its 1-channel last layer): the tiles and z
// chunks of k_conv_zs, with K = the 27 taps of one voxel (padded to 32).  The
// three input planes z-1 .. z+1 of the tile and its margin (one bf16 value per
// voxel) sit in a small LDS ring, each lane gathers its 8 taps from it, and the
// weights, the MFMA's A operand, stay in registers, so each lane ends with
// four consecutive output channels of one voxel like k_conv_zs.  Per output
// the taps are summed inside the MFMA, then the bias is added.
template <int NB, int EPI, int MT>
__global__ void __launch_bounds__(512)
k_conv1_zs(const u16* __restrict__ in, const bf16x8* __restrict__ wp, const float* __restrict__ bias,
           void* __restrict__ out, const void* __restrict__ aux, int nx, int ny, int nz, int ntx, int nty, int zch) {
    constexpr int XW = 16 * MT, LX = XW + 2, LY = kZsRows + 2, NPL = LX * LY;
    static_assert(NPL <= 64 * kZsRows, "one staged voxel per thread");
    __shared__ u16 ring[3 * NPL + 16 * MT];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const int bt = blockIdx.x;
    const int tx = bt % ntx, ty = (bt / ntx) % nty, tz = bt / (ntx * nty);
    const int x0 = tx * XW, y0 = ty * kZsRows;
    const int z0 = tz * zch, z1 = min(nz, z0 + zch);

    bf16x8 wf[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) wf[nb] = wp[nb * 64 + lane];

    // thread q stages voxel q of every plane (zero outside the cube); plane p
    // sits in slot (p - z0 + 1) mod 3, and zeros after the three slots stand
    // for the padding taps 27..31
    const int q = threadIdx.x;
    const int qx = x0 + q % LX - 1, qy = y0 + q / LX - 1;
    const bool qin = q < NPL && qx >= 0 && qx < nx && qy >= 0 && qy < ny;
    const long qoff = qin ? (long)qy * nx + qx : 0;
    const long plane = (long)nx * ny;
    auto fetch = [&](int z) -> u16 { return (qin && z >= 0 && z < nz) ? in[z * plane + qoff] : (u16)0; };
    auto put = [&](int z, u16 v) {
        if (q < NPL) ring[((z - z0 + 1) % 3) * NPL + q] = v;
    };
    if (threadIdx.x < 16 * MT) ring[3 * NPL + threadIdx.x] = 0;
    // this lane's 8 taps t = 8 kg + e of voxel i, for each of the three ring
    // rotations r = (z - z0) mod 3: the LDS index of the tap's input voxel
    int gidx[3][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int t = 8 * kg + e;
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        const int off = (w + dy) * LX + i + dx;
#pragma unroll
        for (int r = 0; r < 3; ++r) gidx[r][e] = t < 27 ? ((r + dz) % 3) * NPL + off : 3 * NPL;
    }
    put(z0 - 1, fetch(z0 - 1));
    put(z0, fetch(z0));
    u16 nxt = fetch(z0 + 1);

    const int y = y0 + w;
    // one plane; R = (z - z0) mod 3 known at compile time
    auto plane_step = [&](int z, auto R) {
        put(z + 1, nxt);
        __syncthreads();
        if (z + 1 < z1) nxt = fetch(z + 2);

        f32x4 acc[MT][NB];
#pragma unroll
        for (int s = 0; s < MT; ++s) {
            bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = __builtin_bit_cast(__bf16, ring[gidx[decltype(R)::value][e] + 16 * s]);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[nb], a, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
        zs_store<NB, EPI, MT>(acc, bias, out, aux, x0, y, z, nx, ny, i, kg);
        __syncthreads();   // every wavefront is done with slot (z - 1) before it takes plane z + 2
    };
    for (int z = z0; z < z1; z += 3) {
        plane_step(z, std::integral_constant<int, 0>{});
        if (z + 1 < z1) plane_step(z + 1, std::integral_constant<int, 1>{});
        if (z + 2 < z1) plane_step(z + 2, std::integral_constant<int, 2>{});
    }
}

// A 32-channel input to one output channel (the network's last layer) as a
// z-stream.  For each plane u of the tile and its one-voxel margin the MFMA
// computes the 27 per-tap sums P_t(v) = sum_c X(v, c) W[t][c] of every voxel
// (weights as the A operand, M = taps, K = channels; activations as B, 16
// voxels per MFMA), into LDS.  Output (x, y, z) then adds P_t at its 27
// neighbours: the dz = 0 taps from plane z-1, the dz = 1 taps from plane z, the
// dz = 2 taps from plane z+1, so it sums its taps in the order 0..26 and then
// adds the bias (and, for the residual, adds that to the input).  Each
// activation is read from memory and multiplied once, instead of once per tap
// with 15 of 16 MFMA columns idle.  P is double-buffered, one barrier per plane.
constexpr int kO1X = 32;                                    // output tile: 32 x kZsRows
constexpr int kO1Vox = (kO1X + 2) * (kZsRows + 2);          // voxels of the tile and margin
constexpr int kO1Groups = (kO1Vox + 15) / 16;               // MFMA column groups of 16 voxels
constexpr int kO1Stride = kO1Groups * 16 + 4;               // floats per tap (4 taps apart: 16 banks apart)
constexpr size_t kO1Lds = (size_t)2 * 27 * kO1Stride * 4;

template <int EPI>
__global__ void __launch_bounds__(512)
k_conv_out1(const u16* __restrict__ in, const bf16x8* __restrict__ wp, const float* __restrict__ bias,
            float* __restrict__ out, const float* __restrict__ aux, int nx, int ny, int nz, int ntx, int nty,
            int zch) {
    static_assert(EPI == EPI_RAW || EPI == EPI_RESID, "raw or residual output");
    constexpr int LX = kO1X + 2;
    constexpr int GPW = (kO1Groups + kZsRows - 1) / kZsRows;   // column groups per wavefront
    extern __shared__ float o1_smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const int bt = blockIdx.x;
    const int tx = bt % ntx, ty = (bt / ntx) % nty, tz = bt / (ntx * nty);
    const int x0 = tx * kO1X, y0 = ty * kZsRows;
    const int z0 = tz * zch, z1 = min(nz, z0 + zch);
    const long plane = (long)nx * ny;

    // A fragments: lane (i + 16 kg) holds W[tap 16 mb + i][channels 8 kg .. 8 kg + 7];
    // the packed B layout of tap t keeps exactly that in its lane 16 kg
    bf16x8 wa[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int t = 16 * mb + i;
        wa[mb] = t < 27 ? wp[t * 64 + 16 * kg] : bf16x8{};
    }
    // this lane's B column: voxel 16 g + i of the tile and margin, channels 8 kg ..
    long voff[GPW];
    bool vin[GPW];
#pragma unroll
    for (int k = 0; k < GPW; ++k) {
        const int g = w + kZsRows * k, q = 16 * g + i;
        const int qx = x0 + q % LX - 1, qy = y0 + q / LX - 1;
        vin[k] = g < kO1Groups && q < kO1Vox && qx >= 0 && qx < nx && qy >= 0 && qy < ny;
        voff[k] = vin[k] ? ((long)qy * nx + qx) * 32 + 8 * kg : 0;
    }
    uint4 b[GPW];
    auto fetch = [&](int u) {
#pragma unroll
        for (int k = 0; k < GPW; ++k)
            b[k] = (vin[k] && u >= 0 && u < nz) ? *reinterpret_cast<const uint4*>(in + u * plane * 32 + voff[k])
                                                : make_uint4(0, 0, 0, 0);
    };

    // output voxel of this thread (threads 256 .. 511 only compute P)
    const int ox = threadIdx.x % kO1X, oy = threadIdx.x / kO1X;
    const bool owner = threadIdx.x < kO1X * kZsRows;
    const int x = x0 + ox, y = y0 + oy;
    const bool store = owner && x < nx && y < ny;
    float a_prev = 0.f, a_cur = 0.f;   // sums of outputs z = u - 1 and z = u

    fetch(z0 - 1);
    for (int u = z0 - 1; u <= z1; ++u) {
        float* P = o1_smem + (u & 1) * 27 * kO1Stride;
#pragma unroll
        for (int k = 0; k < GPW; ++k) {
            const int g = w + kZsRows * k;
            if (g < kO1Groups) {
                const bf16x8 bv = __builtin_bit_cast(bf16x8, b[k]);
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[mb], bv, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int t = 16 * mb + 4 * kg + e;
                        if (t < 27) P[t * kO1Stride + 16 * g + i] = d[e];
                    }
                }
            }
        }
        if (u < z1) fetch(u + 1);
        __syncthreads();
        if (owner) {
            const float* c = P + oy * LX + ox;
            float a_next = c[0];
#pragma unroll
            for (int t = 1; t < 9; ++t) a_next += c[t * kO1Stride + (t / 3) * LX + t % 3];
#pragma unroll
            for (int t = 9; t < 18; ++t) a_cur += c[t * kO1Stride + ((t / 3) % 3) * LX + t % 3];
#pragma unroll
            for (int t = 18; t < 27; ++t) a_prev += c[t * kO1Stride + ((t / 3) % 3) * LX + t % 3];
            const int zo = u - 1;   // a_prev is complete
            if (store && zo >= z0) {
                const long v = (long)zo * plane + (long)y * nx + x;
                if constexpr (EPI == EPI_RESID) {
                    out[v] = aux[v] + (a_prev + bias[0]);
                } else {
                    float4 r0, r1, r2, r3;
                    r0.x = a_prev + (bias ? bias[0] : 0.0f);
                    r0.y = bias ? bias[1] : 0.0f; r0.z = bias ? bias[2] : 0.0f; r0.w = bias ? bias[3] : 0.0f;
                    r1 = bias ? make_float4(bias[4], bias[5], bias[6], bias[7]) : make_float4(0.f, 0.f, 0.f, 0.f);
                    r2 = bias ? make_float4(bias[8], bias[9], bias[10], bias[11]) : make_float4(0.f, 0.f, 0.f, 0.f);
                    r3 = bias ? make_float4(bias[12], bias[13], bias[14], bias[15]) : make_float4(0.f, 0.f, 0.f, 0.f);
                    float4* o = reinterpret_cast<float4*>(out + v * 16);
                    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
                }
            }
            a_prev = a_cur;
            a_cur = a_next;
        }
    }
}

// ---------------------------------------------------------- weight grad
// Partial dW of one workgroup: a contiguous range of "tile-planes" (32 x 4
// voxels of one plane; unit u = (z * nty + ty) * ntx + tx), the same fixed
// split of the units for every call, so the partials and their fold are
// deterministic.  Few workgroups (a couple per CU), each over many units, keep
// the partials (and the fold that reads them) small.
// CIN == 32: rows = input channels, each wavefront owns taps t = w, w+4, ...
// CIN == 1:  rows = taps (27, padded to 32), one set of accumulators.
// COUT = 32 (NB = 2) or 1 (NB = 1, only column 0 non-zero).
// part[wg][27*CIN][COUTP] in FP32; bias partials in part_b[wg][COUTP].
template <int CIN, int NB>
__global__ void __launch_bounds__(256)
k_wgrad(const u16* __restrict__ a, const u16* __restrict__ dz, int cout, float* __restrict__ part,
        float* __restrict__ part_b, int nx, int ny, int nz, int ntx, int nty, long units) {
    constexpr int COUTP = 16 * NB;
    constexpr int LX = TX + 2, LY = TY + 2;
    constexpr int NT = CIN == 32 ? 7 : 1;           // taps per wavefront (CIN == 32)
    constexpr int CS = lds_stride<CIN>();
    __shared__ __attribute__((aligned(16))) u16 at[3 * LY * LX * CS];
    __shared__ __attribute__((aligned(16))) u16 gt[TY * TX * COUTP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    const long wg = blockIdx.x;
    const long u0 = wg * units / gridDim.x, u1 = (wg + 1) * units / gridDim.x;

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

    for (long u = u0; u < u1; ++u) {
        const int x0 = (int)(u % ntx) * TX, y0 = (int)((u / ntx) % nty) * TY, z0 = (int)(u / ((long)ntx * nty));
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
                *reinterpret_cast<uint4*>(at + vox * CS + 8 * c) = v;
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
                                av[e] = __builtin_bit_cast(__bf16, at[vox * CS + 16 * ms + i]);
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

// dW[j] (+)= sum over workgroups of part[wg][j] in a fixed order: wavefront
// q of the block sums the workgroups [q nwg/4, (q+1) nwg/4) in order for 64
// consecutive j (eight loads in flight), then the four sums are added in
// order q = 0..3.
__global__ void __launch_bounds__(256)
k_wgrad_fold(const float* __restrict__ part, long nwg, long len, float* __restrict__ dst, int accumulate) {
    __shared__ float sh[4][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const long j = (long)blockIdx.x * 64 + lane;
    const long k0 = q * nwg / 4, k1 = (q + 1) * nwg / 4;
    float s = 0.0f;
    if (j < len) {
        long k = k0;
        for (; k + 8 <= k1; k += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(k + u) * len + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; k < k1; ++k) s += part[k * len + j];
    }
    sh[q][lane] = s;
    __syncthreads();
    if (q == 0 && j < len) {
        const float t = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
        dst[j] = accumulate ? dst[j] + t : t;
    }
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
// Gradient clipping by global norm: FP64 sum of squares of the gradient per
// workgroup, then one workgroup folds the partials in order and writes the
// factor min(1, max_norm / ||g||) (1 when max_norm <= 0).
__global__ void __launch_bounds__(256)
k_sumsq(const float* __restrict__ g, long n, double* __restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const double v = g[i];
        s += v * v;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_clip_factor(const double* __restrict__ part, int nparts, float max_norm, float* __restrict__ factor,
                              double* __restrict__ norm_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += part[k];
    const double nrm = sqrt(s);
    *norm_out = nrm;
    *factor = (max_norm > 0.0f && nrm > (double)max_norm) ? (float)((double)max_norm / nrm) : 1.0f;
}

// Adam on FP32 master parameters (bias-corrected), grads scaled by *gscale.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float bc1, float bc2,
                       const float* __restrict__ gscale) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] * *gscale;
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
