// FP64 reductions on the device: the noise level rho (root mean square of
// the input; Section 3.3 takes the cube's rms as its noise level), the sums
// used for the conservation check, a non-finite scan, and error norms against
// an FP64 reference cube.
//
// Determinism: every reduction is two-stage with a fixed grid; stage one
// writes one partial per workgroup, stage two folds them in index order in a
// single workgroup.  No floating-point atomics, so results are bitwise
// reproducible run to run.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "stencil_common.h"

namespace igk {

constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide fixed-order reduction of NV doubles (sum or max per slot).
template <int NV>
__device__ void block_reduce(double (&v)[NV], const bool (&is_max)[NV]) {
    __shared__ double sh[RED_THREADS / 64][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = is_max[k] ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wid][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = sh[0][k];
            for (int j = 1; j < RED_THREADS / 64; ++j) a = is_max[k] ? fmax(a, sh[j][k]) : a + sh[j][k];
            v[k] = a;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- sums
// 16-byte loads (4 FP32 or 8 16-bit values), four in flight per thread.
template <typename ST> struct Pack;
template <> struct Pack<float> { using T = float4; static constexpr int N = 4; };
template <> struct Pack<__hip_bfloat16> { using T = uint4; static constexpr int N = 8; };
template <> struct Pack<__half> { using T = uint4; static constexpr int N = 8; };

template <typename ST>
__device__ __forceinline__ void unpack(const typename Pack<ST>::T& q, float (&o)[Pack<ST>::N]) {
    if constexpr (sizeof(ST) == 4) {
        o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
    } else {
        const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned short h = (unsigned short)(w[k >> 1] >> (16 * (k & 1)));
            ST v;
            __builtin_memcpy(&v, &h, 2);
            o[k] = Store<ST>::load(v);
        }
    }
}

__device__ __forceinline__ void acc3(float f, double& s1, double& s2, double& bad) {
    if (!isfinite(f)) { bad += 1.0; return; }
    const double d = f;
    s1 += d;
    s2 += d * d;
}

// vec: x is 16-byte aligned; n_vec packs are read as vectors, the rest singly
template <typename ST>
__global__ void __launch_bounds__(RED_THREADS)
k_sum_partial(const ST* __restrict__ x, long n, int vec, double* __restrict__ part) {
    using PT = typename Pack<ST>::T;
    constexpr int NP = Pack<ST>::N;
    double s1 = 0.0, s2 = 0.0, bad = 0.0;
    const long tid = (long)blockIdx.x * RED_THREADS + threadIdx.x;
    const long nth = (long)gridDim.x * RED_THREADS;
    long done = 0;
    if (vec) {
        const long nv = n / NP;
        const PT* xv = reinterpret_cast<const PT*>(x);
        long i = tid;
        for (; i + 3 * nth < nv; i += 4 * nth) {
            PT q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = xv[i + u * nth];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float f[NP];
                unpack<ST>(q[u], f);
#pragma unroll
                for (int k = 0; k < NP; ++k) acc3(f[k], s1, s2, bad);
            }
        }
        for (; i < nv; i += nth) {
            float f[NP];
            unpack<ST>(xv[i], f);
#pragma unroll
            for (int k = 0; k < NP; ++k) acc3(f[k], s1, s2, bad);
        }
        done = nv * NP;
    }
    for (long i = done + tid; i < n; i += nth) acc3(Store<ST>::load(x[i]), s1, s2, bad);
    double v[3] = {s1, s2, bad};
    const bool mx[3] = {false, false, false};
    block_reduce<3>(v, mx);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = v[0];
        part[3 * blockIdx.x + 1] = v[1];
        part[3 * blockIdx.x + 2] = v[2];
    }
}

// Fold the partials and derive the run's constants (DevParams).
__global__ void __launch_bounds__(RED_THREADS)
k_params_final(const double* __restrict__ part, int nparts, long n, ParamIn in, DevParams* __restrict__ out) {
    double s1 = 0.0, s2 = 0.0, bad = 0.0;
    if (part) {
        for (int j = threadIdx.x; j < nparts; j += RED_THREADS) {
            s1 += part[3 * j];
            s2 += part[3 * j + 1];
            bad += part[3 * j + 2];
        }
    }
    double v[3] = {s1, s2, bad};
    const bool mx[3] = {false, false, false};
    block_reduce<3>(v, mx);
    if (threadIdx.x != 0) return;
    DevParams P;
    P.sum = v[0];
    P.sumsq = v[1];
    P.nonfinite = (long long)v[2];
    P.abort = (part && in.abort_on_nonfinite && P.nonfinite > 0) ? 1 : 0;
    P.pad = 0;
    double rho = in.rms > 0.0 ? in.rms : (n > 0 ? sqrt(v[1] / (double)n) : 0.0);
    P.rho = rho;
    const double kr2 = ((double)in.K * rho) * ((double)in.K * rho);
    const double inv = kr2 > 0.0 ? 1.0 / kr2 : 0.0;  // rho == 0: the cube is all zeros, any value works
    double kap;
    if (in.cond == COND_PM_EXP) kap = -1.4426950408889634 * inv;   // -log2(e) / (K rho)^2
    else kap = inv;
    if (!(fabs(kap) <= 3.0e38)) kap = kap < 0 ? -3.0e38 : 3.0e38;
    P.kap = (float)kap;
    P.tau = in.tau;
    for (int a = 0; a < 3; ++a) {
        const double c = in.C[a];
        if (in.cond == COND_PM_EXP) P.coef[a] = (float)log2((double)in.tau * c);   // -inf when tau*C == 0
        else if (in.cond == COND_PM_RATIONAL) P.coef[a] = (float)((double)in.tau * c);
        else P.coef[a] = in.C[a];
    }
    P.closed = in.cond == COND_PM_EXP ? -INFINITY : 0.0f;
    *out = P;
}

// ---------------------------------------------------------------- compare
template <typename ST>
__global__ void __launch_bounds__(RED_THREADS)
k_compare_partial(const ST* __restrict__ x, const double* __restrict__ ref, long n, double tol,
                  double* __restrict__ part) {
    double mx = 0.0, sq = 0.0, mref = 0.0, sx = 0.0, sr = 0.0, over = 0.0;
    const long stride = (long)gridDim.x * RED_THREADS;
    for (long i = (long)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += stride) {
        const double a = (double)Store<ST>::load(x[i]);
        const double b = ref[i];
        const double e = fabs(a - b);
        const double e2 = isnan(e) ? INFINITY : e;   // NaN counts as an infinite error
        mx = fmax(mx, e2);
        sq += e2 * e2;
        mref = fmax(mref, fabs(b));
        sx += a;
        sr += b;
        over += (e2 > tol) ? 1.0 : 0.0;
    }
    double v[6] = {mx, sq, mref, sx, sr, over};
    const bool m[6] = {true, false, true, false, false, false};
    block_reduce<6>(v, m);
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) part[6 * blockIdx.x + k] = v[k];
}

__global__ void __launch_bounds__(RED_THREADS)
k_compare_final(const double* __restrict__ part, int nparts, double* __restrict__ out) {
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < nparts; j += RED_THREADS) {
        v[0] = fmax(v[0], part[6 * j]);
        v[1] += part[6 * j + 1];
        v[2] = fmax(v[2], part[6 * j + 2]);
        v[3] += part[6 * j + 3];
        v[4] += part[6 * j + 4];
        v[5] += part[6 * j + 5];
    }
    const bool m[6] = {true, false, true, false, false, false};
    block_reduce<6>(v, m);
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) out[k] = v[k];
}

// ---------------------------------------------------------------- copy
template <typename ST>
__global__ void __launch_bounds__(256)
k_copy(const ST* __restrict__ src, ST* __restrict__ dst, long n, const DevParams* __restrict__ dp) {
    if (dp && dp->abort) return;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// The failure of a run whose input held NaN or Inf, made visible in its
// output: every element becomes a quiet NaN.  Otherwise a no-op.
template <typename ST>
__global__ void __launch_bounds__(256)
k_nan_if_abort(ST* __restrict__ x, long n, const DevParams* __restrict__ dp) {
    if (!dp->abort) return;
    const ST q = Store<ST>::store(__builtin_nanf(""));
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = q;
}

// ---------------------------------------------------------------- launchers
template <typename ST>
static hipError_t sum_partial_t(const void* x, long n, double* part, int nblk, hipStream_t s) {
    const int vec = ((uintptr_t)x % 16 == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_sum_partial<ST>, dim3(nblk), dim3(RED_THREADS), 0, s, (const ST*)x, n, vec, part);
    return hipGetLastError();
}

hipError_t launch_sum_partial(int dtype, const void* x, long n, double* part, int nblk, hipStream_t s) {
    switch (dtype) {
        case 0: return sum_partial_t<float>(x, n, part, nblk, s);
        case 1: return sum_partial_t<__hip_bfloat16>(x, n, part, nblk, s);
        default: return sum_partial_t<__half>(x, n, part, nblk, s);
    }
}

hipError_t launch_params_final(const double* part, int nparts, long n, const ParamIn& in, DevParams* out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_params_final, dim3(1), dim3(RED_THREADS), 0, s, part, nparts, n, in, out);
    return hipGetLastError();
}

template <typename ST>
static hipError_t compare_t(const void* x, const double* ref, long n, double tol, double* part, int nblk,
                            double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_compare_partial<ST>, dim3(nblk), dim3(RED_THREADS), 0, s, (const ST*)x, ref, n, tol,
                       part);
    hipLaunchKernelGGL(k_compare_final, dim3(1), dim3(RED_THREADS), 0, s, part, nblk, out);
    return hipGetLastError();
}

hipError_t launch_compare(int dtype, const void* x, const double* ref, long n, double tol, double* part, int nblk,
                          double* out, hipStream_t s) {
    switch (dtype) {
        case 0: return compare_t<float>(x, ref, n, tol, part, nblk, out, s);
        case 1: return compare_t<__hip_bfloat16>(x, ref, n, tol, part, nblk, out, s);
        default: return compare_t<__half>(x, ref, n, tol, part, nblk, out, s);
    }
}

template <typename ST>
static hipError_t copy_t(const void* a, void* b, long n, const DevParams* dp, hipStream_t s) {
    int nblk = (int)((n + 255) / 256);
    if (nblk > 8192) nblk = 8192;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_copy<ST>, dim3(nblk), dim3(256), 0, s, (const ST*)a, (ST*)b, n, dp);
    return hipGetLastError();
}

hipError_t launch_copy(int dtype, const void* a, void* b, long n, const DevParams* dp, hipStream_t s) {
    switch (dtype) {
        case 0: return copy_t<float>(a, b, n, dp, s);
        case 1: return copy_t<__hip_bfloat16>(a, b, n, dp, s);
        default: return copy_t<__half>(a, b, n, dp, s);
    }
}

template <typename ST>
static hipError_t nan_if_abort_t(void* x, long n, const DevParams* dp, hipStream_t s) {
    int nblk = (int)((n + 255) / 256);
    if (nblk > 1024) nblk = 1024;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_nan_if_abort<ST>, dim3(nblk), dim3(256), 0, s, (ST*)x, n, dp);
    return hipGetLastError();
}

hipError_t launch_nan_if_abort(int dtype, void* x, long n, const DevParams* dp, hipStream_t s) {
    switch (dtype) {
        case 0: return nan_if_abort_t<float>(x, n, dp, s);
        case 1: return nan_if_abort_t<__hip_bfloat16>(x, n, dp, s);
        default: return nan_if_abort_t<__half>(x, n, dp, s);
    }
}

}  // namespace igk
