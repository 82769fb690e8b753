// Device-side pieces shared by every schedule of the filter step.
//
// Every kernel evaluates a voxel's update with exactly these functions, in
// the same order, so results are bitwise independent of the schedule (tile
// shape, steps per pass, batch vs single launch).  This file is compiled with
// -ffp-contract=off: no multiply-add is formed unless written as fmaf.
//
// The update (Section 3.3, Eq. 7, with the per-edge weights of the
// Perona-Malik discretisation the paper follows) is written in edge form.
// For the edge between v and its +a neighbour u, with d = I(u) - I(v):
//   PM_EXP      E = d * 2^(d^2 * kap + lc_a),  kap = -log2(e)/(K rho)^2,
//                                              lc_a = log2(tau C_a)
//   PM_RATIONAL E = (d * tc_a) / (1 + d^2 * kap), kap = 1/(K rho)^2, tc_a = tau C_a
//   INTENSITY   E = d * C_a
// and the voxel's new value is
//   PM_*        I + ((Ex+ - Ex-) + (Ey+ - Ey-)) + (Ez+ - Ez-)
//   INTENSITY   I + (tau / (1 + I^2 kap)) * (((Ex+ - Ex-) + (Ey+ - Ey-)) + (Ez+ - Ez-))
// where Ea- is the edge term of the -a edge (the +a edge of the neighbour),
// so each edge term is computed once and shared by its two voxels.  An edge
// through a cube face gets the "closed" coefficient (lc = -inf, tc = 0,
// C = 0), which makes E exactly 0: no flux through the faces.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace igk {

enum { COND_INTENSITY = 0, COND_PM_EXP = 1, COND_PM_RATIONAL = 2 };

// Per-run constants, written on the device by the rms/parameter kernel so a
// run needs no host round trip.
struct DevParams {
    float kap;        // see above, per conductance
    float tau;        // used by INTENSITY only
    float coef[3];    // lc_a / tc_a / C_a per axis (x, y, z)
    float closed;     // coefficient of a closed edge (-inf or 0)
    int32_t abort;    // non-zero: input held NaN/Inf -> kernels write nothing
    int32_t pad;
    double rho;
    double sum;       // sum of the input
    double sumsq;     // sum of squares of the input
    long long nonfinite;
};

// ---------------------------------------------------------------- storage
template <typename ST> struct Store;
template <> struct Store<float> {
    static __device__ __forceinline__ float load(float v) { return v; }
    static __device__ __forceinline__ float store(float v) { return v; }
    // value after rounding to storage and back (identity for FP32)
    static __device__ __forceinline__ float quant(float v) { return v; }
};
template <> struct Store<__hip_bfloat16> {
    static __device__ __forceinline__ float load(__hip_bfloat16 v) { return __bfloat162float(v); }
    static __device__ __forceinline__ __hip_bfloat16 store(float v) { return __float2bfloat16(v); }
    static __device__ __forceinline__ float quant(float v) { return __bfloat162float(__float2bfloat16(v)); }
};
template <> struct Store<__half> {
    static __device__ __forceinline__ float load(__half v) { return __half2float(v); }
    static __device__ __forceinline__ __half store(float v) { return __float2half_rn(v); }
    static __device__ __forceinline__ float quant(float v) { return __half2float(__float2half_rn(v)); }
};

// ---------------------------------------------------------------- edge term
template <int COND>
__device__ __forceinline__ float edge_term(float d, float coef, float kap) {
    if constexpr (COND == COND_PM_EXP) {
        const float x = __builtin_fmaf(d * d, kap, coef);
        return d * __builtin_amdgcn_exp2f(x);
    } else if constexpr (COND == COND_PM_RATIONAL) {
        const float den = __builtin_fmaf(d * d, kap, 1.0f);
        return (d * coef) * __builtin_amdgcn_rcpf(den);
    } else {
        return d * coef;
    }
}

// New value of a voxel from its edge terms (minus side first per axis).
template <int COND>
__device__ __forceinline__ float combine(float I, float exm, float exp_, float eym, float eyp,
                                         float ezm, float ezp, float kap, float tau) {
    const float acc = ((exp_ - exm) + (eyp - eym)) + (ezp - ezm);
    if constexpr (COND == COND_INTENSITY) {
        const float den = __builtin_fmaf(I * I, kap, 1.0f);
        const float ts = tau * __builtin_amdgcn_rcpf(den);
        return I + ts * acc;
    } else {
        return I + acc;
    }
}

}  // namespace igk
