// Instantiates the filter-step kernels for one (conductance, storage type)
// pair, chosen at compile time by IG_COND (0..2) and IG_DTYPE (0 FP32,
// 1 bfloat16, 2 binary16).  The build compiles this file once per pair.
#include "internal.h"
#include "stencil_kernels.h"

#ifndef IG_COND
#error "IG_COND must be defined"
#endif
#ifndef IG_DTYPE
#error "IG_DTYPE must be defined"
#endif

namespace igk {

#if IG_DTYPE == 0
using ST = float;
#elif IG_DTYPE == 1
using ST = __hip_bfloat16;
#else
using ST = __half;
#endif

#define IG_CAT2(a, b) a##b
#define IG_CAT(a, b) IG_CAT2(a, b)
#define IG_SYM(name) IG_CAT(IG_CAT(IG_CAT(name, _c), IG_COND), IG_CAT(_d, IG_DTYPE))

static hipError_t naive_launch(const void* src, void* dst, int nx, int ny, int nz, const DevParams* dp,
                               hipStream_t s) {
    NaiveGeom g{nx, ny, nz};
    const int by = 4;
    dim3 grid((nx + 63) / 64, (ny + by - 1) / by, nz);
    hipLaunchKernelGGL((k_naive<IG_COND, ST>), grid, dim3(64, by), 0, s, (const ST*)src, (ST*)dst, g, dp);
    return hipGetLastError();
}

template <int V, int R, int T>
static hipError_t blocked_one(const void* src, void* dst, const BlockGeom& g, const DevParams* dp,
                              hipStream_t s, int nblocks) {
    auto kern = k_blocked<IG_COND, ST, V, R, T>;
    const size_t lds = (size_t)T * g.W * 2 * 64 * V * sizeof(float);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64, g.W), lds, s, (const ST*)src, (ST*)dst, g, dp);
    return hipGetLastError();
}

template <int V, int R>
static hipError_t blocked_T(const void* src, void* dst, const BlockGeom& g, int T, const DevParams* dp,
                            hipStream_t s, int nb) {
    switch (T) {
        case 1: return blocked_one<V, R, 1>(src, dst, g, dp, s, nb);
        case 2: return blocked_one<V, R, 2>(src, dst, g, dp, s, nb);
        case 3: return blocked_one<V, R, 3>(src, dst, g, dp, s, nb);
        case 4: return blocked_one<V, R, 4>(src, dst, g, dp, s, nb);
        default: return hipErrorInvalidValue;
    }
}

template <int V>
static hipError_t blocked_R(const void* src, void* dst, const BlockGeom& g, int R, int T, const DevParams* dp,
                            hipStream_t s, int nb) {
    switch (R) {
        case 1: return blocked_T<V, 1>(src, dst, g, T, dp, s, nb);
        case 2: return blocked_T<V, 2>(src, dst, g, T, dp, s, nb);
        case 4: return blocked_T<V, 4>(src, dst, g, T, dp, s, nb);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t blocked_launch(const void* src, void* dst, const BlockGeom& g, int V, int R, int T,
                                 const DevParams* dp, hipStream_t s, int nb) {
    switch (V) {
        case 1: return blocked_R<1>(src, dst, g, R, T, dp, s, nb);
        case 2: return blocked_R<2>(src, dst, g, R, T, dp, s, nb);
        case 4: return blocked_R<4>(src, dst, g, R, T, dp, s, nb);
        case 8: return blocked_R<8>(src, dst, g, R, T, dp, s, nb);
        default: return hipErrorInvalidValue;
    }
}

const StencilLaunch* IG_SYM(stencil_launch)() {
    static const StencilLaunch table = {naive_launch, blocked_launch};
    return &table;
}

}  // namespace igk
