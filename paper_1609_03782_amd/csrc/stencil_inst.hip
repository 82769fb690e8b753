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

template <int V, int T, bool VEC, int R>
static hipError_t stream_one(const void* src, void* dst, const BlockGeom& g, const Piece* pieces, int npieces,
                             const DevParams* dp, hipStream_t s) {
    auto kern = k_stream<IG_COND, ST, V, T, VEC, R>;
    if (g.grouped) {   // grouped plans exist for passes of depth 1 and 2 only
        if constexpr (T <= 2) kern = k_stream_grouped<IG_COND, ST, V, T, VEC, R>;
        else return hipErrorInvalidValue;
    }
    const size_t lds = stream_lds_bytes(V, T, g.W);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(npieces), dim3(64, g.W), lds, s, (const ST*)src, (ST*)dst, g, pieces, dp);
    return hipGetLastError();
}

template <int V, bool VEC, int R>
static hipError_t stream_T(const void* src, void* dst, const BlockGeom& g, int T, const Piece* pc, int np,
                           const DevParams* dp, hipStream_t s) {
    switch (T) {
        case 1: return stream_one<V, 1, VEC, R>(src, dst, g, pc, np, dp, s);
        case 2: return stream_one<V, 2, VEC, R>(src, dst, g, pc, np, dp, s);
        case 3: return stream_one<V, 3, VEC, R>(src, dst, g, pc, np, dp, s);
        case 4: return stream_one<V, 4, VEC, R>(src, dst, g, pc, np, dp, s);
        default: return hipErrorInvalidValue;
    }
}

template <int V, int R>
static hipError_t stream_V(const void* src, void* dst, const BlockGeom& g, int T, const Piece* pc, int np,
                           const DevParams* dp, hipStream_t s) {
    return g.vec ? stream_T<V, true, R>(src, dst, g, T, pc, np, dp, s)
                 : stream_T<V, false, R>(src, dst, g, T, pc, np, dp, s);
}

// Rows per wavefront above 1 exist for V = 4 only (narrow cubes).
static hipError_t blocked_launch(const void* src, void* dst, const BlockGeom& g, int V, int T, const Piece* pc,
                                 int np, const DevParams* dp, hipStream_t s) {
    if (g.R != 1 && V != 4) return hipErrorInvalidValue;
    switch (V) {
        case 1: return stream_V<1, 1>(src, dst, g, T, pc, np, dp, s);
        case 2: return stream_V<2, 1>(src, dst, g, T, pc, np, dp, s);
        case 4:
            switch (g.R) {
                case 1: return stream_V<4, 1>(src, dst, g, T, pc, np, dp, s);
                case 2: return stream_V<4, 2>(src, dst, g, T, pc, np, dp, s);
                case 4: return stream_V<4, 4>(src, dst, g, T, pc, np, dp, s);
                default: return hipErrorInvalidValue;
            }
        case 8: return stream_V<8, 1>(src, dst, g, T, pc, np, dp, s);
        default: return hipErrorInvalidValue;
    }
}

const StencilLaunch* IG_SYM(stencil_launch)() {
    static const StencilLaunch table = {naive_launch, blocked_launch};
    return &table;
}

}  // namespace igk
