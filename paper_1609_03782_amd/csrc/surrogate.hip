// Learned surrogate: model state, training step, tiled and residual-checked
// inference, and the convolution building blocks.  See include/igsurrogate.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "igdebug.h"
#include "igsurrogate.h"
#include "internal.h"
#include "surrogate_kernels.h"

using namespace igs;

#define fail igk_fail
#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                             \
    } while (0)

// Largest inference piece in voxels (2^28: 32 GiB of activation buffers);
// larger cubes are cut into slabs or tiles.  Changed by a test hook.
constexpr long kInferPieceVox = 1L << 28;
long g_infer_piece_vox = kInferPieceVox;

extern "C" int64_t ig_debug_set_infer_piece_limit(int64_t voxels) {
    const long prev = g_infer_piece_vox;
    g_infer_piece_vox = voxels > 0 ? voxels : kInferPieceVox;
    return prev;
}

namespace {

constexpr long kWgradGroups = 512;   // workgroups of the weight-gradient kernel (at most)

struct Dev {
    void* p = nullptr;
    size_t bytes = 0;
    ~Dev() { igk_free(p); }
    hipError_t ensure(size_t b) {
        if (b <= bytes && p) return hipSuccess;
        if (p) {   // queued kernels may still use the old buffer
            (void)hipDeviceSynchronize();
            igk_free(p);
            p = nullptr;
            bytes = 0;
        }
        hipError_t e = igk_malloc(&p, std::max<size_t>(b, 256));
        if (e == hipSuccess) bytes = std::max<size_t>(b, 256);
        return e;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

long wgrad_units(long nx, long ny, long nz) { return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) * nz; }
long wgrad_groups(long nx, long ny, long nz) { return std::min(kWgradGroups, wgrad_units(nx, ny, nz)); }

// Grid of the z-streaming kernels (tiles of xw voxels by kZsRows rows, one
// workgroup per (tile, z chunk)): the z chunk that minimises the slowest
// compute unit's share (in planes, counting the two margin planes and the
// set-up as about two more, and for a kernel that computes planes in pairs an
// odd chunk's last plane as a whole pair) with one workgroup per CU.
struct ZsGrid {
    int ntx, nty, zch;
    long groups;
};
ZsGrid zs_grid(long nx, long ny, long nz, int xw, bool pairs) {
    ZsGrid g;
    g.ntx = (int)((nx + xw - 1) / xw);
    g.nty = (int)((ny + kZsRows - 1) / kZsRows);
    const long tiles = (long)g.ntx * g.nty;
    int ncu = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    long best_cost = -1, zch = nz;
    for (long nzc = 1; nzc <= nz; ++nzc) {
        const long zc = (nz + nzc - 1) / nzc;
        const long groups = tiles * ((nz + zc - 1) / zc);
        const long cost = ((groups + ncu - 1) / ncu) * (zc + (pairs ? (zc & 1) : 0) + 4);
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; zch = zc; }
        if (zc == 1) break;
    }
    g.zch = (int)zch;
    g.groups = tiles * ((nz + zch - 1) / zch);
    return g;
}

// 32-channel input: 8 rows of 32 voxels (2 M-tiles) per workgroup, the largest
// tile whose four staged planes and the weights fit the 160 KB of LDS
template <int NB, int EPI>
hipError_t zs_launch(const u16* x, const bf16x8* wp, const float* b, void* out, const void* aux, long nx, long ny,
                     long nz, hipStream_t s) {
    constexpr int MT = 2;
    static_assert(zs_lds_bytes<MT, 2>() <= 160 * 1024, "z-stream tile exceeds LDS");
    const ZsGrid g = zs_grid(nx, ny, nz, 16 * MT, true);
    const size_t lds = zs_lds_bytes<MT, NB>();
    auto kern = k_conv_zs<NB, EPI, MT>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)g.groups), dim3(64 * kZsRows), lds, s, x, wp, b, out, aux, (int)nx,
                       (int)ny, (int)nz, g.ntx, g.nty, g.zch);
    return hipGetLastError();
}

// 1-channel input (first layer; input gradient of a 1-channel output)
template <int NB, int EPI>
hipError_t zs1_launch(const u16* x, const bf16x8* wp, const float* b, void* out, const void* aux, long nx, long ny,
                      long nz, hipStream_t s) {
    constexpr int MT = 2;
    const ZsGrid g = zs_grid(nx, ny, nz, 16 * MT, false);
    hipLaunchKernelGGL((k_conv1_zs<NB, EPI, MT>), dim3((unsigned)g.groups), dim3(64 * kZsRows), 0, s, x, wp, b, out,
                       aux, (int)nx, (int)ny, (int)nz, g.ntx, g.nty, g.zch);
    return hipGetLastError();
}

// 32-channel input, one output channel (last layer): per-tap partial sums
template <int EPI>
hipError_t out1_launch(const u16* x, const bf16x8* wp, const float* b, void* out, const void* aux, long nx, long ny,
                       long nz, hipStream_t s) {
    static_assert(kO1Lds <= 160 * 1024, "tap partials exceed LDS");
    const ZsGrid g = zs_grid(nx, ny, nz, kO1X, false);
    auto kern = k_conv_out1<EPI>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kO1Lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)g.groups), dim3(64 * kZsRows), kO1Lds, s, x, wp, b,
                       static_cast<float*>(out), static_cast<const float*>(aux), (int)nx, (int)ny, (int)nz, g.ntx,
                       g.nty, g.zch);
    return hipGetLastError();
}

// forward conv launch (packed weights); cin is 1 or 32
hipError_t launch_conv(int cin, int cout, int epi, const void* in, const bf16x8* wp, const float* b, void* out,
                       const void* aux, long nx, long ny, long nz, hipStream_t s) {
    const int NB = cout > 16 ? 2 : 1;
    const u16* x = static_cast<const u16*>(in);
    if (cin == 32 && cout == 1 && (epi == EPI_RAW || epi == EPI_RESID)) {
        if (epi == EPI_RAW) return out1_launch<EPI_RAW>(x, wp, b, out, aux, nx, ny, nz, s);
        return out1_launch<EPI_RESID>(x, wp, b, out, aux, nx, ny, nz, s);
    }
#define Z(F, NBV, EPIV) return F<NBV, EPIV>(x, wp, b, out, aux, nx, ny, nz, s)
#define PICK(F)                                                                                             \
    if (NB == 2) {                                                                                          \
        if (epi == EPI_RAW) Z(F, 2, EPI_RAW); else if (epi == EPI_GELU) Z(F, 2, EPI_GELU);                  \
        else if (epi == EPI_BACK_GELU) Z(F, 2, EPI_BACK_GELU); else Z(F, 2, EPI_RESID);                     \
    } else {                                                                                                \
        if (epi == EPI_RAW) Z(F, 1, EPI_RAW); else if (epi == EPI_GELU) Z(F, 1, EPI_GELU);                  \
        else if (epi == EPI_BACK_GELU) Z(F, 1, EPI_BACK_GELU); else Z(F, 1, EPI_RESID);                     \
    }
    if (cin == 32) { PICK(zs_launch) }
    PICK(zs1_launch)
#undef PICK
#undef Z
}

hipError_t launch_pack(const float* W, int cin, int cout, int mode, bf16x8* out, hipStream_t s) {
    const int kin = mode == 0 ? cin : cout, nout = mode == 0 ? cout : cin;
    const int total = (kin == 1 ? 1 : 27) * ((nout + 15) / 16) * 64;
    hipLaunchKernelGGL(k_pack, dim3((total + 255) / 256), dim3(256), 0, s, W, cin, cout, mode, out);
    return hipGetLastError();
}
size_t packed_count(int cin, int cout, int mode) {
    const int kin = mode == 0 ? cin : cout, nout = mode == 0 ? cout : cin;
    return (size_t)(kin == 1 ? 1 : 27) * ((nout + 15) / 16) * 64;
}

// weight gradient of a conv with cin (1 or 32) inputs and cout (1 or 32)
// outputs: per-workgroup partials, then a fixed-order fold into dW [27*cin][COUTP]
// and db [COUTP] (COUTP = 32, or 16 for one output: column 0 is the gradient)
hipError_t launch_wgrad(int cin, int cout, const void* a, const void* dz, Dev& part, Dev& partb, float* dW, float* db,
                        int accumulate, long nx, long ny, long nz, hipStream_t s) {
    const long units = wgrad_units(nx, ny, nz);
    const long nwg = wgrad_groups(nx, ny, nz);
    const int ntx = (int)((nx + TX - 1) / TX), nty = (int)((ny + TY - 1) / TY);
    const dim3 g((unsigned)nwg);
    const int NB = cout > 16 ? 2 : 1, COUTP = 16 * NB;
    hipError_t e = part.ensure((size_t)nwg * 27 * cin * COUTP * sizeof(float));
    if (e == hipSuccess) e = partb.ensure((size_t)nwg * COUTP * sizeof(float));
    if (e != hipSuccess) return e;
    const u16* A = static_cast<const u16*>(a);
    const u16* D = static_cast<const u16*>(dz);
    if (cin == 32 && NB == 2) hipLaunchKernelGGL((k_wgrad<32, 2>), g, dim3(256), 0, s, A, D, cout, part.as<float>(), partb.as<float>(), (int)nx, (int)ny, (int)nz, ntx, nty, units);
    else if (cin == 32) hipLaunchKernelGGL((k_wgrad<32, 1>), g, dim3(256), 0, s, A, D, cout, part.as<float>(), partb.as<float>(), (int)nx, (int)ny, (int)nz, ntx, nty, units);
    else if (NB == 2) hipLaunchKernelGGL((k_wgrad<1, 2>), g, dim3(256), 0, s, A, D, cout, part.as<float>(), partb.as<float>(), (int)nx, (int)ny, (int)nz, ntx, nty, units);
    else hipLaunchKernelGGL((k_wgrad<1, 1>), g, dim3(256), 0, s, A, D, cout, part.as<float>(), partb.as<float>(), (int)nx, (int)ny, (int)nz, ntx, nty, units);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long len = 27L * cin * COUTP;
    hipLaunchKernelGGL(k_wgrad_fold, dim3((len + 63) / 64), dim3(256), 0, s, part.as<float>(), nwg, len, dW, accumulate);
    hipLaunchKernelGGL(k_wgrad_fold, dim3(1), dim3(256), 0, s, partb.as<float>(), nwg, (long)COUTP, db, accumulate);
    return hipGetLastError();
}

__global__ void k_unpad(const float* __restrict__ src, int rows, int colsp, int cols, float* __restrict__ dst,
                        int accumulate) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= rows * cols) return;
    const int r = q / cols, c = q % cols;
    dst[q] = accumulate ? dst[q] + src[r * colsp + c] : src[r * colsp + c];
}

__global__ void k_fill(float* __restrict__ p, long n, float v) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// copy the box [o, o + d) of cube x (FP32) into a dense sub-cube
__global__ void k_gather(const float* __restrict__ x, long nx, long ny, int ox, int oy, int oz, int dx, int dy, int dz,
                         float* __restrict__ sub) {
    const long q = (long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long)dx * dy * dz) return;
    const int i = q % dx, j = (q / dx) % dy, k = q / ((long)dx * dy);
    sub[q] = x[((long)(oz + k) * ny + (oy + j)) * nx + (ox + i)];
}
// write the inner box [h, h + e) of a sub-cube of dims d to y at origin o
__global__ void k_scatter(const float* __restrict__ sub, int dx, int dy, int hx, int hy, int hz, int ex, int ey, int ez,
                          float* __restrict__ y, long nx, long ny, int ox, int oy, int oz) {
    const long q = (long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long)ex * ey * ez) return;
    const int i = q % ex, j = (q / ex) % ey, k = q / ((long)ex * ey);
    y[((long)(oz + k) * ny + (oy + j)) * nx + (ox + i)] = sub[((long)(hz + k) * dy + (hy + j)) * dx + (hx + i)];
}

// FP64 sum of (a - b)^2 per workgroup
__global__ void __launch_bounds__(256) k_diff2(const float* __restrict__ a, const float* __restrict__ b, long n,
                                                double* __restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const double d = (double)a[i] - (double)b[i];
        s += d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

}  // namespace

// ====================================================================== model
struct ig_surrogate {
    ig_surrogate_params p;
    int device;
    int L;
    std::vector<int> cin, cout;
    std::vector<size_t> w_off, b_off;   // offsets into the parameter vector
    size_t nparam = 0;
    Dev params, grads, m, v;            // FP32
    std::vector<Dev> pk_f, pk_d;        // packed bf16 weights (forward, input gradient)
    long step = 0;
    float clip = 0.0f;                  // global gradient-norm limit (0: none)
    Dev clipbuf;                        // [0]: factor (float), [8..]: norm (double), [64..]: partials
    // activations, sized for the largest cube seen
    long cap = 0;
    std::vector<Dev> act, pre;          // act[0] 1 channel, act[1..L-1] 32; pre[1..L-1]
    Dev y, dy, dzA, dzB, part, partb, parts, sub_x, sub_y, tmp;
    // inference: the bf16 input and two 32-channel buffers used in turn
    long icap = 0;
    Dev iact0, iact[2];
};

namespace {

ig_status repack(ig_surrogate* s, hipStream_t st) {
    for (int l = 0; l < s->L; ++l) {
        const float* W = s->params.as<float>() + s->w_off[l];
        HIP_TRY(launch_pack(W, s->cin[l], s->cout[l], 0, s->pk_f[l].as<bf16x8>(), st));
        HIP_TRY(launch_pack(W, s->cin[l], s->cout[l], 1, s->pk_d[l].as<bf16x8>(), st));
    }
    return IG_OK;
}

ig_status ensure_acts(ig_surrogate* s, long n) {
    if (n <= s->cap) return IG_OK;
    s->act.resize(s->L);
    s->pre.resize(s->L);
    HIP_TRY(s->act[0].ensure(n * 2));
    for (int l = 1; l < s->L; ++l) {
        HIP_TRY(s->act[l].ensure(n * 32 * 2));
        HIP_TRY(s->pre[l].ensure(n * 32 * 2));
    }
    HIP_TRY(s->y.ensure(n * 4));
    HIP_TRY(s->dy.ensure(n * 2));
    HIP_TRY(s->dzA.ensure(n * 32 * 2));
    HIP_TRY(s->dzB.ensure(n * 32 * 2));
    s->cap = n;
    return IG_OK;
}

ig_status to_bf16(const float* x, void* a, long n, hipStream_t st);

ig_status ensure_infer(ig_surrogate* s, long n) {
    if (n <= s->icap) return IG_OK;
    HIP_TRY(s->iact0.ensure(n * 2));
    HIP_TRY(s->iact[0].ensure(n * 32 * 2));
    HIP_TRY(s->iact[1].ensure(n * 32 * 2));
    s->icap = n;
    return IG_OK;
}

// inference on one cube: x converted to bf16, then the layers through two
// activation buffers in turn (no pre-activations kept); writes y (FP32)
ig_status forward_infer(ig_surrogate* s, const float* x, float* y, long nx, long ny, long nz, hipStream_t st) {
    const long n = nx * ny * nz;
    ig_status rc = ensure_infer(s, n);
    if (rc != IG_OK) return rc;
    rc = to_bf16(x, s->iact0.p, n, st);
    if (rc != IG_OK) return rc;
    const float* P = s->params.as<float>();
    const void* in = s->iact0.p;
    for (int l = 0; l < s->L; ++l) {
        const float* b = P + s->b_off[l];
        if (l < s->L - 1) {
            void* o = s->iact[l & 1].p;
            HIP_TRY(launch_conv(s->cin[l], s->cout[l], EPI_GELU, in, s->pk_f[l].as<bf16x8>(), b, o, nullptr, nx, ny, nz,
                                st));
            in = o;
        } else {
            HIP_TRY(launch_conv(s->cin[l], s->cout[l], EPI_RESID, in, s->pk_f[l].as<bf16x8>(), b, y, x, nx, ny, nz, st));
        }
    }
    return IG_OK;
}

// forward pass on one cube already converted to act[0]; writes y (FP32)
ig_status forward(ig_surrogate* s, const float* x, float* y, long nx, long ny, long nz, bool keep_pre, hipStream_t st) {
    const float* P = s->params.as<float>();
    for (int l = 0; l < s->L; ++l) {
        const float* b = P + s->b_off[l];
        if (l < s->L - 1) {
            HIP_TRY(launch_conv(s->cin[l], s->cout[l], EPI_GELU, s->act[l].p, s->pk_f[l].as<bf16x8>(), b,
                                s->act[l + 1].p, keep_pre ? s->pre[l + 1].p : nullptr, nx, ny, nz, st));
        } else {
            HIP_TRY(launch_conv(s->cin[l], s->cout[l], EPI_RESID, s->act[l].p, s->pk_f[l].as<bf16x8>(), b, y, x,
                                nx, ny, nz, st));
        }
    }
    return IG_OK;
}

ig_status to_bf16(const float* x, void* a, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, st, x, static_cast<u16*>(a), n);
    HIP_TRY(hipGetLastError());
    return IG_OK;
}

}  // namespace

extern "C" ig_status ig_surrogate_create(const ig_surrogate_params* p, int device, ig_surrogate** out) {
    if (!out) return fail(IG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p || p->struct_size != sizeof(ig_surrogate_params)) return fail(IG_ERR_INVALID_ARG, "bad params/struct_size");
    if (p->depth < 2 || p->depth > 64 || p->width != 32 || p->reserved != 0)
        return fail(IG_ERR_INVALID_ARG, "depth must be 2..64 and width 32");
    if (!(p->lr > 0) || !(p->beta1 >= 0 && p->beta1 < 1) || !(p->beta2 >= 0 && p->beta2 < 1) || !(p->eps > 0))
        return fail(IG_ERR_INVALID_ARG, "bad Adam parameters");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(IG_ERR_DEVICE, "bad device %d", device);
    if (hipSetDevice(device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    auto* s = new ig_surrogate();
    s->p = *p;
    s->device = device;
    s->L = p->depth;
    for (int l = 0; l < s->L; ++l) {
        s->cin.push_back(l == 0 ? 1 : 32);
        s->cout.push_back(l == s->L - 1 ? 1 : 32);
        s->w_off.push_back(s->nparam);
        s->nparam += 27 * s->cin[l] * s->cout[l];
        s->b_off.push_back(s->nparam);
        s->nparam += s->cout[l];
    }
    // initial weights: He normal, last layer zero (identity network)
    std::vector<float> h(s->nparam, 0.0f);
    std::mt19937_64 rng(p->seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int l = 0; l < s->L - 1; ++l) {
        const double sd = std::sqrt(2.0 / (27.0 * s->cin[l]));
        for (size_t k = 0; k < (size_t)27 * s->cin[l] * s->cout[l]; ++k) h[s->w_off[l] + k] = (float)(nd(rng) * sd);
    }
    hipError_t e = s->params.ensure(s->nparam * 4);
    if (e == hipSuccess) e = s->grads.ensure(s->nparam * 4);
    if (e == hipSuccess) e = s->m.ensure(s->nparam * 4);
    if (e == hipSuccess) e = s->v.ensure(s->nparam * 4);
    s->pk_f.resize(s->L);
    s->pk_d.resize(s->L);
    for (int l = 0; l < s->L && e == hipSuccess; ++l) {
        e = s->pk_f[l].ensure(packed_count(s->cin[l], s->cout[l], 0) * 16);
        if (e == hipSuccess) e = s->pk_d[l].ensure(packed_count(s->cin[l], s->cout[l], 1) * 16);
    }
    if (e == hipSuccess) e = s->parts.ensure(1024 * sizeof(double));
    if (e != hipSuccess) { delete s; return fail(IG_ERR_OUT_OF_MEMORY, "surrogate allocation"); }
    *out = s;
    ig_status st = ig_surrogate_set_weights(s, h.data(), (int64_t)h.size());
    if (st != IG_OK) { delete s; *out = nullptr; return st; }
    return IG_OK;
}

extern "C" void ig_surrogate_destroy(ig_surrogate* s) { delete s; }

extern "C" int64_t ig_surrogate_param_count(const ig_surrogate* s) { return s ? (int64_t)s->nparam : 0; }

extern "C" ig_status ig_surrogate_set_weights(ig_surrogate* s, const float* host, int64_t count) {
    if (!s || !host || count != (int64_t)s->nparam) return fail(IG_ERR_INVALID_ARG, "bad weights");
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    HIP_TRY(hipMemcpy(s->params.p, host, s->nparam * 4, hipMemcpyHostToDevice));
    const long n = (long)s->nparam;
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, 0, s->m.as<float>(), n, 0.0f);
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, 0, s->v.as<float>(), n, 0.0f);
    HIP_TRY(hipGetLastError());
    s->step = 0;
    ig_status st = repack(s, 0);
    if (st != IG_OK) return st;
    HIP_TRY(hipDeviceSynchronize());
    return IG_OK;
}

extern "C" ig_status ig_surrogate_get_weights(const ig_surrogate* s, float* host, int64_t count) {
    if (!s || !host || count != (int64_t)s->nparam) return fail(IG_ERR_INVALID_ARG, "bad weights");
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(host, s->params.p, s->nparam * 4, hipMemcpyDeviceToHost));
    return IG_OK;
}

extern "C" ig_status ig_surrogate_get_grads(const ig_surrogate* s, float* host, int64_t count) {
    if (!s || !host || count != (int64_t)s->nparam) return fail(IG_ERR_INVALID_ARG, "bad gradient buffer");
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(host, s->grads.p, s->nparam * 4, hipMemcpyDeviceToHost));
    return IG_OK;
}

extern "C" ig_status ig_surrogate_train_step(ig_surrogate* s, const float* const* d_x, const float* const* d_t,
                                             int32_t batch, int64_t nx, int64_t ny, int64_t nz, void* hip_stream,
                                             double* loss) {
    if (!s || !d_x || !d_t || batch < 1 || nx < 1 || ny < 1 || nz < 1) return fail(IG_ERR_INVALID_ARG, "bad arguments");
    if (nx * ny * nz >= (1LL << 31) / 32) return fail(IG_ERR_INVALID_ARG, "cube too large for training");
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    const long n = nx * ny * nz;
    for (int k = 0; k < batch; ++k) {
        ig_status cb = igk_check_buffer(d_x[k], (size_t)n * 4, s->device, "d_x[k]");
        if (cb == IG_OK) cb = igk_check_buffer(d_t[k], (size_t)n * 4, s->device, "d_t[k]");
        if (cb != IG_OK) return cb;
    }
    ig_status rc = ensure_acts(s, n);
    if (rc != IG_OK) return rc;
    {   // weight-gradient partials for the largest layer, sized before any launch
        const long nwg = wgrad_groups(nx, ny, nz);
        HIP_TRY(s->part.ensure((size_t)nwg * 27 * 32 * 32 * sizeof(float)));
        HIP_TRY(s->partb.ensure((size_t)nwg * 32 * sizeof(float)));
    }
    const long np = (long)s->nparam;
    hipLaunchKernelGGL(k_fill, dim3((np + 255) / 256), dim3(256), 0, st, s->grads.as<float>(), np, 0.0f);
    HIP_TRY(hipGetLastError());
    const int nloss = 256;
    HIP_TRY(s->tmp.ensure((size_t)batch * nloss * sizeof(double) + 64 * 1024 * 4));
    double* lparts = s->tmp.as<double>();
    float* padbuf = reinterpret_cast<float*>(lparts + (size_t)batch * nloss);   // [27*32][16] for 1-output layers
    const double scale = 1.0 / ((double)n * batch);
    for (int k = 0; k < batch; ++k) {
        if (!d_x[k] || !d_t[k]) return fail(IG_ERR_INVALID_ARG, "NULL cube %d", k);
        rc = to_bf16(d_x[k], s->act[0].p, n, st);
        if (rc != IG_OK) return rc;
        rc = forward(s, d_x[k], s->y.as<float>(), nx, ny, nz, true, st);
        if (rc != IG_OK) return rc;
        hipLaunchKernelGGL(k_mse, dim3(nloss), dim3(256), 0, st, s->y.as<float>(), d_t[k], n, scale,
                           s->dy.as<u16>(), lparts + (size_t)k * nloss);
        HIP_TRY(hipGetLastError());
        // backward: dz of layer l lives in `g` (1 channel for the last layer)
        const void* g = s->dy.p;
        for (int l = s->L - 1; l >= 0; --l) {
            float* dW = s->grads.as<float>() + s->w_off[l];
            float* db = s->grads.as<float>() + s->b_off[l];
            if (s->cout[l] == 32) {
                HIP_TRY(launch_wgrad(s->cin[l], 32, s->act[l].p, g, s->part, s->partb, dW, db, 1, nx, ny, nz, st));
            } else {   // 1 output channel: fold into a 16-column buffer, then keep column 0
                HIP_TRY(launch_wgrad(s->cin[l], 1, s->act[l].p, g, s->part, s->partb, padbuf, padbuf + 27 * 32 * 16, 0,
                                     nx, ny, nz, st));
                const int rows = 27 * s->cin[l];
                hipLaunchKernelGGL(k_unpad, dim3((rows + 255) / 256), dim3(256), 0, st, padbuf, rows, 16, 1, dW, 1);
                hipLaunchKernelGGL(k_unpad, dim3(1), dim3(256), 0, st, padbuf + 27 * 32 * 16, 1, 16, 1, db, 1);
                HIP_TRY(hipGetLastError());
            }
            if (l > 0) {   // gradient of the layer's input, through gelu' of the layer below
                void* dst = (g == s->dzA.p) ? s->dzB.p : s->dzA.p;
                HIP_TRY(launch_conv(s->cout[l], s->cin[l], EPI_BACK_GELU, g, s->pk_d[l].as<bf16x8>(), nullptr, dst,
                                    s->pre[l].p, nx, ny, nz, st));
                g = dst;
            }
        }
    }
    // Adam
    ++s->step;
    const float b1 = s->p.beta1, b2 = s->p.beta2;
    const float bc1 = 1.0f - std::pow(b1, (float)s->step), bc2 = 1.0f - std::pow(b2, (float)s->step);
    HIP_TRY(s->clipbuf.ensure(64 + 1024 * sizeof(double)));
    {
        float* factor = s->clipbuf.as<float>();
        double* norm = reinterpret_cast<double*>(s->clipbuf.as<char>() + 8);
        double* cparts = reinterpret_cast<double*>(s->clipbuf.as<char>() + 64);
        hipLaunchKernelGGL(k_sumsq, dim3(1024), dim3(256), 0, st, s->grads.as<float>(), np, cparts);
        hipLaunchKernelGGL(k_clip_factor, dim3(1), dim3(64), 0, st, cparts, 1024, s->clip, factor, norm);
        hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, st, s->params.as<float>(),
                           s->grads.as<float>(), s->m.as<float>(), s->v.as<float>(), np, s->p.lr, b1, b2, s->p.eps, bc1,
                           bc2, (const float*)factor);
    }
    HIP_TRY(hipGetLastError());
    rc = repack(s, st);
    if (rc != IG_OK) return rc;
    if (loss) {
        std::vector<double> h((size_t)batch * nloss);
        HIP_TRY(hipMemcpyAsync(h.data(), lparts, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double tot = 0.0;
        for (double v : h) tot += v;
        *loss = tot / ((double)n * batch);
    }
    return IG_OK;
}

extern "C" ig_status ig_surrogate_infer(ig_surrogate* s, const float* d_x, float* d_y, int64_t nx, int64_t ny,
                                        int64_t nz, int32_t tile, void* hip_stream) {
    if (!s || !d_x || !d_y || nx < 1 || ny < 1 || nz < 1 || tile < 0) return fail(IG_ERR_INVALID_ARG, "bad arguments");
    if (d_x == d_y) return fail(IG_ERR_INVALID_ARG, "in-place inference is not supported");
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    const long n = nx * ny * nz;
    {
        ig_status cb = igk_check_buffer(d_x, (size_t)n * 4, s->device, "d_x");
        if (cb == IG_OK) cb = igk_check_buffer(d_y, (size_t)n * 4, s->device, "d_y");
        if (cb != IG_OK) return cb;
    }
    const int H = s->L;   // receptive radius
    // one piece holds at most g_infer_piece_vox voxels (its two 32-channel
    // bf16 activation buffers take 128 bytes per voxel)
    const long kMaxVox = g_infer_piece_vox;
    auto fits = [&](long t) {
        const long d = t + 2 * H;
        return std::min(nx, d) * std::min(ny, d) * std::min(nz, d) < kMaxVox;
    };
    if (tile > 0 && !(tile >= nx && tile >= ny && tile >= nz) && !fits(tile))
        return fail(IG_ERR_INVALID_ARG, "tile %d too large: (tile + 2 depth)^3 must stay below %lld voxels", tile,
                    (long long)kMaxVox);
    // piece extents per axis: the whole cube; cubes of `tile`; or (tile == 0
    // and a cube too large for one piece) slabs of the whole x-y extent and
    // the fewest equal runs of planes whose piece with its halo fits
    long tx = nx, ty = ny, tz = nz;
    if (tile > 0 && !(tile >= nx && tile >= ny && tile >= nz)) {
        tx = ty = tz = tile;
    } else if (tile == 0 && n >= kMaxVox) {
        tz = 0;
        for (long k = 2; k <= nz; ++k) {
            const long t = (nz + k - 1) / k;
            if (nx * ny * std::min(nz, t + 2 * H) < kMaxVox) { tz = t; break; }
        }
        if (tz == 0) return fail(IG_ERR_UNSUPPORTED, "one plane of %lld x %lld voxels is too large for a piece",
                                 (long long)nx, (long long)ny);
    }
    if (tx >= nx && ty >= ny && tz >= nz) return forward_infer(s, d_x, d_y, nx, ny, nz, st);
    const long pmax = std::min(nx, tx + 2 * H) * std::min(ny, ty + 2 * H) * std::min(nz, tz + 2 * H);
    ig_status rc = ensure_infer(s, pmax);
    if (rc != IG_OK) return rc;
    HIP_TRY(s->sub_x.ensure(pmax * 4));
    HIP_TRY(s->sub_y.ensure(pmax * 4));
    for (long oz = 0; oz < nz; oz += tz)
        for (long oy = 0; oy < ny; oy += ty)
            for (long ox = 0; ox < nx; ox += tx) {
                const long ex = std::min<long>(tx, nx - ox), ey = std::min<long>(ty, ny - oy), ez = std::min<long>(tz, nz - oz);
                const long bx = std::max<long>(0, ox - H), by = std::max<long>(0, oy - H), bz = std::max<long>(0, oz - H);
                const long dx = std::min<long>(nx, ox + ex + H) - bx, dy = std::min<long>(ny, oy + ey + H) - by,
                           dz = std::min<long>(nz, oz + ez + H) - bz;
                const long m = dx * dy * dz;
                hipLaunchKernelGGL(k_gather, dim3((m + 255) / 256), dim3(256), 0, st, d_x, nx, ny, (int)bx, (int)by,
                                   (int)bz, (int)dx, (int)dy, (int)dz, s->sub_x.as<float>());
                HIP_TRY(hipGetLastError());
                rc = forward_infer(s, s->sub_x.as<float>(), s->sub_y.as<float>(), dx, dy, dz, st);
                if (rc != IG_OK) return rc;
                const long e = ex * ey * ez;
                hipLaunchKernelGGL(k_scatter, dim3((e + 255) / 256), dim3(256), 0, st, s->sub_y.as<float>(), (int)dx,
                                   (int)dy, (int)(ox - bx), (int)(oy - by), (int)(oz - bz), (int)ex, (int)ey, (int)ez,
                                   d_y, nx, ny, (int)ox, (int)oy, (int)oz);
                HIP_TRY(hipGetLastError());
            }
    return IG_OK;
}

extern "C" ig_status ig_surrogate_infer_checked(ig_surrogate* s, const ig_params* p, const float* d_x, float* d_y,
                                                int32_t tile, double slope, double threshold, void* hip_stream,
                                                ig_surrogate_report* rep) {
    if (!s || !p || !rep) return fail(IG_ERR_INVALID_ARG, "bad arguments");
    ig_status rc = igk_validate_params(p);
    if (rc != IG_OK) return rc;
    if (p->dtype != IG_F32) return fail(IG_ERR_INVALID_ARG, "FP32 cubes only");
    hipStream_t st = (hipStream_t)hip_stream;
    const long n = (long)(p->nx * p->ny * p->nz);
    rc = ig_surrogate_infer(s, d_x, d_y, p->nx, p->ny, p->nz, tile, hip_stream);
    if (rc != IG_OK) return rc;
    // rho of x (the check uses the input's noise level)
    double sum = 0, sumsq = 0;
    int64_t bad = 0;
    rc = ig_reduce(d_x, IG_F32, n, s->device, hip_stream, &sum, &sumsq, &bad);
    if (rc != IG_OK) return rc;
    if (bad) return fail(IG_ERR_NONFINITE, "input holds non-finite voxels");
    const double rho = p->rms > 0 ? p->rms : std::sqrt(sumsq / (double)n);
    // two plain steps of the prediction
    ig_params q = *p;
    q.n_iter = 2;
    q.rms = rho > 0 ? rho : 1.0;
    ig_filter* f2 = nullptr;
    rc = ig_filter_create(&q, s->device, &f2);
    if (rc != IG_OK) return rc;
    HIP_TRY(s->tmp.ensure((size_t)n * 4 + 1024 * sizeof(double)));
    float* phi = s->tmp.as<float>();
    double* dparts = reinterpret_cast<double*>(phi + n);
    rc = ig_filter_run(f2, d_y, phi, hip_stream, nullptr);
    if (rc == IG_OK) {
        const hipError_t se = hipStreamSynchronize(st);   // the handle's buffers are in use until then
        if (se != hipSuccess) rc = fail(IG_ERR_DEVICE, "sync: %s", hipGetErrorString(se));
    }
    ig_filter_destroy(f2);
    if (rc != IG_OK) return rc;
    hipLaunchKernelGGL(k_diff2, dim3(1024), dim3(256), 0, st, phi, d_y, n, dparts);
    HIP_TRY(hipGetLastError());
    std::vector<double> h(1024);
    HIP_TRY(hipMemcpyAsync(h.data(), dparts, 1024 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double tot = 0;
    for (double v : h) tot += v;
    rep->rho = rho;
    rep->residual = std::sqrt(tot / (double)n) / (rho > 0 ? rho : 1.0);
    rep->predicted_rmse = slope * rep->residual;
    rep->fell_back = 0;
    rep->reserved = 0;
    if (!(rep->predicted_rmse <= threshold)) {
        ig_filter* f = nullptr;
        rc = ig_filter_create(p, s->device, &f);
        if (rc != IG_OK) return rc;
        rc = ig_filter_run(f, d_x, d_y, hip_stream, nullptr);
        if (rc == IG_OK) {
            HIP_TRY(hipStreamSynchronize(st));
        }
        ig_filter_destroy(f);
        if (rc != IG_OK) return rc;
        rep->fell_back = 1;
    }
    return IG_OK;
}

// ------------------------------------------------------------ checkpoints
// File layout (little-endian): a 64-byte header
//   char magic[8] = "IGSURR\0\1"; uint32 header_bytes = 64; uint32 version = 1;
//   int32 depth; int32 width; int64 nparam; int64 step; uint64 seed;
//   float lr, beta1, beta2, eps;
// then FP32 params[nparam], Adam m[nparam], Adam v[nparam], then the 64-bit
// FNV-1a hash of every preceding byte.
namespace {
struct CkptHeader {
    char magic[8];
    uint32_t header_bytes, version;
    int32_t depth, width;
    int64_t nparam, step;
    uint64_t seed;
    float lr, beta1, beta2, eps;
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header must be 64 bytes");
constexpr char kCkptMagic[8] = {'I', 'G', 'S', 'U', 'R', 'R', '\0', '\1'};

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}
constexpr uint64_t kFnvBasis = 14695981039346656037ull;

// Read and check a whole checkpoint file (host only): header, sizes, hash.
ig_status read_checkpoint(const char* path, CkptHeader* hd, std::vector<float>* body) {
    if (!path || !hd) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(IG_ERR_INVALID_ARG, "cannot open %s", path);
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = fread(chunk, 1, sizeof chunk, f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    fclose(f);
    if (buf.size() < sizeof(CkptHeader) + 8) return fail(IG_ERR_INVALID_ARG, "%s: too short for a checkpoint", path);
    std::memcpy(hd, buf.data(), sizeof(CkptHeader));
    if (std::memcmp(hd->magic, kCkptMagic, 8) != 0) return fail(IG_ERR_INVALID_ARG, "%s: not a surrogate checkpoint", path);
    if (hd->header_bytes != sizeof(CkptHeader) || hd->version != 1)
        return fail(IG_ERR_INVALID_ARG, "%s: unsupported checkpoint version %u", path, hd->version);
    if (hd->nparam < 1 || hd->nparam > (1LL << 32) || hd->depth < 2 || hd->depth > 64 || hd->width != 32 || hd->step < 0)
        return fail(IG_ERR_INVALID_ARG, "%s: bad checkpoint header", path);
    const size_t want = sizeof(CkptHeader) + (size_t)hd->nparam * 12 + 8;
    if (buf.size() != want) return fail(IG_ERR_INVALID_ARG, "%s: %zu bytes, the header implies %zu", path, buf.size(), want);
    uint64_t stored;
    std::memcpy(&stored, buf.data() + want - 8, 8);
    if (fnv1a(kFnvBasis, buf.data(), want - 8) != stored)
        return fail(IG_ERR_INVALID_ARG, "%s: checksum mismatch (corrupt or truncated)", path);
    if (body) {
        body->resize((size_t)hd->nparam * 3);
        std::memcpy(body->data(), buf.data() + sizeof(CkptHeader), (size_t)hd->nparam * 12);
    }
    return IG_OK;
}
}  // namespace

extern "C" ig_status ig_surrogate_save(const ig_surrogate* s, const char* path) {
    if (!s || !path) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize());
    const size_t n = s->nparam;
    std::vector<float> body(3 * n);
    HIP_TRY(hipMemcpy(body.data(), s->params.p, n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(body.data() + n, s->m.p, n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(body.data() + 2 * n, s->v.p, n * 4, hipMemcpyDeviceToHost));
    CkptHeader hd{};
    std::memcpy(hd.magic, kCkptMagic, 8);
    hd.header_bytes = sizeof(CkptHeader);
    hd.version = 1;
    hd.depth = s->p.depth;
    hd.width = s->p.width;
    hd.nparam = (int64_t)n;
    hd.step = s->step;
    hd.seed = s->p.seed;
    hd.lr = s->p.lr; hd.beta1 = s->p.beta1; hd.beta2 = s->p.beta2; hd.eps = s->p.eps;
    uint64_t h = fnv1a(kFnvBasis, &hd, sizeof hd);
    h = fnv1a(h, body.data(), body.size() * 4);
    // write beside the target, then rename: a reader never sees a partial file
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return fail(IG_ERR_INVALID_ARG, "cannot write %s", tmp.c_str());
    bool ok = fwrite(&hd, sizeof hd, 1, f) == 1 && fwrite(body.data(), 4, body.size(), f) == body.size() &&
              fwrite(&h, 8, 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(IG_ERR_DEVICE, "writing %s failed", path);
    }
    return IG_OK;
}

extern "C" ig_status ig_surrogate_load(ig_surrogate* s, const char* path) {
    if (!s || !path) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    CkptHeader hd;
    std::vector<float> body;
    ig_status st = read_checkpoint(path, &hd, &body);
    if (st != IG_OK) return st;
    if (hd.depth != s->p.depth || hd.width != s->p.width || hd.nparam != (int64_t)s->nparam)
        return fail(IG_ERR_INVALID_ARG, "%s: network of depth %d, the handle has depth %d", path, hd.depth, s->p.depth);
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize());
    const size_t n = s->nparam;
    HIP_TRY(hipMemcpy(s->params.p, body.data(), n * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->m.p, body.data() + n, n * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->v.p, body.data() + 2 * n, n * 4, hipMemcpyHostToDevice));
    s->step = hd.step;
    s->p.seed = hd.seed;
    st = repack(s, 0);
    if (st != IG_OK) return st;
    HIP_TRY(hipDeviceSynchronize());
    return IG_OK;
}

extern "C" ig_status ig_surrogate_checkpoint_info(const char* path, int32_t* depth, int32_t* width, int64_t* nparam,
                                                  int64_t* step, uint64_t* seed) {
    CkptHeader hd;
    ig_status st = read_checkpoint(path, &hd, nullptr);
    if (st != IG_OK) return st;
    if (depth) *depth = hd.depth;
    if (width) *width = hd.width;
    if (nparam) *nparam = hd.nparam;
    if (step) *step = hd.step;
    if (seed) *seed = hd.seed;
    return IG_OK;
}

extern "C" ig_status ig_surrogate_set_lr(ig_surrogate* s, float lr) {
    if (!s || !(lr > 0) || !std::isfinite(lr)) return fail(IG_ERR_INVALID_ARG, "lr must be finite and > 0");
    s->p.lr = lr;
    return IG_OK;
}

extern "C" int64_t ig_surrogate_get_step(const ig_surrogate* s) { return s ? (int64_t)s->step : -1; }

extern "C" ig_status ig_surrogate_set_clip(ig_surrogate* s, float max_norm) {
    if (!s || !(max_norm >= 0.0f) || !std::isfinite(max_norm))
        return fail(IG_ERR_INVALID_ARG, "max_norm must be finite and >= 0");
    s->clip = max_norm;
    return IG_OK;
}

extern "C" ig_status ig_surrogate_last_grad_norm(const ig_surrogate* s, double* norm) {
    if (!s || !norm) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    if (!s->clipbuf.p || s->step == 0) return fail(IG_ERR_INVALID_ARG, "no training step taken yet");
    if (hipSetDevice(s->device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(norm, s->clipbuf.as<char>() + 8, sizeof(double), hipMemcpyDeviceToHost));
    return IG_OK;
}

// ------------------------------------------------------------ building blocks
// The single-layer entry points run one kernel over the whole cube, whose
// activations are addressed with 32-bit element offsets.
constexpr int64_t kMaxConvVox = (1LL << 31) / 32;

extern "C" ig_status ig_conv3d_forward(const void* d_in, int32_t c_in, const float* d_w, const float* d_b, int32_t c_out,
                                       int32_t epilogue, void* d_aux, void* d_out, int64_t nx, int64_t ny, int64_t nz,
                                       void* hip_stream) {
    if (!d_in || !d_w || !d_out || !(c_in == 1 || c_in == 32) || c_out < 1 || c_out > 32)
        return fail(IG_ERR_INVALID_ARG, "bad conv arguments");
    if (!(epilogue == EPI_RAW || epilogue == EPI_GELU || epilogue == EPI_RESID)) return fail(IG_ERR_INVALID_ARG, "bad epilogue");
    if (epilogue == EPI_GELU && c_out != 32) return fail(IG_ERR_INVALID_ARG, "gelu epilogue needs 32 outputs");
    if (epilogue == EPI_RESID && (c_out != 1 || !d_aux || !d_b)) return fail(IG_ERR_INVALID_ARG, "residual epilogue");
    if (nx < 1 || ny < 1 || nz < 1) return fail(IG_ERR_INVALID_ARG, "bad shape");
    if (nx * ny * nz >= kMaxConvVox) return fail(IG_ERR_INVALID_ARG, "cube too large: voxels x 32 must stay below 2^31");
    hipStream_t st = (hipStream_t)hip_stream;
    Dev pk, bias;
    HIP_TRY(pk.ensure(packed_count(c_in, c_out, 0) * 16));
    HIP_TRY(bias.ensure(32 * 4));
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, st, bias.as<float>(), 32, 0.0f);
    if (d_b) HIP_TRY(hipMemcpyAsync(bias.p, d_b, c_out * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_pack(d_w, c_in, c_out, 0, pk.as<bf16x8>(), st));
    HIP_TRY(launch_conv(c_in, c_out, epilogue, d_in, pk.as<bf16x8>(), bias.as<float>(), d_out, d_aux, nx, ny, nz, st));
    HIP_TRY(hipStreamSynchronize(st));
    return IG_OK;
}

extern "C" ig_status ig_conv3d_input_grad(const void* d_dz, int32_t c_out, const float* d_w, int32_t c_in,
                                          const void* d_aux, void* d_out, int64_t nx, int64_t ny, int64_t nz,
                                          void* hip_stream) {
    if (!d_dz || !d_w || !d_out || !(c_out == 1 || c_out == 32) || c_in < 1 || c_in > 32)
        return fail(IG_ERR_INVALID_ARG, "bad conv arguments");
    if (d_aux && c_in != 32) return fail(IG_ERR_INVALID_ARG, "gelu' epilogue needs 32 inputs");
    if (nx < 1 || ny < 1 || nz < 1) return fail(IG_ERR_INVALID_ARG, "bad shape");
    if (nx * ny * nz >= kMaxConvVox) return fail(IG_ERR_INVALID_ARG, "cube too large: voxels x 32 must stay below 2^31");
    hipStream_t st = (hipStream_t)hip_stream;
    Dev pk;
    HIP_TRY(pk.ensure(packed_count(c_in, c_out, 1) * 16));
    HIP_TRY(launch_pack(d_w, c_in, c_out, 1, pk.as<bf16x8>(), st));
    HIP_TRY(launch_conv(c_out, c_in, d_aux ? EPI_BACK_GELU : EPI_RAW, d_dz, pk.as<bf16x8>(), nullptr, d_out, d_aux, nx,
                        ny, nz, st));
    HIP_TRY(hipStreamSynchronize(st));
    return IG_OK;
}

extern "C" ig_status ig_conv3d_weight_grad(const void* d_a, int32_t c_in, const void* d_dz, int32_t c_out, float* d_dw,
                                           float* d_db, int64_t nx, int64_t ny, int64_t nz, void* hip_stream) {
    if (!d_a || !d_dz || !d_dw || !d_db || !(c_in == 1 || c_in == 32) || !(c_out == 1 || c_out == 32))
        return fail(IG_ERR_INVALID_ARG, "bad conv arguments");
    if (nx < 1 || ny < 1 || nz < 1) return fail(IG_ERR_INVALID_ARG, "bad shape");
    if (nx * ny * nz >= kMaxConvVox) return fail(IG_ERR_INVALID_ARG, "cube too large: voxels x 32 must stay below 2^31");
    hipStream_t st = (hipStream_t)hip_stream;
    Dev part, partb, pad;
    if (c_out == 32) {
        HIP_TRY(launch_wgrad(c_in, 32, d_a, d_dz, part, partb, d_dw, d_db, 0, nx, ny, nz, st));
    } else {
        HIP_TRY(pad.ensure((27 * 32 * 16 + 16) * 4));
        float* pw = pad.as<float>();
        HIP_TRY(launch_wgrad(c_in, 1, d_a, d_dz, part, partb, pw, pw + 27 * 32 * 16, 0, nx, ny, nz, st));
        const int rows = 27 * c_in;
        hipLaunchKernelGGL(k_unpad, dim3((rows + 255) / 256), dim3(256), 0, st, pw, rows, 16, 1, d_dw, 0);
        hipLaunchKernelGGL(k_unpad, dim3(1), dim3(256), 0, st, pw + 27 * 32 * 16, 1, 16, 1, d_db, 0);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(st));
    return IG_OK;
}
