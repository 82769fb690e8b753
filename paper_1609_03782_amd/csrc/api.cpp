// C ABI of the filter library: validation, handles, the pass schedule, and
// the reductions behind rho and the statistics.  See include/igfilter.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "igfilter.h"
#include "internal.h"
#include "stencil_kernels.h"

using namespace igk;

namespace igk {
const StencilLaunch* stencil_launch_c0_d0();
const StencilLaunch* stencil_launch_c0_d1();
const StencilLaunch* stencil_launch_c0_d2();
const StencilLaunch* stencil_launch_c1_d0();
const StencilLaunch* stencil_launch_c1_d1();
const StencilLaunch* stencil_launch_c1_d2();
const StencilLaunch* stencil_launch_c2_d0();
const StencilLaunch* stencil_launch_c2_d1();
const StencilLaunch* stencil_launch_c2_d2();

const StencilLaunch* stencil_table(int cond, int dtype) {
    using Get = const StencilLaunch* (*)();
    static const Get tab[3][3] = {
        {stencil_launch_c0_d0, stencil_launch_c0_d1, stencil_launch_c0_d2},
        {stencil_launch_c1_d0, stencil_launch_c1_d1, stencil_launch_c1_d2},
        {stencil_launch_c2_d0, stencil_launch_c2_d1, stencil_launch_c2_d2}};
    if (cond < 0 || cond > 2 || dtype < 0 || dtype > 2) return nullptr;
    return tab[cond][dtype]();
}
}  // namespace igk

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static ig_status fail(ig_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static ig_status fail(ig_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                             \
    } while (0)

extern "C" const char* ig_status_string(ig_status s) {
    switch (s) {
        case IG_OK: return "ok";
        case IG_ERR_INVALID_ARG: return "invalid argument";
        case IG_ERR_OUT_OF_MEMORY: return "out of device memory";
        case IG_ERR_DEVICE: return "device error";
        case IG_ERR_NONFINITE: return "non-finite input";
        case IG_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" const char* ig_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* ig_version(void) { return "0.1.0"; }

// ------------------------------------------------------------------ device guard
namespace {
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t dtype_size(int dt) { return dt == IG_F32 ? 4 : 2; }

bool finite_f(float v) { return std::isfinite(v); }
}  // namespace

// ------------------------------------------------------------------ validation
ig_status igk_validate_params(const ig_params* p) {
    if (!p) return fail(IG_ERR_INVALID_ARG, "params is NULL");
    if (p->struct_size != sizeof(ig_params))
        return fail(IG_ERR_INVALID_ARG, "params.struct_size %u != %zu", p->struct_size, sizeof(ig_params));
    if (p->dtype < IG_F32 || p->dtype > IG_F16) return fail(IG_ERR_INVALID_ARG, "bad dtype %d", p->dtype);
    if (p->cond < IG_COND_INTENSITY || p->cond > IG_COND_PM_RATIONAL)
        return fail(IG_ERR_INVALID_ARG, "bad conductance %d", p->cond);
    if (p->n_iter < 0) return fail(IG_ERR_INVALID_ARG, "n_iter %d < 0", p->n_iter);
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(IG_ERR_INVALID_ARG, "shape %lld x %lld x %lld", (long long)p->nx, (long long)p->ny,
                    (long long)p->nz);
    if (p->nx > (1LL << 30) || p->ny > (1LL << 30) || p->nz > (1LL << 30) ||
        p->nx * p->ny * p->nz >= (1LL << 31))
        return fail(IG_ERR_INVALID_ARG, "cube too large (nx*ny*nz must be < 2^31)");
    if (!finite_f(p->K) || !(p->K > 0.0f)) return fail(IG_ERR_INVALID_ARG, "K must be finite and > 0");
    if (!finite_f(p->tau) || !(p->tau >= 0.0f)) return fail(IG_ERR_INVALID_ARG, "tau must be finite and >= 0");
    for (int a = 0; a < 3; ++a)
        if (!finite_f(p->C[a]) || !(p->C[a] >= 0.0f))
            return fail(IG_ERR_INVALID_ARG, "C[%d] must be finite and >= 0", a);
    if (p->reserved0 != 0.0f) return fail(IG_ERR_INVALID_ARG, "reserved0 must be 0");
    if (std::isnan(p->rms) || std::isinf(p->rms)) return fail(IG_ERR_INVALID_ARG, "rms must be finite");
    return IG_OK;
}

// ------------------------------------------------------------------ schedule
struct Plan {
    ig_schedule s;
    BlockGeom g;
    int nblocks;
};

static int pick_vec(int64_t nx) {
    for (int v : {1, 2, 4, 8})
        if (64 * v >= nx) return v;
    return 8;
}

// Fill the blocked geometry for schedule s; false if s cannot serve the shape.
static bool make_geom(const ig_params* p, const ig_schedule& s, int T, BlockGeom* g, int* nblocks) {
    const int nx = (int)p->nx, ny = (int)p->ny, nz = (int)p->nz;
    const int V = s.vec, R = s.rows, W = s.waves;
    if (!(V == 1 || V == 2 || V == 4 || V == 8)) return false;
    if (!(R == 1 || R == 2 || R == 4)) return false;
    if (W < 1 || W > 8 || T < 1 || T > 4 || s.zchunk < 1) return false;
    const int RX = 64 * V, RY = W * R;
    g->nx = nx; g->ny = ny; g->nz = nz;
    g->W = W;
    if (nx <= RX) { g->ntx = 1; g->ox = nx; }
    else {
        g->ox = RX - 2 * T;
        if (g->ox < 1) return false;
        g->ntx = (nx + g->ox - 1) / g->ox;
    }
    if (ny <= RY) { g->nty = 1; g->oy = ny; }
    else {
        g->oy = RY - 2 * T;
        if (g->oy < 1) return false;
        g->nty = (ny + g->oy - 1) / g->oy;
    }
    g->oz = std::min(s.zchunk, nz);
    g->nzc = (nz + g->oz - 1) / g->oz;
    const long nb = (long)g->ntx * g->nty * g->nzc;
    if (nb > 0x7fffffff) return false;
    *nblocks = (int)nb;
    g->remap = (nb % 8 == 0 && nb >= 64) ? 1 : 0;
    g->vec = (g->ntx == 1 && nx % V == 0) ? 1 : 0;
    return true;
}

// Heuristic schedule when no tuned entry exists.
static ig_schedule auto_schedule(const ig_params* p) {
    ig_schedule s{};
    s.kind = IG_SCHED_BLOCKED;
    s.vec = pick_vec(p->nx);
    s.rows = 2;
    s.waves = 8;
    s.t_block = std::max(1, std::min(2, p->n_iter));
    // z chunk: enough workgroups to fill 256 CUs a few times over
    const int RY = s.waves * s.rows;
    const long tiles_xy = (long)((p->nx + 64 * s.vec - 1) / (64 * s.vec)) * ((p->ny + RY - 1) / std::max(1, RY - 2 * s.t_block));
    long zc = p->nz;
    const long want = 1024;
    if (tiles_xy * 1 < want) zc = std::max<long>(16, (p->nz * tiles_xy + want - 1) / want);
    s.zchunk = (int)std::min<long>(zc, p->nz);
    return s;
}

// ------------------------------------------------------------------ handle
struct ig_filter {
    ig_params p;
    int device;
    void* scratch = nullptr;
    DevParams* dparams = nullptr;
    double* parts = nullptr;     // kPartBlocks * 6 doubles
    double* results = nullptr;   // 8 doubles
    ig_schedule sched{};         // kind == AUTO: heuristic
};

extern "C" ig_status ig_filter_create(const ig_params* p, int device, ig_filter** out) {
    if (!out) return fail(IG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(IG_ERR_DEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(IG_ERR_INVALID_ARG, "device %d of %d", device, ndev);
    DeviceGuard dg(device);
    if (!dg.ok) return fail(IG_ERR_DEVICE, "hipSetDevice(%d) failed", device);
    ig_filter* f = new ig_filter();
    f->p = *p;
    f->device = device;
    const size_t bytes = (size_t)(p->nx * p->ny * p->nz) * dtype_size(p->dtype);
    hipError_t e = hipMalloc(&f->scratch, bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&f->dparams, sizeof(DevParams));
    if (e == hipSuccess) e = hipMalloc((void**)&f->parts, sizeof(double) * kPartBlocks * 6);
    if (e == hipSuccess) e = hipMalloc((void**)&f->results, sizeof(double) * 8);
    if (e != hipSuccess) {
        ig_filter_destroy(f);
        return fail(e == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "allocation: %s",
                    hipGetErrorString(e));
    }
    f->sched.kind = IG_SCHED_AUTO;
    *out = f;
    return IG_OK;
}

extern "C" void ig_filter_destroy(ig_filter* f) {
    if (!f) return;
    DeviceGuard dg(f->device);
    if (f->scratch) (void)hipFree(f->scratch);
    if (f->dparams) (void)hipFree(f->dparams);
    if (f->parts) (void)hipFree(f->parts);
    if (f->results) (void)hipFree(f->results);
    delete f;
}

static ig_schedule resolve_schedule(const ig_filter* f) {
    if (f->sched.kind == IG_SCHED_AUTO) return auto_schedule(&f->p);
    ig_schedule s = f->sched;
    if (s.kind == IG_SCHED_BLOCKED && s.vec == 0) s.vec = pick_vec(f->p.nx);
    return s;
}

static ig_status check_schedule(const ig_params* p, const ig_schedule* s) {
    if (s->kind == IG_SCHED_AUTO || s->kind == IG_SCHED_NAIVE) return IG_OK;
    if (s->kind != IG_SCHED_BLOCKED) return fail(IG_ERR_INVALID_ARG, "bad schedule kind %d", s->kind);
    ig_schedule t = *s;
    if (t.vec == 0) t.vec = pick_vec(p->nx);
    BlockGeom g;
    int nb;
    for (int T = 1; T <= std::max(1, t.t_block); ++T)
        if (!make_geom(p, t, T, &g, &nb))
            return fail(IG_ERR_INVALID_ARG,
                        "schedule (T=%d rows=%d waves=%d zchunk=%d vec=%d) cannot serve %lldx%lldx%lld", T,
                        t.rows, t.waves, t.zchunk, t.vec, (long long)p->nx, (long long)p->ny, (long long)p->nz);
    return IG_OK;
}

extern "C" ig_status ig_schedule_check(const ig_params* p, const ig_schedule* s) {
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    if (!s) return fail(IG_ERR_INVALID_ARG, "schedule is NULL");
    return check_schedule(p, s);
}

extern "C" ig_status ig_filter_set_schedule(ig_filter* f, const ig_schedule* s) {
    if (!f) return fail(IG_ERR_INVALID_ARG, "handle is NULL");
    if (!s) { f->sched = ig_schedule{}; f->sched.kind = IG_SCHED_AUTO; return IG_OK; }
    ig_status st = check_schedule(&f->p, s);
    if (st != IG_OK) return st;
    f->sched = *s;
    return IG_OK;
}

extern "C" ig_status ig_filter_get_schedule(const ig_filter* f, ig_schedule* s) {
    if (!f || !s) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    *s = resolve_schedule(f);
    return IG_OK;
}

// Enqueue the whole filter: parameters (+ scan), passes, optional output sum.
ig_status igk_enqueue(const ig_params& p, const ig_schedule& sched, const void* d_in, void* d_out, void* scratch,
                      DevParams* dparams, double* parts, bool scan, hipStream_t stream, int* passes_out) {
    const long n = (long)(p.nx * p.ny * p.nz);
    ParamIn in{};
    in.K = p.K; in.tau = p.tau;
    for (int a = 0; a < 3; ++a) in.C[a] = p.C[a];
    in.cond = p.cond;
    in.abort_on_nonfinite = 1;
    in.rms = p.rms;
    if (scan) {
        HIP_TRY(launch_sum_partial(p.dtype, d_in, n, parts, kPartBlocks, stream));
        HIP_TRY(launch_params_final(parts, kPartBlocks, n, in, dparams, stream));
    } else {
        HIP_TRY(launch_params_final(nullptr, 0, n, in, dparams, stream));
    }
    const StencilLaunch* L = stencil_table(p.cond, p.dtype);
    if (!L) return fail(IG_ERR_UNSUPPORTED, "no kernels for cond %d dtype %d", p.cond, p.dtype);

    // pass depths
    int depths[4096];
    int P = 0;
    const int T = sched.kind == IG_SCHED_BLOCKED ? std::max(1, sched.t_block) : 1;
    if (p.n_iter > 0) {
        const int full = p.n_iter / T, rem = p.n_iter % T;
        if (full + (rem ? 1 : 0) > 4096) return fail(IG_ERR_UNSUPPORTED, "too many passes");
        for (int k = 0; k < full; ++k) depths[P++] = T;
        if (rem) depths[P++] = rem;
    }
    const void* src = d_in;
    if (P == 0) {
        if (d_in != d_out) HIP_TRY(launch_copy(p.dtype, d_in, d_out, n, dparams, stream));
        if (passes_out) *passes_out = 0;
        return IG_OK;
    }
    // buffers: pass k writes out if (P - k) is even, else scratch; the last pass writes d_out.
    if (d_in == d_out && (P % 2 == 1)) {
        // pass 1 would write the buffer it reads: split a pass if possible, else stage through scratch
        int k = -1;
        for (int j = 0; j < P; ++j) if (depths[j] >= 2) { k = j; break; }
        if (k >= 0 && P < 4096) {
            for (int j = P; j > k + 1; --j) depths[j] = depths[j - 1];
            const int d = depths[k];
            depths[k] = d / 2;
            depths[k + 1] = d - d / 2;
            ++P;
        } else {
            HIP_TRY(launch_copy(p.dtype, d_in, scratch, n, dparams, stream));
            src = scratch;
            // with src == scratch, pass 1 must write d_out: (P - 1) even holds for odd P
        }
    }
    for (int k = 1; k <= P; ++k) {
        void* dst = ((P - k) % 2 == 0) ? d_out : scratch;
        const int D = depths[k - 1];
        hipError_t e;
        if (sched.kind == IG_SCHED_NAIVE) {
            e = L->naive(src, dst, (int)p.nx, (int)p.ny, (int)p.nz, dparams, stream);
        } else {
            BlockGeom g;
            int nb;
            if (!make_geom(&p, sched, D, &g, &nb))
                return fail(IG_ERR_INVALID_ARG, "schedule cannot serve this shape");
            // vector I/O also needs both buffers aligned to a lane chunk
            const size_t al = (size_t)sched.vec * dtype_size(p.dtype);
            if (((uintptr_t)src % al) || ((uintptr_t)dst % al)) g.vec = 0;
            e = L->blocked(src, dst, g, sched.vec, sched.rows, D, dparams, stream, nb);
        }
        if (e != hipSuccess) return fail(IG_ERR_DEVICE, "stencil launch: %s", hipGetErrorString(e));
        src = dst;
    }
    if (passes_out) *passes_out = P;
    return IG_OK;
}

static bool ranges_overlap(const void* a, const void* b, size_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

extern "C" ig_status ig_filter_run(ig_filter* f, const void* d_in, void* d_out, void* hip_stream,
                                   ig_stats* stats) {
    if (!f) return fail(IG_ERR_INVALID_ARG, "handle is NULL");
    if (!d_in || !d_out) return fail(IG_ERR_INVALID_ARG, "NULL buffer");
    if (stats && stats->struct_size != sizeof(ig_stats))
        return fail(IG_ERR_INVALID_ARG, "stats.struct_size %u != %zu", stats->struct_size, sizeof(ig_stats));
    const ig_params& p = f->p;
    const size_t bytes = (size_t)(p.nx * p.ny * p.nz) * dtype_size(p.dtype);
    if (d_in != d_out && ranges_overlap(d_in, d_out, bytes))
        return fail(IG_ERR_INVALID_ARG, "input and output overlap partially");
    if (ranges_overlap(d_in, f->scratch, bytes) || ranges_overlap(d_out, f->scratch, bytes))
        return fail(IG_ERR_INVALID_ARG, "buffer overlaps the handle's scratch");
    if (((uintptr_t)d_in % dtype_size(p.dtype)) || ((uintptr_t)d_out % dtype_size(p.dtype)))
        return fail(IG_ERR_INVALID_ARG, "buffers must be aligned to the element size");
    DeviceGuard dg(f->device);
    if (!dg.ok) return fail(IG_ERR_DEVICE, "hipSetDevice(%d) failed", f->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const ig_schedule sched = resolve_schedule(f);
    const bool scan = p.rms <= 0.0 || stats != nullptr;
    int passes = 0;
    ig_status st = igk_enqueue(p, sched, d_in, d_out, f->scratch, f->dparams, f->parts, scan, s, &passes);
    if (st != IG_OK) return st;
    if (!stats) return IG_OK;

    DevParams hp;
    HIP_TRY(hipMemcpyAsync(&hp, f->dparams, sizeof hp, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->passes = passes;
    stats->rms_used = hp.rho;
    stats->sum_in = hp.sum;
    stats->nonfinite = hp.nonfinite;
    stats->monotone = (2.0 * (double)p.tau * ((double)p.C[0] + p.C[1] + p.C[2]) <= 1.0) ? 1 : 0;
    stats->schedule = sched;
    stats->sum_out = 0.0;
    if (hp.abort) return fail(IG_ERR_NONFINITE, "input holds %lld non-finite voxels", (long long)hp.nonfinite);
    const long n = (long)(p.nx * p.ny * p.nz);
    HIP_TRY(launch_sum_partial(p.dtype, d_out, n, f->parts, kPartBlocks, s));
    ParamIn dummy{};
    dummy.K = 1.0f; dummy.rms = 1.0; dummy.cond = p.cond;
    // fold the output partials with the same fixed-order kernel, into a scratch DevParams slot
    DevParams* tmp = reinterpret_cast<DevParams*>(f->results);
    static_assert(sizeof(DevParams) <= 8 * sizeof(double), "results buffer too small");
    HIP_TRY(launch_params_final(f->parts, kPartBlocks, n, dummy, tmp, s));
    DevParams ho;
    HIP_TRY(hipMemcpyAsync(&ho, tmp, sizeof ho, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->sum_out = ho.sum;
    return IG_OK;
}

// ------------------------------------------------------------------ utilities
namespace {
struct Scratch {
    int device = -1;
    double* parts = nullptr;
    double* out = nullptr;
};
thread_local Scratch g_scratch;

ig_status util_scratch(int device) {
    if (g_scratch.device == device && g_scratch.parts) return IG_OK;
    if (g_scratch.parts) {
        DeviceGuard old(g_scratch.device);
        (void)hipFree(g_scratch.parts);
        (void)hipFree(g_scratch.out);
        g_scratch = Scratch{};
    }
    HIP_TRY(hipMalloc((void**)&g_scratch.parts, sizeof(double) * kPartBlocks * 6));
    HIP_TRY(hipMalloc((void**)&g_scratch.out, sizeof(double) * 8));
    g_scratch.device = device;
    return IG_OK;
}
}  // namespace

extern "C" ig_status ig_compare(const void* d_x, int32_t x_dtype, const double* d_ref, int64_t n, double tol,
                                int device, void* hip_stream, ig_compare_result* res) {
    if (!d_x || !d_ref || !res || n < 0) return fail(IG_ERR_INVALID_ARG, "bad argument");
    if (x_dtype < 0 || x_dtype > 2) return fail(IG_ERR_INVALID_ARG, "bad dtype");
    DeviceGuard dg(device);
    if (!dg.ok) return fail(IG_ERR_DEVICE, "hipSetDevice(%d) failed", device);
    ig_status st = util_scratch(device);
    if (st != IG_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(launch_compare(x_dtype, d_x, d_ref, (long)n, tol, g_scratch.parts, kPartBlocks, g_scratch.out, s));
    double h[6];
    HIP_TRY(hipMemcpyAsync(h, g_scratch.out, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    res->max_abs = h[0];
    res->rms = n > 0 ? std::sqrt(h[1] / (double)n) : 0.0;
    res->max_ref = h[2];
    res->sum_x = h[3];
    res->sum_ref = h[4];
    res->n_over = (int64_t)h[5];
    return IG_OK;
}

extern "C" ig_status ig_reduce(const void* d_x, int32_t x_dtype, int64_t n, int device, void* hip_stream,
                               double* sum, double* sumsq, int64_t* nonfinite) {
    if (!d_x || n < 0) return fail(IG_ERR_INVALID_ARG, "bad argument");
    if (x_dtype < 0 || x_dtype > 2) return fail(IG_ERR_INVALID_ARG, "bad dtype");
    DeviceGuard dg(device);
    if (!dg.ok) return fail(IG_ERR_DEVICE, "hipSetDevice(%d) failed", device);
    ig_status st = util_scratch(device);
    if (st != IG_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(launch_sum_partial(x_dtype, d_x, (long)n, g_scratch.parts, kPartBlocks, s));
    ParamIn dummy{};
    dummy.K = 1.0f; dummy.rms = 1.0;
    DevParams* tmp = reinterpret_cast<DevParams*>(g_scratch.out);
    HIP_TRY(launch_params_final(g_scratch.parts, kPartBlocks, (long)n, dummy, tmp, s));
    DevParams h;
    HIP_TRY(hipMemcpyAsync(&h, tmp, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (sum) *sum = h.sum;
    if (sumsq) *sumsq = h.sumsq;
    if (nonfinite) *nonfinite = h.nonfinite;
    return IG_OK;
}
