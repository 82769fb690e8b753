// C ABI of the filter library: validation, handles, the pass schedule, and
// the reductions behind rho and the statistics.  See include/igfilter.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "igdebug.h"
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

#define fail igk_fail
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

extern "C" const char* ig_version(void) { return "0.1.0"; }

// ------------------------------------------------------------------ allocation
// Every device (and pinned host) allocation of the library goes through
// igk_malloc / igk_host_malloc: they count live allocations and can be made
// to fail on purpose (ig_debug_fail_alloc, or IG_FAULT_INJECT=alloc[:N] in the
// environment: the N-th allocation after the library loads, default the
// first), so the error paths can be tested for their status and their leaks.
namespace {
std::atomic<long long> g_live{0};
std::atomic<long long> g_fail_in{-1};   // > 0: allocations until the injected failure; -1: none

long long fault_env() {
    const char* e = getenv("IG_FAULT_INJECT");
    if (!e || strncmp(e, "alloc", 5) != 0) return -1;
    long long n = 1;
    if (e[5] == ':') n = atoll(e + 6);
    return n > 0 ? n : -1;
}
struct FaultInit {
    FaultInit() { g_fail_in = fault_env(); }
} g_fault_init;

bool inject_failure() {
    long long cur = g_fail_in.load();
    while (cur > 0) {
        if (g_fail_in.compare_exchange_weak(cur, cur - 1)) {
            if (cur == 1) { g_fail_in = -1; return true; }
            return false;
        }
    }
    return false;
}
}  // namespace

hipError_t igk_malloc(void** p, size_t bytes) {
    *p = nullptr;
    if (inject_failure()) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) ++g_live;
    return e;
}
void igk_free(void* p) {
    if (!p) return;
    (void)hipFree(p);
    --g_live;
}
hipError_t igk_host_malloc(void** p, size_t bytes) {
    *p = nullptr;
    if (inject_failure()) return hipErrorOutOfMemory;
    const hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) ++g_live;
    return e;
}
void igk_host_free(void* p) {
    if (!p) return;
    (void)hipHostFree(p);
    --g_live;
}

extern "C" void ig_debug_fail_alloc(int64_t nth) { g_fail_in = nth > 0 ? nth : -1; }
extern "C" int64_t ig_debug_live_allocations(void) { return (int64_t)g_live.load(); }

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

}  // namespace

// ------------------------------------------------------------------ handle
struct ig_filter {
    ig_params p;
    int device;
    void* scratch = nullptr;
    DevParams* dparams = nullptr;
    double* parts = nullptr;     // kPartBlocks * 6 doubles
    double* results = nullptr;   // 8 doubles
    ig_schedule sched{};         // kind == AUTO: heuristic
    int ncu = 256;               // compute units of the device
    // piece tables per pass depth T (index T), for the current schedule
    PassPlan plans[5];
    Piece* dpieces[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool planned[5] = {false, false, false, false, false};
    bool timing = false;         // bracket each stencil launch with events
    std::vector<hipEvent_t> ev;  // pool, pairs (start, end)
    size_t ev_used = 0;          // events recorded since the last reset
};

// Timing hook of igk_enqueue_run (unused when timing is off).
struct TimingHook {
    ig_filter* f;
    hipStream_t s;
    hipError_t record() {
        if (f->ev_used == f->ev.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            f->ev.push_back(e);
        }
        return hipEventRecord(f->ev[f->ev_used++], s);
    }
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
    hipError_t e = igk_malloc(&f->scratch, bytes);
    if (e == hipSuccess) e = igk_malloc((void**)&f->dparams, sizeof(DevParams));
    if (e == hipSuccess) e = igk_malloc((void**)&f->parts, sizeof(double) * kPartBlocks * 6);
    if (e == hipSuccess) e = igk_malloc((void**)&f->results, sizeof(double) * 8);
    if (e != hipSuccess) {
        ig_filter_destroy(f);
        return fail(e == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "allocation: %s",
                    hipGetErrorString(e));
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        f->ncu = ncu;
    f->sched.kind = IG_SCHED_AUTO;
    *out = f;
    return IG_OK;
}

extern "C" ig_status ig_filter_set_params(ig_filter* f, const ig_params* p) {
    if (!f) return fail(IG_ERR_INVALID_ARG, "handle is NULL");
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    if (p->nx != f->p.nx || p->ny != f->p.ny || p->nz != f->p.nz || p->dtype != f->p.dtype)
        return fail(IG_ERR_INVALID_ARG, "set_params keeps the shape and storage type of the handle");
    // the piece tables depend on the shape, the schedule and the pass depth only
    f->p = *p;
    return IG_OK;
}

extern "C" void ig_filter_destroy(ig_filter* f) {
    if (!f) return;
    DeviceGuard dg(f->device);
    igk_free(f->scratch);
    igk_free(f->dparams);
    igk_free(f->parts);
    igk_free(f->results);
    for (hipEvent_t e : f->ev) (void)hipEventDestroy(e);
    for (Piece* d : f->dpieces) igk_free(d);
    delete f;
}

static ig_schedule resolve_schedule(const ig_filter* f) {
    if (f->sched.kind == IG_SCHED_AUTO) return igk_auto_schedule(&f->p);
    ig_schedule s = f->sched;
    if (s.kind == IG_SCHED_BLOCKED) {
        if (s.vec == 0) {
            int V, R;
            auto_vec_rows(f->p.nx, &V, &R);
            s.vec = V;
            if (s.rows == 0) s.rows = R;
        }
        if (s.rows == 0) s.rows = 1;
    }
    return s;
}

static ig_status check_schedule(const ig_params* p, const ig_schedule* s, int ncu) {
    if (s->kind == IG_SCHED_AUTO || s->kind == IG_SCHED_NAIVE) return IG_OK;
    if (s->kind != IG_SCHED_BLOCKED) return fail(IG_ERR_INVALID_ARG, "bad schedule kind %d", s->kind);
    if (s->t_block < 1 || s->t_block > 4) return fail(IG_ERR_INVALID_ARG, "t_block must be in 1..4");
    PassPlan pp;
    // every depth a pass of this schedule may have (the remainder pass is shallower)
    for (int T = 1; T <= s->t_block; ++T) {
        const char* why = plan_pass(*p, *s, T, ncu, &pp);
        if (why)
            return fail(IG_ERR_INVALID_ARG,
                        "schedule (t_block=%d waves=%d zchunk=%d vec=%d rows=%d) cannot serve %lldx%lldx%lld: %s",
                        s->t_block, s->waves, s->zchunk, s->vec, s->rows, (long long)p->nx, (long long)p->ny,
                        (long long)p->nz, why);
    }
    return IG_OK;
}

extern "C" ig_status ig_schedule_check(const ig_params* p, const ig_schedule* s) {
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    if (!s) return fail(IG_ERR_INVALID_ARG, "schedule is NULL");
    return check_schedule(p, s, 256);
}

extern "C" ig_status ig_schedule_plan(const ig_params* p, const ig_schedule* s, int32_t t_block, int32_t ncu,
                                      int32_t* geom, int32_t* pieces, int64_t cap, int64_t* count) {
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    if (!s || !geom || !count || ncu < 1) return fail(IG_ERR_INVALID_ARG, "bad argument");
    if (s->kind != IG_SCHED_BLOCKED) return fail(IG_ERR_INVALID_ARG, "only BLOCKED schedules have a work split");
    PassPlan pp;
    const char* why = plan_pass(*p, *s, t_block, ncu, &pp);
    if (why) return fail(IG_ERR_INVALID_ARG, "%s", why);
    const int32_t g[9] = {pp.g.ntx, pp.g.nty, pp.g.ox, pp.g.oy, pp.g.W, pp.g.vec, pp.V, (int32_t)pp.pieces.size(),
                          pp.g.R};
    for (int k = 0; k < 9; ++k) geom[k] = g[k];
    *count = (int64_t)pp.pieces.size();
    if (pieces)
        for (int64_t k = 0; k < std::min<int64_t>(cap, *count); ++k) {
            pieces[4 * k] = pp.pieces[k].tx;
            pieces[4 * k + 1] = pp.pieces[k].ty;
            pieces[4 * k + 2] = pp.pieces[k].z0;
            pieces[4 * k + 3] = pp.pieces[k].z1;
        }
    return IG_OK;
}

extern "C" ig_status ig_schedule_auto(const ig_params* p, ig_schedule* out) {
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    if (!out) return fail(IG_ERR_INVALID_ARG, "out is NULL");
    *out = igk_auto_schedule(p);
    return IG_OK;
}

extern "C" ig_status ig_schedule_plan_groups(const ig_params* p, const ig_schedule* s, int32_t t_block, int32_t ncu,
                                             int32_t* first, int64_t cap, int64_t* nwg) {
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    if (!s || !nwg || ncu < 1) return fail(IG_ERR_INVALID_ARG, "bad argument");
    if (s->kind != IG_SCHED_BLOCKED) return fail(IG_ERR_INVALID_ARG, "only BLOCKED schedules have a work split");
    PassPlan pp;
    const char* why = plan_pass(*p, *s, t_block, ncu, &pp);
    if (why) return fail(IG_ERR_INVALID_ARG, "%s", why);
    *nwg = pp.first.empty() ? 0 : (int64_t)pp.first.size() - 1;
    if (first)
        for (int64_t k = 0; k < std::min<int64_t>(cap, (int64_t)pp.first.size()); ++k) first[k] = pp.first[k];
    return IG_OK;
}

static void drop_plans(ig_filter* f) {
    for (int T = 0; T < 5; ++T) {
        igk_free(f->dpieces[T]);
        f->dpieces[T] = nullptr;
        f->planned[T] = false;
    }
}

extern "C" ig_status ig_filter_set_schedule(ig_filter* f, const ig_schedule* s) {
    if (!f) return fail(IG_ERR_INVALID_ARG, "handle is NULL");
    ig_schedule next{};
    next.kind = IG_SCHED_AUTO;
    if (s) {
        ig_status st = check_schedule(&f->p, s, f->ncu);
        if (st != IG_OK) return st;
        next = *s;
    }
    DeviceGuard dg(f->device);
    drop_plans(f);
    f->sched = next;
    return IG_OK;
}

extern "C" ig_status ig_filter_get_schedule(const ig_filter* f, ig_schedule* s) {
    if (!f || !s) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    *s = resolve_schedule(f);
    return IG_OK;
}

// Plan (once) and upload the piece table of the pass of depth T.
static ig_status get_plan(ig_filter* f, const ig_schedule& sched, int T, const PassPlan** out, const Piece** dev) {
    if (!f->planned[T]) {
        const char* why = plan_pass(f->p, sched, T, f->ncu, &f->plans[T]);
        if (why) return fail(IG_ERR_INVALID_ARG, "schedule cannot serve this shape: %s", why);
        // the piece table, then (grouped plans) each workgroup's first piece
        const PassPlan& pl = f->plans[T];
        const size_t bytes = pl.pieces.size() * sizeof(Piece), extra = pl.first.size() * sizeof(int);
        igk_free(f->dpieces[T]);
        f->dpieces[T] = nullptr;
        HIP_TRY(igk_malloc((void**)&f->dpieces[T], bytes + extra));
        HIP_TRY(hipMemcpy(f->dpieces[T], pl.pieces.data(), bytes, hipMemcpyHostToDevice));
        if (extra)
            HIP_TRY(hipMemcpy(reinterpret_cast<char*>(f->dpieces[T]) + bytes, pl.first.data(), extra,
                              hipMemcpyHostToDevice));
        f->planned[T] = true;
    }
    *out = &f->plans[T];
    *dev = f->dpieces[T];
    return IG_OK;
}

static ig_status handle_plan(void* self, const ig_schedule& sched, int T, const PassPlan** out, const Piece** dev) {
    return get_plan(static_cast<ig_filter*>(self), sched, T, out, dev);
}

static hipError_t hook_record(void* self, hipStream_t s) { return static_cast<TimingHook*>(self)->record(); }

// Enqueue the whole filter: parameters (+ scan), then the passes, then (when
// the scan ran) the kernel that turns the output into NaN if the input held a
// non-finite voxel.
ig_status igk_enqueue_run(const RunCtx& c, const ig_schedule& sched, const void* d_in, void* d_out, bool scan,
                          hipStream_t stream, int* passes_out) {
    const ig_params& p = *c.p;
    const long n = (long)(p.nx * p.ny * p.nz);
    ParamIn in{};
    in.K = p.K; in.tau = p.tau;
    for (int a = 0; a < 3; ++a) in.C[a] = p.C[a];
    in.cond = p.cond;
    in.abort_on_nonfinite = 1;
    in.rms = p.rms;
    if (scan) {
        HIP_TRY(launch_sum_partial(p.dtype, d_in, n, c.parts, kPartBlocks, stream));
        HIP_TRY(launch_params_final(c.parts, kPartBlocks, n, in, c.dparams, stream));
    } else {
        HIP_TRY(launch_params_final(nullptr, 0, n, in, c.dparams, stream));
    }
    const StencilLaunch* L = stencil_table(p.cond, p.dtype);
    if (!L) return fail(IG_ERR_UNSUPPORTED, "no kernels for cond %d dtype %d", p.cond, p.dtype);
    auto record = [&]() -> hipError_t { return c.hook ? c.hook(c.hook_self, stream) : hipSuccess; };

    // pass depths
    std::vector<int> depths;
    const int T = sched.kind == IG_SCHED_BLOCKED ? std::max(1, sched.t_block) : 1;
    if (p.n_iter > 0) {
        const int full = p.n_iter / T, rem = p.n_iter % T;
        depths.assign(full, T);
        if (rem) depths.push_back(rem);
    }
    void* scratch = c.scratch;
    const void* src = d_in;
    int P = 0;
    if (depths.empty()) {
        if (d_in != d_out) HIP_TRY(launch_copy(p.dtype, d_in, d_out, n, c.dparams, stream));
    } else {
        // pass k (1-based) of P writes d_out if (P - k) is even, else scratch,
        // so the last pass writes d_out.  In place, pass 1 must not write d_in.
        if (d_in == d_out && depths.size() % 2 == 1) {
            int k = -1;
            for (size_t j = 0; j < depths.size(); ++j)
                if (depths[j] >= 2) { k = (int)j; break; }
            if (k >= 0) {   // split one pass in two: results do not depend on the split
                const int d = depths[k];
                depths[k] = d / 2;
                depths.insert(depths.begin() + k + 1, d - d / 2);
            } else {        // all passes are single steps: stage the input through scratch
                HIP_TRY(launch_copy(p.dtype, d_in, scratch, n, c.dparams, stream));
                src = scratch;
            }
        }
        P = (int)depths.size();
        for (int k = 1; k <= P; ++k) {
            void* dst = ((P - k) % 2 == 0) ? d_out : scratch;
            const int D = depths[k - 1];
            hipError_t e;
            if (sched.kind == IG_SCHED_NAIVE) {
                HIP_TRY(record());
                e = L->naive(src, dst, (int)p.nx, (int)p.ny, (int)p.nz, c.dparams, stream);
            } else {
                const PassPlan* pp;
                const Piece* dev;
                ig_status st = c.plan(c.plan_self, sched, D, &pp, &dev);
                if (st != IG_OK) return st;
                BlockGeom g = pp->g;
                // vector I/O also needs both buffers aligned to a lane chunk
                const size_t al = (size_t)pp->V * dtype_size(p.dtype);
                if (((uintptr_t)src % al) || ((uintptr_t)dst % al)) g.vec = 0;
                HIP_TRY(record());
                e = L->blocked(src, dst, g, pp->V, D, dev, pp->workgroups(), c.dparams, stream);
            }
            if (e != hipSuccess) return fail(IG_ERR_DEVICE, "stencil launch: %s", hipGetErrorString(e));
            HIP_TRY(record());
            src = dst;
        }
    }
    // a non-finite input voxel (found by the scan) turns the whole output into
    // NaN, so a caller that asked for no statistics still sees the failure
    if (scan) HIP_TRY(launch_nan_if_abort(p.dtype, d_out, n, c.dparams, stream));
    if (passes_out) *passes_out = P;
    return IG_OK;
}

// Statistics of a finished run (waits for the stream): rho, the sums, the
// non-finite count; IG_ERR_NONFINITE if the input held NaN or Inf.
ig_status igk_finish_stats(const RunCtx& c, const ig_schedule& sched, int passes, const void* d_out,
                           hipStream_t s, ig_stats* stats) {
    const ig_params& p = *c.p;
    DevParams hp;
    HIP_TRY(hipMemcpyAsync(&hp, c.dparams, sizeof hp, hipMemcpyDeviceToHost, s));
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
    HIP_TRY(launch_sum_partial(p.dtype, d_out, n, c.parts, kPartBlocks, s));
    ParamIn dummy{};
    dummy.K = 1.0f; dummy.rms = 1.0; dummy.cond = p.cond;
    // fold the output partials with the same fixed-order kernel, into a scratch DevParams slot
    DevParams* tmp = reinterpret_cast<DevParams*>(c.results);
    static_assert(sizeof(DevParams) <= 8 * sizeof(double), "results buffer too small");
    HIP_TRY(launch_params_final(c.parts, kPartBlocks, n, dummy, tmp, s));
    DevParams ho;
    HIP_TRY(hipMemcpyAsync(&ho, tmp, sizeof ho, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->sum_out = ho.sum;
    return IG_OK;
}

ig_status igk_check_buffer(const void* p, size_t bytes, int device, const char* what) {
    if (!p) return fail(IG_ERR_INVALID_ARG, "%s is NULL", what);
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // not a sticky error: clear it for the caller's next check
        return fail(IG_ERR_INVALID_ARG, "%s (%p) is not memory the GPU runtime knows", what, p);
    }
    const bool dev_mem = a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
    if (!dev_mem) return fail(IG_ERR_INVALID_ARG, "%s (%p) is not device memory", what, p);
    if (a.type == hipMemoryTypeDevice && a.device != device)
        return fail(IG_ERR_INVALID_ARG, "%s lives on device %d, the call uses device %d", what, a.device, device);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) == hipSuccess && base) {
        const uintptr_t b = (uintptr_t)base, q = (uintptr_t)p;
        if (q < b || q - b > size || bytes > size - (q - b))
            return fail(IG_ERR_INVALID_ARG, "%s: %zu bytes from %p run past the end of its allocation", what, bytes, p);
    } else {
        (void)hipGetLastError();
    }
    return IG_OK;
}

int igk_current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) d = 0;
    return d;
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
    ig_status cb = igk_check_buffer(d_in, bytes, f->device, "d_in");
    if (cb == IG_OK) cb = igk_check_buffer(d_out, bytes, f->device, "d_out");
    if (cb != IG_OK) return cb;
    DeviceGuard dg(f->device);
    if (!dg.ok) return fail(IG_ERR_DEVICE, "hipSetDevice(%d) failed", f->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const ig_schedule sched = resolve_schedule(f);
    const bool scan = p.rms <= 0.0 || stats != nullptr;
    int passes = 0;
    TimingHook hook{f, s};
    RunCtx c{&f->p, f->scratch, f->dparams, f->parts, f->results, handle_plan, f,
             f->timing ? hook_record : nullptr, &hook};
    ig_status st = igk_enqueue_run(c, sched, d_in, d_out, scan, s, &passes);
    if (st != IG_OK) return st;
    if (!stats) return IG_OK;
    return igk_finish_stats(c, sched, passes, d_out, s, stats);
}

extern "C" ig_status ig_filter_set_timing(ig_filter* f, int enable) {
    if (!f) return fail(IG_ERR_INVALID_ARG, "handle is NULL");
    f->timing = enable != 0;
    return IG_OK;
}

extern "C" ig_status ig_filter_get_timing(ig_filter* f, double* total_ms, int64_t* launches, int reset) {
    if (!f) return fail(IG_ERR_INVALID_ARG, "handle is NULL");
    DeviceGuard dg(f->device);
    double tot = 0.0;
    for (size_t k = 0; k + 1 < f->ev_used; k += 2) {
        HIP_TRY(hipEventSynchronize(f->ev[k + 1]));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, f->ev[k], f->ev[k + 1]));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)(f->ev_used / 2);
    if (reset) f->ev_used = 0;
    return IG_OK;
}

// ------------------------------------------------------------------ autotuner
namespace {
std::string tune_key(const ig_filter* f, const char* arch) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s|dtype=%d|cond=%d|%lldx%lldx%lld|n=%d", arch, f->p.dtype, f->p.cond,
             (long long)f->p.nx, (long long)f->p.ny, (long long)f->p.nz, f->p.n_iter);
    return buf;
}

// Look the key up in the cache file (lines: {"key": "...", "t_block": T, "waves": W, "rounds": R, "ms": x})
bool tune_lookup(const char* path, const std::string& key, ig_schedule* s) {
    FILE* fp = fopen(path, "r");
    if (!fp) return false;
    char line[1024];
    bool found = false;
    const std::string want = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, fp)) {
        if (!strstr(line, want.c_str())) continue;
        int T = 0, W = 0, R = 0;
        const char* a = strstr(line, "\"t_block\":");
        const char* b = strstr(line, "\"waves\":");
        const char* c = strstr(line, "\"rounds\":");
        if (a && b && c && sscanf(a, "\"t_block\": %d", &T) == 1 && sscanf(b, "\"waves\": %d", &W) == 1 &&
            sscanf(c, "\"rounds\": %d", &R) == 1) {
            *s = ig_schedule{IG_SCHED_BLOCKED, T, W, 0, 0, R};
            found = true;   // the last entry for a key wins
        }
    }
    fclose(fp);
    return found;
}

void tune_store(const char* path, const std::string& key, const ig_schedule& s, double ms) {
    FILE* fp = fopen(path, "a");
    if (!fp) return;
    fprintf(fp, "{\"key\": \"%s\", \"t_block\": %d, \"waves\": %d, \"rounds\": %d, \"ms\": %.6f}\n", key.c_str(),
            s.t_block, s.waves, s.rounds, ms);
    fclose(fp);
}
}  // namespace

extern "C" ig_status ig_filter_autotune(ig_filter* f, const void* d_in, void* d_work, void* hip_stream,
                                        ig_schedule* best, double* best_ms) {
    if (!f || !d_in || !d_work || !best) return fail(IG_ERR_INVALID_ARG, "NULL argument");
    if (d_in == d_work) return fail(IG_ERR_INVALID_ARG, "d_work must differ from d_in");
    {
        const size_t bytes = (size_t)(f->p.nx * f->p.ny * f->p.nz) * dtype_size(f->p.dtype);
        ig_status cb = igk_check_buffer(d_in, bytes, f->device, "d_in");
        if (cb == IG_OK) cb = igk_check_buffer(d_work, bytes, f->device, "d_work");
        if (cb != IG_OK) return cb;
    }
    DeviceGuard dg(f->device);
    if (!dg.ok) return fail(IG_ERR_DEVICE, "hipSetDevice(%d) failed", f->device);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, f->device));
    const std::string key = tune_key(f, prop.gcnArchName);
    const char* cache = getenv("IG_TUNE_CACHE");
    ig_schedule s{};
    if (cache && *cache && tune_lookup(cache, key, &s) && check_schedule(&f->p, &s, f->ncu) == IG_OK) {
        ig_status st = ig_filter_set_schedule(f, &s);
        if (st != IG_OK) return st;
        *best = resolve_schedule(f);
        if (best_ms) *best_ms = -1.0;
        return IG_OK;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best_t = 1e300;
    ig_schedule best_s{};
    const int maxT = std::max(1, std::min(4, f->p.n_iter));
    for (int T = 1; T <= maxT; ++T)
        for (int W : {8, 12, 16})
            for (int R : {1, 2}) {
                ig_schedule c{IG_SCHED_BLOCKED, T, W, 0, 0, R};
                if (check_schedule(&f->p, &c, f->ncu) != IG_OK) continue;
                if (ig_filter_set_schedule(f, &c) != IG_OK) continue;
                ig_status st = ig_filter_run(f, d_in, d_work, hip_stream, nullptr);   // warm-up + plan upload
                if (st != IG_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return st; }
                float ms = 0.0f;
                if (hipEventRecord(e0, stream) != hipSuccess) continue;
                for (int k = 0; k < 2; ++k) (void)ig_filter_run(f, d_in, d_work, hip_stream, nullptr);
                if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) continue;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) continue;
                if (ms / 2 < best_t) { best_t = ms / 2; best_s = c; }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_t >= 1e300) return fail(IG_ERR_UNSUPPORTED, "no blocked schedule serves this shape");
    ig_status st = ig_filter_set_schedule(f, &best_s);
    if (st != IG_OK) return st;
    *best = resolve_schedule(f);
    if (best_ms) *best_ms = best_t;
    if (cache && *cache) tune_store(cache, key, best_s, best_t);
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

void util_scratch_release() {
    if (g_scratch.parts || g_scratch.out) {
        DeviceGuard old(g_scratch.device);
        igk_free(g_scratch.parts);
        igk_free(g_scratch.out);
    }
    g_scratch = Scratch{};
}

ig_status util_scratch(int device) {
    if (g_scratch.device == device && g_scratch.parts && g_scratch.out) return IG_OK;
    util_scratch_release();
    Scratch sc;
    hipError_t e = igk_malloc((void**)&sc.parts, sizeof(double) * kPartBlocks * 6);
    if (e == hipSuccess) e = igk_malloc((void**)&sc.out, sizeof(double) * 8);
    if (e != hipSuccess) {
        igk_free(sc.parts);
        igk_free(sc.out);
        return fail(e == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "reduction scratch: %s",
                    hipGetErrorString(e));
    }
    sc.device = device;
    g_scratch = sc;
    return IG_OK;
}
}  // namespace

void igk_quality_cache_release();
extern "C" void ig_debug_release_caches(void) {
    util_scratch_release();
    igk_quality_cache_release();
    ig_batch_cache_clear();
}

extern "C" ig_status ig_compare(const void* d_x, int32_t x_dtype, const double* d_ref, int64_t n, double tol,
                                int device, void* hip_stream, ig_compare_result* res) {
    if (!d_x || !d_ref || !res || n < 0) return fail(IG_ERR_INVALID_ARG, "bad argument");
    if (x_dtype < 0 || x_dtype > 2) return fail(IG_ERR_INVALID_ARG, "bad dtype");
    {
        ig_status cb = igk_check_buffer(d_x, (size_t)n * dtype_size(x_dtype), device, "d_x");
        if (cb == IG_OK) cb = igk_check_buffer(d_ref, (size_t)n * sizeof(double), device, "d_ref");
        if (cb != IG_OK) return cb;
    }
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
    {
        ig_status cb = igk_check_buffer(d_x, (size_t)n * dtype_size(x_dtype), device, "d_x");
        if (cb != IG_OK) return cb;
    }
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
