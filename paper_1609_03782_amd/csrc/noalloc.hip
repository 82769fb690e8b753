// ig_filter_run_static: the filter of ig_filter_run for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).  See include/igfilter.h.
//
// Everything a run needs besides the caller's input and output lives in one
// file-scope device array, `scratch`, carved into: the run's constants, the
// FP64 reduction partials, one piece table per pass depth, and the ping-pong
// cube (at most kStaticCubeBytes).  Each GPU holds its own copy of the array
// from the library's load to the end of the process; its address on a device
// is read once with hipGetSymbolAddress (the array's name in host code is only
// a stand-in for the symbol) and cached per device.  Piece tables are written
// by a kernel from the regular (x tile, y tile, z chunk) grid, so the call
// issues no host-to-device copy either.  Calls that overlap on one GPU share
// the array and race; every part of it a run reads is written by that run
// first, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "igfilter.h"
#include "internal.h"

using namespace igk;

namespace {

constexpr size_t kStaticCubeBytes = (size_t)IG_STATIC_MAX_CUBE_BYTES;
constexpr int kStaticMaxPieces = 16384;   // per pass depth 1..4
constexpr size_t kOffParams = 0;
constexpr size_t kOffResults = 256;
constexpr size_t kOffParts = 512;
constexpr size_t kOffPieces = kOffParts + (((size_t)kPartBlocks * 6 * sizeof(double) + 255) / 256) * 256;
constexpr size_t kOffCube = kOffPieces + (size_t)4 * kStaticMaxPieces * sizeof(Piece);
constexpr size_t kScratchBytes = kOffCube + kStaticCubeBytes;
static_assert(sizeof(DevParams) <= 256 && 8 * sizeof(double) <= 256, "header slots too small");
static_assert(kOffCube % 256 == 0, "cube region must stay 256-byte aligned");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // scratch's device address, per device (null: not read yet)

#define fail igk_fail

ig_status scratch_ptr(int device, unsigned char** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(IG_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
        g_ptr[device] = p;
    }
    *out = static_cast<unsigned char*>(g_ptr[device]);
    return IG_OK;
}

// Piece b of the regular grid, in the planner's order (z chunk, then y tile,
// then x tile): outputs in planes [tz*zchunk, min(nz, (tz+1)*zchunk)).
__global__ void __launch_bounds__(256)
k_grid_pieces(Piece* __restrict__ out, int count, int ntx, int nty, int zchunk, int nz) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= count) return;
    const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
    out[b] = Piece{tx, ty, tz * zchunk, min(nz, (tz + 1) * zchunk)};
}

// The static run's plans: the host geometry per depth, the table on the device.
struct StaticPlans {
    const ig_params* p;
    int ncu;
    Piece* dev_base;          // kStaticMaxPieces pieces per depth
    hipStream_t stream;
    PassPlan plans[5];
    bool planned[5] = {false, false, false, false, false};
};

ig_status static_plan(void* self, const ig_schedule& sched, int T, const PassPlan** out, const Piece** dev) {
    StaticPlans& sp = *static_cast<StaticPlans*>(self);
    if (T < 1 || T > 4) return fail(IG_ERR_INVALID_ARG, "pass depth %d", T);
    Piece* d = sp.dev_base + (size_t)(T - 1) * kStaticMaxPieces;
    if (!sp.planned[T]) {
        PassPlan& pp = sp.plans[T];
        const char* why = plan_pass(*sp.p, sched, T, sp.ncu, &pp);
        if (why) return fail(IG_ERR_INVALID_ARG, "schedule cannot serve this shape: %s", why);
        const int count = (int)pp.pieces.size();
        if (count > kStaticMaxPieces) return fail(IG_ERR_UNSUPPORTED, "%d pieces exceed the static table", count);
        const int nzc = (sp.p->nz + sched.zchunk - 1) / sched.zchunk;
        if (count != pp.g.ntx * pp.g.nty * nzc) return fail(IG_ERR_DEVICE, "piece grid mismatch");
        hipLaunchKernelGGL(k_grid_pieces, dim3((count + 255) / 256), dim3(256), 0, sp.stream, d, count, pp.g.ntx,
                           pp.g.nty, sched.zchunk, (int)sp.p->nz);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(IG_ERR_DEVICE, "piece table kernel: %s", hipGetErrorString(e));
        sp.planned[T] = true;
    }
    *out = &sp.plans[T];
    *dev = d;
    return IG_OK;
}

// The library's automatic layout, with z chunks sized so that the pieces of
// one pass fill one round of the resident workgroups; the naive schedule
// when the regular grid would not fit the static table.
ig_schedule static_schedule(const ig_params& p, int ncu) {
    ig_schedule s = igk_auto_schedule(&p);
    if (s.kind != IG_SCHED_BLOCKED) return s;
    // the 16-wave layout pays only through a grouped plan (equal shares of
    // the tiles' planes), which the regular grid of the static tables is not
    if (s.waves == 16 && s.t_block == 2 && s.vec == 8 && s.rows == 1) s.waves = 12;
    s.rounds = 0;
    s.zchunk = (int)p.nz;
    PassPlan pp;
    if (plan_pass(p, s, s.t_block, ncu, &pp)) {
        ig_schedule n{};
        n.kind = IG_SCHED_NAIVE;
        return n;
    }
    const long tiles = (long)pp.g.ntx * pp.g.nty;
    const long slots = (long)ncu * resident_per_cu(s.waves, stream_lds_bytes(pp.V, s.t_block, s.waves));
    const long per_tile = std::max<long>(1, slots / std::max<long>(1, tiles));
    s.zchunk = (int)std::max<long>(1, (p.nz + per_tile - 1) / per_tile);
    const long nzc = (p.nz + s.zchunk - 1) / s.zchunk;
    if (tiles * nzc > kStaticMaxPieces) {
        ig_schedule n{};
        n.kind = IG_SCHED_NAIVE;
        return n;
    }
    return s;
}

bool overlap(const void* a, const void* b, size_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

}  // namespace

extern "C" ig_status ig_filter_run_static(const ig_params* p, int device, const void* d_in, void* d_out,
                                          void* hip_stream, ig_stats* stats) {
    ig_status st = igk_validate_params(p);
    if (st != IG_OK) return st;
    if (!d_in || !d_out) return fail(IG_ERR_INVALID_ARG, "NULL buffer");
    if (stats && stats->struct_size != sizeof(ig_stats))
        return fail(IG_ERR_INVALID_ARG, "stats.struct_size %u != %zu", stats->struct_size, sizeof(ig_stats));
    const size_t bytes = (size_t)(p->nx * p->ny * p->nz) * dtype_size(p->dtype);
    if (bytes > kStaticCubeBytes)
        return fail(IG_ERR_INVALID_ARG, "cube of %zu bytes exceeds the static workspace (%zu bytes)", bytes,
                    kStaticCubeBytes);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(IG_ERR_DEVICE, "no HIP device");
    if (device < 0 || device >= ndev || device >= kMaxDevices)
        return fail(IG_ERR_INVALID_ARG, "device %d of %d", device, ndev);
    if (d_in != d_out && overlap(d_in, d_out, bytes)) return fail(IG_ERR_INVALID_ARG, "input and output overlap partially");
    if (((uintptr_t)d_in % dtype_size(p->dtype)) || ((uintptr_t)d_out % dtype_size(p->dtype)))
        return fail(IG_ERR_INVALID_ARG, "buffers must be aligned to the element size");
    ig_status cb = igk_check_buffer(d_in, bytes, device, "d_in");
    if (cb == IG_OK) cb = igk_check_buffer(d_out, bytes, device, "d_out");
    if (cb != IG_OK) return cb;

    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice(%d) failed", device);
    struct Restore { int d; ~Restore() { if (d >= 0) (void)hipSetDevice(d); } } restore{prev};

    unsigned char* base = nullptr;
    st = scratch_ptr(device, &base);
    if (st != IG_OK) return st;
    void* cube = base + kOffCube;
    if (overlap(d_in, cube, bytes) || overlap(d_out, cube, bytes))
        return fail(IG_ERR_INVALID_ARG, "buffer overlaps the static workspace");
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1)
        ncu = 256;
    hipStream_t s = (hipStream_t)hip_stream;
    const ig_schedule sched = static_schedule(*p, ncu);
    StaticPlans plans{p, ncu, reinterpret_cast<Piece*>(base + kOffPieces), s};
    RunCtx c{p,
             cube,
             reinterpret_cast<DevParams*>(base + kOffParams),
             reinterpret_cast<double*>(base + kOffParts),
             reinterpret_cast<double*>(base + kOffResults),
             static_plan,
             &plans,
             nullptr,
             nullptr};
    const bool scan = p->rms <= 0.0 || stats != nullptr;
    int passes = 0;
    st = igk_enqueue_run(c, sched, d_in, d_out, scan, s, &passes);
    if (st != IG_OK) return st;
    if (!stats) return IG_OK;
    return igk_finish_stats(c, sched, passes, d_out, s, stats);
}

extern "C" int64_t ig_filter_static_max_bytes(void) { return (int64_t)kStaticCubeBytes; }
