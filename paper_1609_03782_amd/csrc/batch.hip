// Batched filter: many independent FP32 cubes of uneven sizes and parameters,
// captured once per batch signature into one HIP graph and replayed.  See
// ig_filter_batch in include/igfilter.h.
//
// Work items are (cube, pass, piece).  Round r of the graph is one launch of
// k_batch_round over the pieces of pass r of every cube that has one, largest
// cubes first; the kernel boundary between rounds orders the passes, so no
// workgroup ever waits on another.  The graph holds the counter reset (which
// also stamps the start on the GPU's constant-rate clock), the per-cube FP64
// noise-level scan, the staging copies and the rounds; the descriptor tables
// are uploaded once when the plan is built.  The last piece of a cube's last
// pass stamps the clock, giving each cube's completion latency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "internal.h"

using namespace igk;

namespace igk {

struct BatchCube {
    const float* in;
    float* out;
    float* scratch;
    BlockGeom g;
    int V;
    int npieces;       // pieces per pass
    int piece_off;     // first piece in the shared table
    int npass;         // passes
    int stage;         // 1: input copied to scratch first (in place, odd passes); 2: no passes, copy in -> out
    int pad;
    long n;
};

struct BatchItem {
    int cube, pass, piece, depth;
};

constexpr int kCtrDone = 0;   // + cube: pieces of its last pass that are done

// ------------------------------------------------------------ rms pre-pass
struct SumChunk {
    int cube;
    int pad;
    long off, len;
};

__global__ void __launch_bounds__(256)
k_batch_sum(const BatchCube* __restrict__ cubes, const SumChunk* __restrict__ chunks, double* __restrict__ part,
            int from_out) {
    const SumChunk ch = chunks[blockIdx.x];
    const float* x = from_out ? cubes[ch.cube].out : cubes[ch.cube].in;
    double s1 = 0.0, s2 = 0.0, bad = 0.0;
    for (long i = threadIdx.x; i < ch.len; i += 256) {
        const float f = x[ch.off + i];
        if (!isfinite(f)) { bad += 1.0; continue; }
        s1 += (double)f;
        s2 += (double)f * (double)f;
    }
    __shared__ double sh[3][4];
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
        bad += __shfl_xor(bad, o, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sh[0][wid] = s1; sh[1][wid] = s2; sh[2][wid] = bad; }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = ((sh[k][0] + sh[k][1]) + sh[k][2]) + sh[k][3];
}

// One workgroup per cube: fold its chunk partials in order, derive DevParams.
__global__ void __launch_bounds__(64)
k_batch_params(const ParamIn* __restrict__ pin, const int* __restrict__ chunk_first, const double* __restrict__ part,
               const long* __restrict__ nvox, DevParams* __restrict__ out, int sums_only) {
    const int c = blockIdx.x;
    if (threadIdx.x != 0) return;
    double s1 = 0.0, s2 = 0.0, bad = 0.0;
    for (int j = chunk_first[c]; j < chunk_first[c + 1]; ++j) {
        s1 += part[3 * j];
        s2 += part[3 * j + 1];
        bad += part[3 * j + 2];
    }
    if (sums_only) {   // output sums for the statistics: only the sum slot
        out[c].sum = s1;
        return;
    }
    const ParamIn in = pin[c];
    const long n = nvox[c];
    DevParams P;
    P.sum = s1;
    P.sumsq = s2;
    P.nonfinite = (long long)bad;
    P.abort = P.nonfinite > 0 ? 1 : 0;
    P.pad = 0;
    const double rho = in.rms > 0.0 ? in.rms : (n > 0 ? sqrt(s2 / (double)n) : 0.0);
    P.rho = rho;
    const double kr2 = ((double)in.K * rho) * ((double)in.K * rho);
    const double inv = kr2 > 0.0 ? 1.0 / kr2 : 0.0;
    double kap = in.cond == COND_PM_EXP ? -1.4426950408889634 * inv : inv;
    if (!(fabs(kap) <= 3.0e38)) kap = kap < 0 ? -3.0e38 : 3.0e38;
    P.kap = (float)kap;
    P.tau = in.tau;
    for (int a = 0; a < 3; ++a) {
        if (in.cond == COND_PM_EXP) P.coef[a] = (float)log2((double)in.tau * in.C[a]);
        else if (in.cond == COND_PM_RATIONAL) P.coef[a] = (float)((double)in.tau * in.C[a]);
        else P.coef[a] = in.C[a];
    }
    P.closed = in.cond == COND_PM_EXP ? -INFINITY : 0.0f;
    out[c] = P;
}

// Clear the counters and stamps (a kernel, so graph replays start clean) and
// stamp the start of the batch.
__global__ void k_batch_reset(int* __restrict__ ctr, int nctr, unsigned long long* __restrict__ stamps, int nst) {
    for (int i = threadIdx.x; i < nctr; i += blockDim.x) ctr[i] = 0;
    const unsigned long long t0 = wall_clock64();
    for (int i = threadIdx.x; i < nst; i += blockDim.x) stamps[i] = i == 0 ? t0 : 0ULL;
}

// Stage in-place inputs with an odd pass count through scratch (copy), so
// the last pass lands in the output buffer.
__global__ void __launch_bounds__(256)
k_batch_stage(const BatchCube* __restrict__ cubes, const SumChunk* __restrict__ chunks, const DevParams* __restrict__ prm) {
    const SumChunk ch = chunks[blockIdx.x];
    const BatchCube& cb = cubes[ch.cube];
    if (!cb.stage || prm[ch.cube].abort) return;
    float* to = cb.stage == 1 ? cb.scratch : cb.out;
    for (long i = threadIdx.x; i < ch.len; i += 256) to[ch.off + i] = cb.in[ch.off + i];
}

// Batch cubes have nx <= 256, so the automatic layout is 4 voxels per lane
// with 1, 2 or 4 rows per wavefront.
template <int COND, int T, int D>
__device__ __forceinline__ void run_piece_v(const BatchCube& cb, const float* src, float* dst, const Piece pc,
                                            const DevParams& P, float* lds) {
    const bool vec = cb.g.vec;
    switch (cb.g.R) {
        case 4: vec ? stream_piece<COND, float, 4, D, true, 4>(src, dst, cb.g, pc, P, lds)
                    : stream_piece<COND, float, 4, D, false, 4>(src, dst, cb.g, pc, P, lds); break;
        case 2: vec ? stream_piece<COND, float, 4, D, true, 2>(src, dst, cb.g, pc, P, lds)
                    : stream_piece<COND, float, 4, D, false, 2>(src, dst, cb.g, pc, P, lds); break;
        default: vec ? stream_piece<COND, float, 4, D, true, 1>(src, dst, cb.g, pc, P, lds)
                     : stream_piece<COND, float, 4, D, false, 1>(src, dst, cb.g, pc, P, lds); break;
    }
}

// One round: workgroup b runs piece items[b] (one pass of one piece of one cube).
template <int COND, int T>
__global__ void __launch_bounds__(1024)
k_batch_round(const BatchCube* __restrict__ cubes, const BatchItem* __restrict__ items,
              const Piece* __restrict__ pieces, const DevParams* __restrict__ prm, int* __restrict__ ctr,
              unsigned long long* __restrict__ stamps) {
    extern __shared__ float lds[];
    const int tid = threadIdx.y * 64 + threadIdx.x;
    const BatchItem item = items[blockIdx.x];
    const BatchCube& cb = cubes[item.cube];
    const DevParams P = prm[item.cube];
    if (P.abort) return;
    // pass k (1-based) writes out if (npass - k) is even, else scratch
    const int k = item.pass + 1;
    const float* src = item.pass == 0 ? (cb.stage ? cb.scratch : cb.in)
                                      : (((cb.npass - (k - 1)) % 2 == 0) ? cb.out : cb.scratch);
    float* dst = ((cb.npass - k) % 2 == 0) ? cb.out : cb.scratch;
    const Piece pc = pieces[cb.piece_off + item.piece];
    if constexpr (T >= 1) if (item.depth == 1) run_piece_v<COND, T, 1>(cb, src, dst, pc, P, lds);
    if constexpr (T >= 2) if (item.depth == 2) run_piece_v<COND, T, 2>(cb, src, dst, pc, P, lds);
    if constexpr (T >= 3) if (item.depth == 3) run_piece_v<COND, T, 3>(cb, src, dst, pc, P, lds);
    if constexpr (T >= 4) if (item.depth == 4) run_piece_v<COND, T, 4>(cb, src, dst, pc, P, lds);
    if (item.pass == cb.npass - 1) {   // completion stamp of the cube
        __syncthreads();
        if (tid == 0) {
            const int prev = atomicAdd(&ctr[kCtrDone + item.cube], 1);
            if (prev + 1 == cb.npieces) stamps[1 + item.cube] = wall_clock64();
        }
    }
}

using BatchKernel = void (*)(const BatchCube*, const BatchItem*, const Piece*, const DevParams*, int*,
                             unsigned long long*);

template <int COND>
static BatchKernel batch_kernel_T(int T) {
    switch (T) {
        case 1: return k_batch_round<COND, 1>;
        case 2: return k_batch_round<COND, 2>;
        case 3: return k_batch_round<COND, 3>;
        default: return k_batch_round<COND, 4>;
    }
}
static BatchKernel batch_kernel(int cond, int T) {
    switch (cond) {
        case COND_INTENSITY: return batch_kernel_T<COND_INTENSITY>(T);
        case COND_PM_EXP: return batch_kernel_T<COND_PM_EXP>(T);
        default: return batch_kernel_T<COND_PM_RATIONAL>(T);
    }
}

}  // namespace igk

// ====================================================================== host
#define fail igk_fail
#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? IG_ERR_OUT_OF_MEMORY : IG_ERR_DEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                             \
    } while (0)

namespace {

constexpr long kChunk = 1L << 16;   // voxels per rms partial (many workgroups even for small batches)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    ~DevBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t count) {
        n = count;
        return hipMalloc((void**)&p, std::max<size_t>(1, count) * sizeof(T));
    }
};
struct BatchPlan {
    int device = 0;
    int cond = 0, T = 1, W = 16, Z = 32;
    int count = 0;
    std::vector<int> passes;
    DevBuf<float> scratch;
    DevBuf<BatchCube> d_cubes;
    DevBuf<BatchItem> d_items;
    DevBuf<Piece> d_pieces;
    DevBuf<SumChunk> d_chunks;
    DevBuf<int> d_chunk_first;
    DevBuf<double> d_part;
    DevBuf<ParamIn> d_pin;
    DevBuf<long> d_nvox;
    DevBuf<DevParams> d_params;
    DevBuf<DevParams> d_outsum;
    DevBuf<int> d_ctr;
    DevBuf<unsigned long long> d_stamps;
    std::vector<int> round_off;   // items of round r: [round_off[r], round_off[r+1])
    int nitems = 0, nchunks = 0;
    size_t lds = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

std::mutex g_mu;
std::map<std::vector<uint64_t>, std::unique_ptr<BatchPlan>> g_cache;
int g_batch_T = 0;    // 0: default choice
int g_batch_W = 16;
int g_batch_Z = 32;   // planes per z-chunk of a piece

std::vector<uint64_t> signature(const ig_batch_item* items, int count, int device) {
    std::vector<uint64_t> key;
    key.push_back((uint64_t)device);
    key.push_back((uint64_t)g_batch_T);
    key.push_back((uint64_t)g_batch_W);
    key.push_back((uint64_t)g_batch_Z);
    for (int i = 0; i < count; ++i) {
        uint64_t w[(sizeof(ig_params) + 7) / 8] = {};
        std::memcpy(w, &items[i].p, sizeof(ig_params));
        for (uint64_t v : w) key.push_back(v);
        key.push_back((uint64_t)(uintptr_t)items[i].d_in);
        key.push_back((uint64_t)(uintptr_t)items[i].d_out);
    }
    return key;
}

ig_status build_plan(const ig_batch_item* items, int count, int device, BatchPlan* bp) {
    bp->device = device;
    bp->count = count;
    bp->cond = items[0].p.cond;
    int maxn = 0;
    long maxnx = 0;
    for (int i = 0; i < count; ++i) {
        maxn = std::max(maxn, items[i].p.n_iter);
        maxnx = std::max<long>(maxnx, items[i].p.nx);
    }
    bp->W = g_batch_W;
    bp->Z = g_batch_Z;
    bp->T = g_batch_T > 0 ? g_batch_T : std::max(1, std::min(2, maxn));
    const int T = bp->T, W = bp->W;
    if (maxnx > 256) return fail(IG_ERR_UNSUPPORTED, "batch items need nx <= 256");
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);

    // per-cube plans (pieces of ~32 planes), scratch offsets, chunk tables
    std::vector<BatchCube> cubes(count);
    std::vector<Piece> pieces;
    std::vector<SumChunk> chunks;
    std::vector<int> chunk_first(count + 1, 0);
    std::vector<ParamIn> pin(count);
    std::vector<long> nvox(count);
    std::vector<std::vector<int>> depths(count);
    size_t scratch_total = 0;
    std::vector<size_t> scratch_off(count);
    size_t lds = 0;
    for (int c = 0; c < count; ++c) {
        const ig_params& p = items[c].p;
        const long n = (long)(p.nx * p.ny * p.nz);
        nvox[c] = n;
        scratch_off[c] = scratch_total;
        scratch_total += (size_t)((n + 63) / 64 * 64);
        ig_schedule s{};
        s.kind = IG_SCHED_BLOCKED;
        s.t_block = T;
        s.waves = W;
        s.zchunk = g_batch_Z;
        s.vec = 0;
        PassPlan pp;
        const char* why = plan_pass(p, s, T, ncu, &pp);
        if (why) return fail(IG_ERR_INVALID_ARG, "batch item %d: %s", c, why);
        if (pp.V != 4) return fail(IG_ERR_UNSUPPORTED, "batch item %d: layout with %d voxels per lane", c, pp.V);
        lds = std::max(lds, stream_lds_bytes(pp.V, T, W));
        BatchCube& cb = cubes[c];
        cb.in = (const float*)items[c].d_in;
        cb.out = (float*)items[c].d_out;
        cb.g = pp.g;
        if (((uintptr_t)cb.in % (pp.V * 4)) || ((uintptr_t)cb.out % (pp.V * 4))) cb.g.vec = 0;
        cb.V = pp.V;
        cb.npieces = (int)pp.pieces.size();
        cb.piece_off = (int)pieces.size();
        cb.n = n;
        pieces.insert(pieces.end(), pp.pieces.begin(), pp.pieces.end());
        // pass depths (a remainder pass is shallower); in place with an odd count: stage
        std::vector<int>& d = depths[c];
        if (p.n_iter > 0) {
            d.assign(p.n_iter / T, T);
            if (p.n_iter % T) d.push_back(p.n_iter % T);
        }
        cb.npass = (int)d.size();
        cb.stage = (items[c].d_in == items[c].d_out && cb.npass % 2 == 1) ? 1
                   : (cb.npass == 0 && items[c].d_in != items[c].d_out) ? 2 : 0;
        chunk_first[c] = (int)chunks.size();
        for (long off = 0; off < n; off += kChunk) chunks.push_back(SumChunk{c, 0, off, std::min(kChunk, n - off)});
        ParamIn& q = pin[c];
        q.K = p.K; q.tau = p.tau;
        for (int a = 0; a < 3; ++a) q.C[a] = p.C[a];
        q.cond = p.cond;
        q.abort_on_nonfinite = 1;
        q.rms = p.rms;
    }
    chunk_first[count] = (int)chunks.size();
    if (lds > kMaxLds) return fail(IG_ERR_UNSUPPORTED, "batch tile needs too much LDS");
    bp->lds = lds;
    bp->passes.resize(count);
    for (int c = 0; c < count; ++c) bp->passes[c] = cubes[c].npass;

    // rounds: round r holds pass r of every cube that has one, largest cubes first
    std::vector<int> order(count);
    for (int c = 0; c < count; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nvox[a] > nvox[b]; });
    int maxpass = 0;
    for (int c = 0; c < count; ++c) maxpass = std::max(maxpass, cubes[c].npass);
    std::vector<BatchItem> its;
    bp->round_off.assign(1, 0);
    for (int k = 0; k < maxpass; ++k) {
        for (int c : order)
            if (k < cubes[c].npass)
                for (int j = 0; j < cubes[c].npieces; ++j) its.push_back(BatchItem{c, k, j, depths[c][k]});
        bp->round_off.push_back((int)its.size());
    }
    bp->nitems = (int)its.size();
    bp->nchunks = (int)chunks.size();

    HIP_TRY(bp->scratch.alloc(scratch_total));
    for (int c = 0; c < count; ++c) cubes[c].scratch = bp->scratch.p + scratch_off[c];
    HIP_TRY(bp->d_cubes.alloc(count));
    HIP_TRY(bp->d_items.alloc(its.size()));
    HIP_TRY(bp->d_pieces.alloc(pieces.size()));
    HIP_TRY(bp->d_chunks.alloc(chunks.size()));
    HIP_TRY(bp->d_chunk_first.alloc(count + 1));
    HIP_TRY(bp->d_part.alloc(3 * chunks.size()));
    HIP_TRY(bp->d_pin.alloc(count));
    HIP_TRY(bp->d_nvox.alloc(count));
    HIP_TRY(bp->d_params.alloc(count));
    HIP_TRY(bp->d_outsum.alloc(count));
    HIP_TRY(bp->d_ctr.alloc(kCtrDone + count));
    HIP_TRY(bp->d_stamps.alloc(1 + count));
    // descriptor tables: fixed for the plan's signature, uploaded once
    HIP_TRY(hipMemcpy(bp->d_cubes.p, cubes.data(), count * sizeof(BatchCube), hipMemcpyHostToDevice));
    if (!its.empty())
        HIP_TRY(hipMemcpy(bp->d_items.p, its.data(), its.size() * sizeof(BatchItem), hipMemcpyHostToDevice));
    if (!pieces.empty())
        HIP_TRY(hipMemcpy(bp->d_pieces.p, pieces.data(), pieces.size() * sizeof(Piece), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bp->d_chunks.p, chunks.data(), chunks.size() * sizeof(SumChunk), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bp->d_chunk_first.p, chunk_first.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bp->d_pin.p, pin.data(), count * sizeof(ParamIn), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bp->d_nvox.p, nvox.data(), count * sizeof(long), hipMemcpyHostToDevice));

    BatchKernel kern = batch_kernel(bp->cond, T);
    if (lds > 65536)
        HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));

    // capture: counter reset, noise-level pre-pass, staging, the rounds
    HIP_TRY(hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal));
    hipStream_t s = bp->cap;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, s, bp->d_ctr.p, kCtrDone + count, bp->d_stamps.p,
                       1 + count);
    chk(hipGetLastError());
    if (bp->nchunks > 0) {
        hipLaunchKernelGGL(k_batch_sum, dim3(bp->nchunks), dim3(256), 0, s, bp->d_cubes.p, bp->d_chunks.p,
                           bp->d_part.p, 0);
        chk(hipGetLastError());
    }
    hipLaunchKernelGGL(k_batch_params, dim3(count), dim3(64), 0, s, bp->d_pin.p, bp->d_chunk_first.p,
                       bp->d_part.p, bp->d_nvox.p, bp->d_params.p, 0);
    chk(hipGetLastError());
    if (bp->nchunks > 0) {
        hipLaunchKernelGGL(k_batch_stage, dim3(bp->nchunks), dim3(256), 0, s, bp->d_cubes.p, bp->d_chunks.p,
                           bp->d_params.p);
        chk(hipGetLastError());
    }
    for (size_t r = 0; r + 1 < bp->round_off.size(); ++r) {
        const int n = bp->round_off[r + 1] - bp->round_off[r];
        if (n <= 0) continue;
        hipLaunchKernelGGL(kern, dim3(n), dim3(64, W), lds, s, bp->d_cubes.p, bp->d_items.p + bp->round_off[r],
                           bp->d_pieces.p, bp->d_params.p, bp->d_ctr.p, bp->d_stamps.p);
        chk(hipGetLastError());
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return fail(IG_ERR_DEVICE, "capture: %s", hipGetErrorString(e)); }
    HIP_TRY(e2);
    bp->graph = g;
    HIP_TRY(hipGraphInstantiate(&bp->exec, g, nullptr, nullptr, 0));
    return IG_OK;
}

}  // namespace

extern "C" ig_status ig_filter_batch(const ig_batch_item* items, int32_t count, int device, void* hip_stream,
                                     ig_stats* per_item, double* latency_ms) {
    if (!items || count < 1) return fail(IG_ERR_INVALID_ARG, "empty batch");
    for (int i = 0; i < count; ++i) {
        ig_status st = igk_validate_params(&items[i].p);
        if (st != IG_OK) return st;
        if (items[i].p.dtype != IG_F32) return fail(IG_ERR_UNSUPPORTED, "batch item %d: only FP32 storage", i);
        if (items[i].p.cond != items[0].p.cond)
            return fail(IG_ERR_UNSUPPORTED, "batch items must share one conductance");
        if (!items[i].d_in || !items[i].d_out) return fail(IG_ERR_INVALID_ARG, "batch item %d: NULL buffer", i);
        if (per_item && per_item[i].struct_size != sizeof(ig_stats))
            return fail(IG_ERR_INVALID_ARG, "per_item[%d].struct_size", i);
    }
    // buffers of distinct items must not overlap
    {
        std::vector<std::pair<uintptr_t, uintptr_t>> rng;
        for (int i = 0; i < count; ++i) {
            const size_t bytes = (size_t)(items[i].p.nx * items[i].p.ny * items[i].p.nz) * 4;
            const uintptr_t a = (uintptr_t)items[i].d_in, b = (uintptr_t)items[i].d_out;
            if (a != b && a < b + bytes && b < a + bytes)
                return fail(IG_ERR_INVALID_ARG, "batch item %d: input and output overlap partially", i);
            rng.push_back({a, a + bytes});
            if (b != a) rng.push_back({b, b + bytes});
        }
        std::sort(rng.begin(), rng.end());
        for (size_t k = 1; k < rng.size(); ++k)
            if (rng[k].first < rng[k - 1].second) return fail(IG_ERR_INVALID_ARG, "batch items share buffers");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(IG_ERR_INVALID_ARG, "bad device %d", device);
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return fail(IG_ERR_DEVICE, "hipSetDevice(%d)", device);
    struct Restore { int d; ~Restore() { if (d >= 0) (void)hipSetDevice(d); } } restore{prev};

    std::lock_guard<std::mutex> lk(g_mu);
    auto key = signature(items, count, device);
    auto it = g_cache.find(key);
    BatchPlan* bp;
    if (it == g_cache.end()) {
        auto plan = std::make_unique<BatchPlan>();
        ig_status st = build_plan(items, count, device, plan.get());
        if (st != IG_OK) return st;
        bp = plan.get();
        g_cache[key] = std::move(plan);
    } else {
        bp = it->second.get();
    }
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(hipGraphLaunch(bp->exec, s));
    if (!per_item && !latency_ms) return IG_OK;

    std::vector<unsigned long long> stamps(1 + count);
    HIP_TRY(hipMemcpyAsync(stamps.data(), bp->d_stamps.p, stamps.size() * 8, hipMemcpyDeviceToHost, s));
    std::vector<DevParams> prm(count);
    HIP_TRY(hipMemcpyAsync(prm.data(), bp->d_params.p, count * sizeof(DevParams), hipMemcpyDeviceToHost, s));
    if (per_item) {
        hipLaunchKernelGGL(k_batch_sum, dim3(bp->nchunks), dim3(256), 0, s, bp->d_cubes.p, bp->d_chunks.p,
                           bp->d_part.p, 1);
        hipLaunchKernelGGL(k_batch_params, dim3(count), dim3(64), 0, s, bp->d_pin.p, bp->d_chunk_first.p,
                           bp->d_part.p, bp->d_nvox.p, bp->d_outsum.p, 1);
        HIP_TRY(hipGetLastError());
    }
    std::vector<DevParams> osum(count);
    if (per_item)
        HIP_TRY(hipMemcpyAsync(osum.data(), bp->d_outsum.p, count * sizeof(DevParams), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int khz = 0;
    (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
    bool bad = false;
    for (int c = 0; c < count; ++c) {
        if (latency_ms)
            latency_ms[c] = (khz > 0 && stamps[1 + c] >= stamps[0]) ? (double)(stamps[1 + c] - stamps[0]) / khz : 0.0;
        if (per_item) {
            ig_stats& st = per_item[c];
            const ig_params& p = items[c].p;
            st.passes = bp->passes[c];
            st.rms_used = prm[c].rho;
            st.sum_in = prm[c].sum;
            st.sum_out = osum[c].sum;
            st.nonfinite = prm[c].nonfinite;
            st.monotone = (2.0 * (double)p.tau * ((double)p.C[0] + p.C[1] + p.C[2]) <= 1.0) ? 1 : 0;
            st.schedule = ig_schedule{IG_SCHED_BLOCKED, bp->T, bp->W, bp->Z, 4, 0, 0};
        }
        if (prm[c].abort) bad = true;
    }
    if (bad) return fail(IG_ERR_NONFINITE, "a batch item holds non-finite voxels (left untouched)");
    return IG_OK;
}

extern "C" void ig_batch_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
}

extern "C" ig_status ig_batch_autotune(const ig_batch_item* items, int32_t count, int device, void* hip_stream,
                                       int32_t* best_t_block, int32_t* best_waves, int32_t* best_zchunk,
                                       double* best_ms) {
    if (!items || count < 1) return fail(IG_ERR_INVALID_ARG, "empty batch");
    for (int i = 0; i < count; ++i)
        if (items[i].d_in == items[i].d_out) return fail(IG_ERR_INVALID_ARG, "autotuning needs d_in != d_out");
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int maxn = 0;
    for (int i = 0; i < count; ++i) maxn = std::max(maxn, items[i].p.n_iter);
    // drop the plan of a candidate that is not kept (each plan holds scratch
    // cubes for the whole batch)
    auto drop = [&](int T, int W, int Z) {
        std::lock_guard<std::mutex> lk(g_mu);
        const int t0 = g_batch_T, w0 = g_batch_W, z0 = g_batch_Z;
        g_batch_T = T; g_batch_W = W; g_batch_Z = Z;
        g_cache.erase(signature(items, count, device));
        g_batch_T = t0; g_batch_W = w0; g_batch_Z = z0;
    };
    double best = 1e300;
    int bT = 0, bW = 16, bZ = 32;
    for (int T = 1; T <= std::max(1, std::min(4, maxn)); ++T)
        for (int W : {8, 12, 16})
            for (int Z : {32, 64}) {
                if (W <= 2 * T) continue;
                if (ig_batch_set_schedule(T, W, Z) != IG_OK) continue;
                if (ig_filter_batch(items, count, device, hip_stream, nullptr, nullptr) != IG_OK) {   // build + warm
                    drop(T, W, Z);
                    continue;
                }
                float ms = 0.0f;
                bool ok = hipEventRecord(e0, s) == hipSuccess;
                for (int k = 0; k < 2 && ok; ++k)
                    ok = ig_filter_batch(items, count, device, hip_stream, nullptr, nullptr) == IG_OK;
                ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (ok && ms / 2 < best) {
                    if (best < 1e300) drop(bT, bW, bZ);
                    best = ms / 2; bT = T; bW = W; bZ = Z;
                } else {
                    drop(T, W, Z);
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best >= 1e300) return fail(IG_ERR_UNSUPPORTED, "no batch schedule ran");
    ig_status st = ig_batch_set_schedule(bT, bW, bZ);
    if (st != IG_OK) return st;
    if (best_t_block) *best_t_block = bT;
    if (best_waves) *best_waves = bW;
    if (best_zchunk) *best_zchunk = bZ;
    if (best_ms) *best_ms = best;
    return IG_OK;
}

extern "C" ig_status ig_batch_set_schedule(int32_t t_block, int32_t waves, int32_t zchunk) {
    if (t_block < 0 || t_block > 4 || waves < 1 || waves > 16 || zchunk < 1 || zchunk > 4096)
        return fail(IG_ERR_INVALID_ARG, "bad batch schedule");
    std::lock_guard<std::mutex> lk(g_mu);
    g_batch_T = t_block;
    g_batch_W = waves;
    g_batch_Z = zchunk;
    return IG_OK;
}
