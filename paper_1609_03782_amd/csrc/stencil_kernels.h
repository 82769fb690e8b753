// Filter-step kernels for gfx950 (wave64).
//
//  k_naive   one step per launch, one voxel per thread, neighbours straight
//            from global memory.  The reference schedule.
//  k_stream  T steps per launch.  A workgroup owns an xy tile (halo of T
//            voxels where it borders another tile) and a range of z-planes;
//            it streams the planes in z order, keeping every intermediate
//            step of the pass on chip:
//              lane      -> V consecutive x voxels (two 16-byte loads for
//                           V = 8 in FP32, one in 16-bit storage);
//              wavefront -> one row; x neighbours cross lanes by DPP wave
//                           shifts, so an x edge term is computed once;
//              workgroup -> W wavefronts stacked in y, rows shared in LDS;
//              z         -> each level keeps its current plane, the plane
//                           above and the edge term to the plane below in
//                           registers, so a z edge term is computed once.
//            Level t of a pass turns plane p of level t-1 into plane p of
//            level t as soon as plane p+1 of level t-1 exists; the last level
//            is written to global memory.  Rows, columns and planes that a
//            level cannot compute correctly (they would need data outside
//            the tile) are halo; the tile's outputs never depend on them.
//
// Both kernels use edge_term/combine from stencil_common.h in the same order,
// so their results are bitwise identical.
#pragma once
#include <type_traits>

#include "plan.h"
#include "stencil_common.h"

namespace igk {

struct NaiveGeom {
    int nx, ny, nz;
};



__device__ __forceinline__ float lane_shr1(float v) {  // lane i <- lane i-1, lane 0 <- 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_shl1(float v) {  // lane i <- lane i+1, lane 63 <- 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

// ------------------------------------------------------------------ naive
template <int COND, typename ST>
__global__ void __launch_bounds__(256)
k_naive(const ST* __restrict__ src, ST* __restrict__ dst, NaiveGeom g,
        const DevParams* __restrict__ dp) {
    const DevParams P = *dp;
    if (P.abort) return;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const long sy = g.nx, sz = (long)g.nx * g.ny;
    const long v = x + y * sy + z * sz;
    const float I = Store<ST>::load(src[v]);
    auto at = [&](long o) { return Store<ST>::load(src[v + o]); };
    // minus-side edge of v is the plus-side edge of the neighbour: d = I(v) - I(v - e)
    const float exm = edge_term<COND>(x > 0 ? I - at(-1) : 0.0f, x > 0 ? P.coef[0] : P.closed, P.kap);
    const float exp_ = edge_term<COND>(x + 1 < g.nx ? at(1) - I : 0.0f,
                                       x + 1 < g.nx ? P.coef[0] : P.closed, P.kap);
    const float eym = edge_term<COND>(y > 0 ? I - at(-sy) : 0.0f, y > 0 ? P.coef[1] : P.closed, P.kap);
    const float eyp = edge_term<COND>(y + 1 < g.ny ? at(sy) - I : 0.0f,
                                      y + 1 < g.ny ? P.coef[1] : P.closed, P.kap);
    const float ezm = edge_term<COND>(z > 0 ? I - at(-sz) : 0.0f, z > 0 ? P.coef[2] : P.closed, P.kap);
    const float ezp = edge_term<COND>(z + 1 < g.nz ? at(sz) - I : 0.0f,
                                      z + 1 < g.nz ? P.coef[2] : P.closed, P.kap);
    const float o = combine<COND>(I, exm, exp_, eym, eyp, ezm, ezp, P.kap, P.tau);
    dst[v] = Store<ST>::store(o);
}

// ------------------------------------------------------------ vector I/O
template <typename ST, int V> struct Vec;
template <int V> struct Vec<float, V> {
    static __device__ __forceinline__ void load(const float* p, float (&o)[V]) {
        if constexpr (V % 4 == 0) {
#pragma unroll
            for (int k = 0; k < V / 4; ++k) {
                const float4 q = reinterpret_cast<const float4*>(p)[k];
                o[4 * k] = q.x; o[4 * k + 1] = q.y; o[4 * k + 2] = q.z; o[4 * k + 3] = q.w;
            }
        } else if constexpr (V == 2) {
            const float2 q = *reinterpret_cast<const float2*>(p);
            o[0] = q.x; o[1] = q.y;
        } else {
            o[0] = p[0];
        }
    }
    static __device__ __forceinline__ void store(float* p, const float (&v)[V]) {
        if constexpr (V % 4 == 0) {
#pragma unroll
            for (int k = 0; k < V / 4; ++k)
                reinterpret_cast<float4*>(p)[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
        } else if constexpr (V == 2) {
            *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
        } else {
            p[0] = v[0];
        }
    }
};
// 16-bit storage: V halfwords, moved as one integer vector
template <typename ST, int V> struct Vec16 {
    using U = unsigned short;
    static __device__ __forceinline__ void load(const ST* p, float (&o)[V]) {
        U u[V];
        if constexpr (V == 8) {
            const uint4 q = *reinterpret_cast<const uint4*>(p);
            const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) { u[2 * k] = w[k] & 0xFFFF; u[2 * k + 1] = w[k] >> 16; }
        } else if constexpr (V == 4) {
            const uint2 q = *reinterpret_cast<const uint2*>(p);
            u[0] = q.x & 0xFFFF; u[1] = q.x >> 16; u[2] = q.y & 0xFFFF; u[3] = q.y >> 16;
        } else if constexpr (V == 2) {
            const unsigned q = *reinterpret_cast<const unsigned*>(p);
            u[0] = q & 0xFFFF; u[1] = q >> 16;
        } else {
            u[0] = *reinterpret_cast<const U*>(p);
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            ST s;
            __builtin_memcpy(&s, &u[i], 2);
            o[i] = Store<ST>::load(s);
        }
    }
    static __device__ __forceinline__ void store(ST* p, const float (&v)[V]) {
        U u[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const ST s = Store<ST>::store(v[i]);
            __builtin_memcpy(&u[i], &s, 2);
        }
        if constexpr (V == 8) {
            *reinterpret_cast<uint4*>(p) = make_uint4(u[0] | (unsigned)u[1] << 16, u[2] | (unsigned)u[3] << 16,
                                                      u[4] | (unsigned)u[5] << 16, u[6] | (unsigned)u[7] << 16);
        } else if constexpr (V == 4) {
            *reinterpret_cast<uint2*>(p) = make_uint2(u[0] | (unsigned)u[1] << 16, u[2] | (unsigned)u[3] << 16);
        } else if constexpr (V == 2) {
            *reinterpret_cast<unsigned*>(p) = u[0] | (unsigned)u[1] << 16;
        } else {
            *reinterpret_cast<U*>(p) = u[0];
        }
    }
};
template <int V> struct Vec<__hip_bfloat16, V> : Vec16<__hip_bfloat16, V> {};
template <int V> struct Vec<__half, V> : Vec16<__half, V> {};

// V consecutive values at an address aligned only to the element: rows of a
// cube whose nx is not a multiple of V start anywhere.  The types carry the
// element's alignment, so the compiler emits wide accesses only where the
// target allows unaligned ones and splits them otherwise.
template <typename ST, int V> struct VecU;
template <int V> struct VecU<float, V> {
    typedef float vt __attribute__((ext_vector_type(V), aligned(4)));
    static __device__ __forceinline__ void load(const float* p, float (&o)[V]) {
        const vt q = *reinterpret_cast<const vt*>(p);
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = q[i];
    }
    static __device__ __forceinline__ void store(float* p, const float (&v)[V]) {
        vt q;
#pragma unroll
        for (int i = 0; i < V; ++i) q[i] = v[i];
        *reinterpret_cast<vt*>(p) = q;
    }
};
template <typename ST, int V> struct VecU16 {
    typedef unsigned short vt __attribute__((ext_vector_type(V), aligned(2)));
    static __device__ __forceinline__ void load(const ST* p, float (&o)[V]) {
        const vt q = *reinterpret_cast<const vt*>(p);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const unsigned short u = q[i];
            ST h;
            __builtin_memcpy(&h, &u, 2);
            o[i] = Store<ST>::load(h);
        }
    }
    static __device__ __forceinline__ void store(ST* p, const float (&v)[V]) {
        vt q;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const ST h = Store<ST>::store(v[i]);
            unsigned short u;
            __builtin_memcpy(&u, &h, 2);
            q[i] = u;
        }
        *reinterpret_cast<vt*>(p) = q;
    }
};
template <int V> struct VecU<__hip_bfloat16, V> : VecU16<__hip_bfloat16, V> {};
template <int V> struct VecU<__half, V> : VecU16<__half, V> {};

// o[i] = q[clamp(i + sh, 0, V - 1)]: a lane's loaded chunk moved to where its
// voxels are, the row's end value repeated past it.  sh < 0 only occurs for a
// chunk wholly left of the cube (tiles start at multiples of V), whose voxels
// all take the row's first value, q[0].  log2 V select stages.
template <int V>
__device__ __forceinline__ void shift_clamp(const float (&q)[V], int sh, float (&o)[V]) {
    float t[V];
#pragma unroll
    for (int i = 0; i < V; ++i) t[i] = q[i];
    const int s = sh < 0 ? 0 : (sh > V - 1 ? V - 1 : sh);
#pragma unroll
    for (int b = 1; b < V; b <<= 1) {
        const bool on = (s & b) != 0;
        float u[V];
#pragma unroll
        for (int i = 0; i < V; ++i) u[i] = t[i + b < V ? i + b : V - 1];
#pragma unroll
        for (int i = 0; i < V; ++i) t[i] = on ? u[i] : t[i];
    }
#pragma unroll
    for (int i = 0; i < V; ++i) o[i] = sh < 0 ? q[0] : t[i];
}

// Raw buffer access for the 16-bit storage types.  The hardware drops an
// access at or past the buffer's byte size (a load returns zeros), so an
// access that must not happen can still be issued: give the buffer size 0, or
// the lane an offset past the end.  Word 3 of the gfx9 buffer descriptor:
// 32-bit data format, no swizzle, no index stride.
constexpr int kBufWord3 = 0x00020000;
constexpr int kBufOffNone = 0x40000000;   // past the end of every buffer made here
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <typename ST, int V> struct BufRow16 {
    static_assert(sizeof(ST) == 2, "16-bit storage only");
    static constexpr int NW = V / 2;   // 32-bit words of a lane's V values (V >= 2)
    static __device__ __forceinline__ float val(unsigned short u) {
        ST h;
        __builtin_memcpy(&h, &u, 2);
        return Store<ST>::load(h);
    }
    static __device__ __forceinline__ unsigned short bits(float v) {
        const ST h = Store<ST>::store(v);
        unsigned short u;
        __builtin_memcpy(&u, &h, 2);
        return u;
    }
    // V values from byte offset off of buffer r (zeros past its end)
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, int off, float (&o)[V]) {
        if constexpr (V == 1) {
            o[0] = val(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
        } else {
            unsigned wd[NW];
            if constexpr (NW == 4) {
                const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
                wd[0] = q.x; wd[1] = q.y; wd[2] = q.z; wd[3] = q.w;
            } else if constexpr (NW == 2) {
                const u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
                wd[0] = q.x; wd[1] = q.y;
            } else {
                wd[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                o[2 * k] = val(wd[k] & 0xFFFF);
                o[2 * k + 1] = val(wd[k] >> 16);
            }
        }
    }
    // V values to byte offset off of buffer r (dropped past its end)
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, int off, const float (&v)[V]) {
        if constexpr (V == 1) {
            __builtin_amdgcn_raw_buffer_store_b16(bits(v[0]), r, off, 0, 0);
        } else {
            unsigned wd[NW];
#pragma unroll
            for (int k = 0; k < NW; ++k) wd[k] = bits(v[2 * k]) | (unsigned)bits(v[2 * k + 1]) << 16;
            if constexpr (NW == 4) {
                __builtin_amdgcn_raw_buffer_store_b128(u32x4{wd[0], wd[1], wd[2], wd[3]}, r, off, 0, 0);
            } else if constexpr (NW == 2) {
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{wd[0], wd[1]}, r, off, 0, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b32(wd[0], r, off, 0, 0);
            }
        }
    }
};

// FP32 scalar path, branch-free output: a lane whose chunk lies wholly in the
// output range stores it whole at byte offset `full` (else kBufOffNone); the
// lane at the row's end stores its first k values (k < V) as chunks of 4, 2
// and 1 chosen by the bits of k, at byte offset `tail` (else kBufOffNone).
// Every lane issues the same stores; the hardware drops those past the end.
template <int V>
__device__ __forceinline__ void store_row_f32(__amdgpu_buffer_rsrc_t r, int full, int tail, int k,
                                              const float (&v)[V]) {
    typedef unsigned u32x4_ __attribute__((ext_vector_type(4)));
    typedef unsigned u32x2_ __attribute__((ext_vector_type(2)));
    unsigned w[V];
#pragma unroll
    for (int i = 0; i < V; ++i) w[i] = __builtin_bit_cast(unsigned, v[i]);
    if constexpr (V >= 4) {
#pragma unroll
        for (int c = 0; c < V / 4; ++c)
            __builtin_amdgcn_raw_buffer_store_b128(u32x4_{w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3]}, r,
                                                   full == kBufOffNone ? kBufOffNone : full + 16 * c, 0, 0);
    } else if constexpr (V == 2) {
        __builtin_amdgcn_raw_buffer_store_b64(u32x2_{w[0], w[1]}, r, full, 0, 0);
    }
    if constexpr (V >= 2) {
        // chunk of 4 at element 0 (V = 8 only: k < 8), of 2 at element k & 4,
        // of 1 at element k & 6
        if constexpr (V == 8)
            __builtin_amdgcn_raw_buffer_store_b128(u32x4_{w[0], w[1], w[2], w[3]}, r,
                                                   (k & 4) ? tail : kBufOffNone, 0, 0);
        if constexpr (V >= 4) {
            const bool hi = (k & 4) != 0;
            __builtin_amdgcn_raw_buffer_store_b64(u32x2_{hi ? w[4 % V] : w[0], hi ? w[5 % V] : w[1]}, r,
                                                  (k & 2) ? tail + 4 * (k & 4) : kBufOffNone, 0, 0);
        }
        const int e = k & 6;
        unsigned x1 = w[0];
#pragma unroll
        for (int i = 2; i < V; i += 2) x1 = e == i ? w[i] : x1;
        __builtin_amdgcn_raw_buffer_store_b32(x1, r, (k & 1) ? tail + 4 * e : kBufOffNone, 0, 0);
    }
}

// ---------------------------------------------------------------- streaming
// One workgroup = W wavefronts = W*R consecutive rows of a tile; R rows per
// wavefront (64/R lanes per row, used for narrow cubes: R > 1 needs one x
// tile), V voxels per lane (a row spans 64/R*V voxels).  Work comes from a
// host-built piece table: piece b is (x tile, y tile, z0, z1) with outputs in
// planes [z0, z1).  Per step s the workgroup takes the input plane loaded one
// step earlier, issues the load of the next one, and advances every level by
// one plane: level L turns plane p of level L-1 into plane p of level L from
// its own row (x edges inside the lane and via DPP across lanes), the rows
// above and below at level L (y edges, through LDS) and the planes above and
// below (z edges, registers; the edge to the plane below is the one computed
// one step earlier).  Two ways to share the y edges:
//
//  edge-shared (exponential and rational conductances, where an edge term
//  costs an exponential or a reciprocal): each level's new row is published
//  to LDS (barrier), each wavefront computes the edge term to the row above
//  and publishes it (barrier); every y edge term is evaluated once.
//
//  row-shared (intensity conductance, where an edge term is one product):
//  each level's new row is published to one of two LDS buffers by step
//  parity (one barrier); each wavefront computes both of its y edge terms
//  itself from the rows above and below.  An edge term depends only on the
//  two voxels' values, so both wavefronts obtain the same bits.
//
// LDS holds, per level, W+2 slots of 64*V floats: wavefront w uses slot w+1
// (its R rows side by side, lane groups of 64/R), slots 0 and W+1 hold zeros so
// the rows at the tile's edge read without a branch (their edge coefficient is
// the closed one, or the row is halo).  Element i of a lane's chunk sits at
// i*64 + lane: consecutive lanes hit consecutive banks.  With R > 1 the x edge
// between the last lane of one row and the first lane of the next (adjacent
// lanes, exchanged by the same DPP shifts) has the closed coefficient, since
// a row's lanes cover the whole row, so no value crosses rows.
// (Piece: plan.h)

// Which of the two y edge schemes a conductance uses (above).
template <int COND>
constexpr bool y_row_shared() {
    return COND == COND_INTENSITY;
}

// One piece of one pass: the whole per-workgroup algorithm above.  `lds`
// must hold stream_lds_bytes(V, T, W) bytes.  Called by k_stream (one cube)
// and by the batch round kernel.
// Calls f(std::integral_constant<int, 2^k - 1>) for the k in 0..K with
// vmask == 2^k - 1 (k = 0 when no larger one matches).
template <int K, typename F>
__device__ __forceinline__ void level_mask_dispatch(int vmask, F&& f) {
    if constexpr (K == 0) {
        f(std::integral_constant<int, 0>{});
    } else {
        if (vmask == (1 << K) - 1) f(std::integral_constant<int, (1 << K) - 1>{});
        else level_mask_dispatch<K - 1>(vmask, f);
    }
}

template <int COND, typename ST, int V, int T, bool VEC, int R>
__device__ __forceinline__ void stream_piece(const ST* __restrict__ src, ST* __restrict__ dst, const BlockGeom& g,
                                             const Piece pc, const DevParams& P, float* __restrict__ lds) {
    constexpr int RX = 64 * V;
    constexpr int LR = 64 / R;                    // lanes per row
    constexpr bool RS = y_row_shared<COND>();
    const int lane = threadIdx.x;
    const int sr = R == 1 ? 0 : lane / LR;        // this lane's row within the wavefront
    const int lr = R == 1 ? lane : lane % LR;     // this lane's place in its row
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int W = g.W;
    const int rows = W * R;
    const int nx = g.nx, ny = g.ny, nz = g.nz;

    // tiles share the rows evenly (tile k outputs rows [k ny / nty, (k+1) ny / nty))
    // and the columns evenly in whole lane chunks (tile k starts at k nx / ntx
    // rounded up to a multiple of V), so no tile is a thin ragged remainder;
    // the planner's geometry guarantees each tile's outputs fit ox x oy
    const int oy0 = (int)((long)pc.ty * ny / g.nty), oy1 = (int)((long)(pc.ty + 1) * ny / g.nty);
    const long xq = (long)g.ntx * V;
    const int ox0 = V * (int)(((long)pc.tx * nx + xq - 1) / xq);
    const int ox1 = pc.tx + 1 == g.ntx ? nx : V * (int)(((long)(pc.tx + 1) * nx + xq - 1) / xq);
    const int oz0 = pc.z0, oz1 = pc.z1;
    const int rx0 = g.ntx > 1 ? ox0 - g.hx : 0;
    const int ry0 = g.nty > 1 ? oy0 - T : 0;
    const int zin0 = max(oz0 - T, 0), zin1 = min(oz1 + T, nz);
    const int nin = zin1 - zin0;
    const int y = ry0 + w * R + sr;               // this lane's row
    const int xl0 = rx0 + lr * V;

    // x edge coefficients.  Vector path (nx a multiple of V, tile origins
    // multiples of V): a lane's chunk lies wholly inside or wholly outside the
    // cube, so the edges inside a chunk are open (a chunk outside the cube
    // holds clamped, finite values that never reach the cube), and only the
    // edge to the next lane can cross a face: closed unless both of its
    // voxels are in the cube.  Scalar path: per edge.
    float cx[VEC ? 1 : V];
    if constexpr (VEC) {
        cx[0] = (xl0 + V >= 1 && xl0 + V < nx) ? P.coef[0] : P.closed;
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int x = xl0 + i;
            cx[i] = (x >= 0 && x + 1 < nx) ? P.coef[0] : P.closed;
        }
    }
    const float cyu = (y >= 0 && y + 1 < ny) ? P.coef[1] : P.closed;   // edge (y, y+1)
    const float cyd = (y >= 1 && y < ny) ? P.coef[1] : P.closed;       // edge (y-1, y)
    const bool row_in = y >= 0 && y < ny;
    const bool row_store = y >= oy0 && y < oy1;
    const int lo_base = ry0 <= 0 ? 0 : ry0;
    const int hi_base = ry0 + rows >= ny ? ny : ry0 + rows;
    const int lo_step = ry0 <= 0 ? 0 : 1;
    const int hi_step = ry0 + rows >= ny ? 0 : 1;

    const int ycl = min(max(y, 0), ny - 1);
    // 16-bit storage, vector path: input and output rows move through raw
    // buffers over this tile's rows of one plane (at most 64 rows; the planner
    // keeps them below 2^30 bytes).  A plane with nothing to load or store gets a buffer of size
    // 0 and a lane outside the output rows or columns a store offset past the
    // end, so every step issues the same memory operations and the compiler's
    // waits for an input plane count exactly the operations issued after it
    // (measured: 760 -> 870 Gvoxel-iter/s for bfloat16 on the 512^3 cube; FP32
    // keeps plain loads and stores, which the halo rows skip, and is 2 % faster so).
    constexpr bool BUF = VEC && sizeof(ST) == 2;
    const int yb = max(ry0, 0);
    const int tile_bytes = (min(ry0 + rows, ny) - yb) * nx * (int)sizeof(ST);
    const int st_off = (row_store && xl0 >= ox0 && xl0 + V <= ox1) ? ((y - yb) * nx + xl0) * (int)sizeof(ST)
                                                                   : kBufOffNone;
    const long plane = (long)nx * ny;
    const ST* rowp = src + (long)ycl * nx;
    const int xv = min(max(xl0, 0), nx - V);

    // LDS regions of T levels each (lvl floats per level): edge-shared uses
    // region 0 for rows and region 1 for up-edge terms; row-shared uses them
    // as the two parity buffers of rows.
    const int lvl = (W + 2) * RX;
    const int reg1 = T * lvl;
    const int slot = (w + 1) * RX + lane;            // + t * lvl + i * 64 (+ reg1)
    // offsets to the same lane place in the rows above and below
    const int up_off = (R == 1 || sr == R - 1) ? RX - (R - 1) * LR : LR;
    const int dn_off = (R == 1 || sr == 0) ? -(RX - (R - 1) * LR) : -LR;

    // Register rotation (the step loop is unrolled by two, parity p known at
    // compile time): lv[t][p] is level t's current plane and lv[t][p^1] the
    // plane above it; level t writes its result straight into lv[t+1][p^1],
    // and the next step swaps the roles, so no plane is copied between
    // registers.  Only the prefetched input plane is copied into lv[0][p^1].
    // fz[t] is the z edge term below the current plane of level t.
    float lv[T][2][V], fz[T][V];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int i = 0; i < V; ++i) {
            lv[t][0][i] = 0.0f;
            lv[t][1][i] = 0.0f;
            fz[t][i] = 0.0f;
        }
    // zero this wavefront's slots and, from wavefront 0, the pad slots
#pragma unroll
    for (int r = 0; r < 2 * T; ++r)
#pragma unroll
        for (int i = 0; i < V; ++i) {
            lds[r * lvl + slot + 64 * i] = 0.0f;
            if (w == 0) {
                lds[r * lvl + lane + 64 * i] = 0.0f;
                lds[r * lvl + (W + 1) * RX + lane + 64 * i] = 0.0f;
            }
        }

    float pf[V];
    const int ld_off = ((ycl - yb) * nx + xv) * (int)sizeof(ST);
    // scalar path: this lane's chunk lies wholly inside the row; its loads
    // start at xs (nx >= V, which the planner guarantees) and shift by sh
    const bool inside = xl0 >= 0 && xl0 + V <= nx;
    const int xs = min(max(xl0, 0), nx - V), sh = xl0 - xs;
    // FP32 scalar path stores (store_row_f32): whole chunks in the output
    // range, or the first k values of the chunk that reaches the range's end
    constexpr bool RAG = !VEC && sizeof(ST) == 4 && V >= 2;
    const int rag_k = ox1 - xl0;
    const bool rag_rowok = row_store && xl0 >= ox0;
    const int rag_full = (rag_rowok && xl0 + V <= ox1) ? ((y - yb) * nx + xl0) * 4 : kBufOffNone;
    const int rag_tail = (rag_rowok && rag_k > 0 && rag_k < V) ? ((y - yb) * nx + xl0) * 4 : kBufOffNone;
    // input plane zin0 + k into pf (buffer path: zeros, with no memory access,
    // when k is past the input range; otherwise not issued then)
    auto load = [&](int k) {
        if constexpr (BUF) {
            const int kc = max(min(k, nin - 1), 0);
            const auto rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(src + (long)(zin0 + kc) * plane + (long)yb * nx), 0, k < nin ? tile_bytes : 0, kBufWord3);
            BufRow16<ST, V>::load(rs, ld_off, pf);
        } else if (k < nin) {
            const ST* r = rowp + (long)(zin0 + k) * plane;
            if constexpr (VEC) {
                Vec<ST, V>::load(r + xv, pf);
            } else {
                // every lane: one vector access (aligned to the element only)
                // at its chunk clamped into the row; shift_clamp moves the
                // values into place when the plane is used (no branch around
                // the load, so the loop's waits stay exact)
                VecU<ST, V>::load(r + xs, pf);
            }
        }
    };
    if (nin > 0) load(0);
    __syncthreads();

    const int nsteps = nin + T;
    // level t (0-based) is exact on this row when y lies in [lo_t, hi_t)
    bool valid[T];
#pragma unroll
    for (int t = 0; t < T; ++t)
        valid[t] = row_in && y >= lo_base + (t + 1) * lo_step && y < hi_base - (t + 1) * hi_step;

    // Levels exact on this wavefront's row(s): bit t for level t.  A row's
    // validity holds for the whole piece, and level t + 1 valid implies level t
    // valid, so the mask is 2^k - 1.  In passes of depth 1 and 2 the steady
    // loop is compiled once per mask, with the mask a compile-time constant: with no skip branch inside
    // the loop there are no control-flow joins, and the compiler keeps the
    // register rotation without copies.
    int vmask = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        bool v;
        if constexpr (R == 1) v = valid[t];
        else v = __any(valid[t]);
        vmask |= v ? 1 << t : 0;
    }

    // One step.  STEADY: every level computes and has the plane above (the
    // steps T <= s < nin), so none of the start/end conditions are evaluated.
    // VM >= 0: the validity mask, known at compile time; -1: test valid[] here.
    auto step = [&](auto parity, auto steady, auto vm, int s) {
        constexpr int p = decltype(parity)::value, q = p ^ 1;
        constexpr bool STEADY = decltype(steady)::value;
        constexpr int VM = decltype(vm)::value;
        if (STEADY || s < nin) {
            if constexpr (VEC) {
#pragma unroll
                for (int i = 0; i < V; ++i) lv[0][q][i] = pf[i];
            } else {
                shift_clamp<V>(pf, sh, lv[0][q]);
            }
        }
        load(s + 1);

        // every level advances one plane; out holds the last level's new row
        float out[V];
        if constexpr (BUF || RAG) {
#pragma unroll
            for (int i = 0; i < V; ++i) out[i] = 0.0f;
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const bool has_nxt = STEADY || ((s - t >= 0) && (s - t < nin));
            const bool compute = STEADY || ((s - t - 1 >= 0) && (s - t - 1 < nin));
            const int pz = zin0 + s - t - 1;
            // halo rows of a level are never used by a valid row: skip them
            // (with R > 1, when no row of the wavefront is valid)
            if (!compute) continue;
            if constexpr (VM >= 0) {
                if (((VM >> t) & 1) == 0) continue;   // a constant once the level loop is unrolled
            } else if constexpr (R == 1) {
                if (!valid[t]) continue;
            } else {
                if (!__any(valid[t])) continue;
            }
            const float czp = (STEADY || (pz + 1 < nz && has_nxt)) ? P.coef[2] : P.closed;
            float ex[V];
#pragma unroll
            for (int i = 0; i < V - 1; ++i)
                ex[i] = edge_term<COND>(lv[t][p][i + 1] - lv[t][p][i], VEC ? P.coef[0] : cx[i], P.kap);
            const float right = lane_shl1(lv[t][p][0]);
            ex[V - 1] = edge_term<COND>(right - lv[t][p][V - 1], cx[VEC ? 0 : V - 1], P.kap);
            const float exm0 = lane_shr1(ex[V - 1]);
            // rows of this level's current plane (published one step earlier)
            const int ro = (RS ? p * reg1 : reg1) + t * lvl + slot;
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const float c = lv[t][p][i];
                float eyd, eyu;
                if constexpr (RS) {
                    eyd = edge_term<COND>(c - lds[ro + dn_off + 64 * i], cyd, P.kap);
                    eyu = edge_term<COND>(lds[ro + up_off + 64 * i] - c, cyu, P.kap);
                } else {
                    eyd = lds[ro + dn_off + 64 * i];
                    eyu = lds[ro + 64 * i];
                }
                const float up_z = has_nxt ? lv[t][q][i] : c;
                const float ezp = edge_term<COND>(up_z - c, czp, P.kap);
                const float o = combine<COND>(c, i == 0 ? exm0 : ex[i - 1], ex[i], eyd, eyu, fz[t][i], ezp,
                                              P.kap, P.tau);
                fz[t][i] = ezp;
                if (t + 1 < T) lv[t + 1][q][i] = Store<ST>::quant(o);
                else out[i] = Store<ST>::quant(o);
            }
            if (!BUF && !RAG && t == T - 1 && row_store && pz >= oz0 && pz < oz1) {
                ST* r = dst + (long)pz * plane + (long)y * nx;
                if constexpr (VEC) {
                    if (xl0 >= ox0 && xl0 + V <= ox1) Vec<ST, V>::store(r + xl0, out);
                } else if (inside && xl0 >= ox0 && xl0 + V <= ox1) {
                    VecU<ST, V>::store(r + xl0, out);
                } else {
#pragma unroll
                    for (int i = 0; i < V; ++i) {
                        const int x = xl0 + i;
                        if (x >= ox0 && x < ox1) r[x] = Store<ST>::store(out[i]);
                    }
                }
            }
        }
        // buffer path: the last level's row goes out on every step, outside
        // the per-row skip above (a row that skipped it is never an output
        // row, so its lanes hold kBufOffNone; a plane the step does not
        // produce gets a buffer of size 0)
        if constexpr (RAG) {
            const int pz = zin0 + s - T;
            const bool zon = pz >= oz0 && pz < oz1;
            const int pzc = max(min(pz, zin1 - 1), zin0);
            const auto rs = __builtin_amdgcn_make_buffer_rsrc((void*)(dst + (long)pzc * plane + (long)yb * nx), 0,
                                                              zon ? tile_bytes : 0, kBufWord3);
            store_row_f32<V>(rs, rag_full, rag_tail, rag_k, out);
        }
        if constexpr (BUF) {
            const int pz = zin0 + s - T;
            const bool zon = pz >= oz0 && pz < oz1;
            const int pzc = max(min(pz, zin1 - 1), zin0);
            const auto rs = __builtin_amdgcn_make_buffer_rsrc((void*)(dst + (long)pzc * plane + (long)yb * nx), 0,
                                                              zon ? tile_bytes : 0, kBufWord3);
            BufRow16<ST, V>::store(rs, st_off, out);
        }
        // publish each level's new current row (lv[t][q])
        const int wo = (RS ? q * reg1 : 0) + slot;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            if (STEADY || ((s - t >= 0) && (s - t < nin))) {
#pragma unroll
                for (int i = 0; i < V; ++i) lds[wo + t * lvl + 64 * i] = lv[t][q][i];
            }
        }
        __syncthreads();
        if constexpr (!RS) {
            // y edge term from the new current row to the row above
#pragma unroll
            for (int t = 0; t < T; ++t) {
                if (STEADY || ((s - t >= 0) && (s - t < nin))) {
                    const int ro = t * lvl + slot;
#pragma unroll
                    for (int i = 0; i < V; ++i)
                        lds[reg1 + ro + 64 * i] =
                            edge_term<COND>(lds[ro + up_off + 64 * i] - lv[t][q][i], cyu, P.kap);
                }
            }
            __syncthreads();
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using GEN = std::false_type;
    using STD = std::true_type;
    constexpr int PT = T & 1;   // parity of step T
    using PA = std::integral_constant<int, PT>;
    using PB = std::integral_constant<int, PT ^ 1>;

    using VRT = std::integral_constant<int, -1>;   // validity tested at run time

    // prologue: steps 0 .. T-1 (parity s & 1)
#pragma unroll
    for (int s0 = 0; s0 < T; ++s0) {
        if (s0 < nsteps) {
            if ((s0 & 1) == 0) step(I0{}, GEN{}, VRT{}, s0);
            else step(I1{}, GEN{}, VRT{}, s0);
        }
    }
    // steady state: steps T .. nin-1, two per iteration
    int s = T;
    auto steady_loop = [&](auto vm) {
        for (; s + 1 < nin; s += 2) {
            step(PA{}, STD{}, vm, s);
            step(PB{}, STD{}, vm, s + 1);
        }
    };
    // deeper passes keep one loop: their T + 1 copies would not fit the
    // register file without spilling
    if constexpr (T <= 2) level_mask_dispatch<T>(vmask, steady_loop);
    else steady_loop(VRT{});
    // remaining steps: at most one steady one, then the epilogue
    for (; s < nsteps; ++s) {
        if (((s - T) & 1) == 0) step(PA{}, GEN{}, VRT{}, s);
        else step(PB{}, GEN{}, VRT{}, s);
    }
}

template <int COND, typename ST, int V, int T, bool VEC, int R>
__global__ void __launch_bounds__(1024)
k_stream(const ST* __restrict__ src, ST* __restrict__ dst, BlockGeom g, const Piece* __restrict__ pieces,
         const DevParams* __restrict__ dp) {
    extern __shared__ float lds[];
    const DevParams P = *dp;
    if (P.abort) return;
    stream_piece<COND, ST, V, T, VEC, R>(src, dst, g, pieces[blockIdx.x], P, lds);
}

// Grouped plans: workgroup b runs pieces [first[b], first[b + 1]) in turn
// (first: the ints after the piece table; the bounds come from
// workgroup-uniform addresses, so the loop is uniform).  A kernel of its own:
// the loop around the streaming body raises register pressure (the per-lane
// geometry stays live across pieces), which the one-piece kernel should not pay.
template <int COND, typename ST, int V, int T, bool VEC, int R>
__global__ void __launch_bounds__(1024)
k_stream_grouped(const ST* __restrict__ src, ST* __restrict__ dst, BlockGeom g, const Piece* __restrict__ pieces,
                 const DevParams* __restrict__ dp) {
    extern __shared__ float lds[];
    const DevParams P = *dp;
    if (P.abort) return;
    const int* first = reinterpret_cast<const int*>(pieces + g.npieces);
    const int k0 = first[blockIdx.x], k1 = first[blockIdx.x + 1];
    for (int k = k0; k < k1; ++k) {
        if (k > k0) __syncthreads();   // the previous piece is done with the LDS
        stream_piece<COND, ST, V, T, VEC, R>(src, dst, g, pieces[k], P, lds);
    }
}

}  // namespace igk
