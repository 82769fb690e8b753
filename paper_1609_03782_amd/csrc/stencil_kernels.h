// Filter-step kernels for gfx950 (wave64).
//
//  k_naive   one step per launch, one voxel per thread, neighbours straight
//            from global memory.  The reference schedule.
//  k_blocked t_block steps per launch.  A workgroup owns an xy tile (halo of
//            t_block voxels where it borders another tile) and a chunk of
//            z-planes; it streams the planes in z order, keeping every
//            intermediate step of the pass on chip:
//              lane      -> V consecutive x voxels (one 16-byte load for V=8
//                           in 16-bit storage, two for FP32);
//              wavefront -> R consecutive rows; x neighbours cross lanes by
//                           DPP wave shifts, so an x edge term is computed once;
//              workgroup -> W wavefronts stacked in y; the first and last row
//                           of each wavefront go through LDS to its neighbours;
//              z         -> each step level keeps its current plane and the
//                           edge term to the plane below in registers, so a z
//                           edge term is computed once.
//            Level t of a pass turns plane p of level t-1 into plane p of
//            level t as soon as plane p+1 of level t-1 exists; the last level
//            is written to global memory.  Rows, columns and planes that a
//            level cannot compute correctly (they would need data outside
//            the tile) are halo; the tile's outputs never depend on them.
//
// Both kernels use edge_term/combine from stencil_common.h in the same order,
// so their results are bitwise identical.
#pragma once
#include "stencil_common.h"

namespace igk {

struct NaiveGeom {
    int nx, ny, nz;
};

struct BlockGeom {
    int nx, ny, nz;
    int ntx, nty, nzc;    // tile counts in x, y, z
    int ox, oy, oz;       // output extent of a tile in x, y, z
    int W;                // wavefronts per workgroup (== blockDim.y)
    int remap;            // spread consecutive tiles over one XCD's L2
    int vec;              // 1: lane chunks are whole and aligned (vector I/O)
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

// ---------------------------------------------------------------- blocked
template <int COND, typename ST, int V, int R, int T>
__global__ void __launch_bounds__(512)
k_blocked(const ST* __restrict__ src, ST* __restrict__ dst, BlockGeom g,
          const DevParams* __restrict__ dp) {
    extern __shared__ float lds[];   // [T][W][2][64*V]: first/last row of each level's current plane
    const DevParams P = *dp;
    if (P.abort) return;

    const int lane = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int W = g.W;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    constexpr int RX = 64 * V;
    const int RY = W * R;

    int bid = blockIdx.x;
    if (g.remap) {                       // consecutive tiles -> same XCD (round-robin dispatch)
        const int nb = gridDim.x;
        bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    }
    const int tx = bid % g.ntx;
    const int rest = bid / g.ntx;
    const int ty = rest % g.nty;
    const int tz = rest / g.nty;

    const int ox0 = tx * g.ox, oy0 = ty * g.oy, oz0 = tz * g.oz;
    const int ox1 = min(ox0 + g.ox, nx), oy1 = min(oy0 + g.oy, ny), oz1 = min(oz0 + g.oz, nz);
    const int rx0 = g.ntx > 1 ? ox0 - T : 0;
    const int ry0 = g.nty > 1 ? oy0 - T : 0;
    const int zin0 = max(oz0 - T, 0), zin1 = min(oz1 + T, nz);
    const int nin = zin1 - zin0;

    const int xl0 = rx0 + lane * V;           // first x of this lane
    const int yw0 = ry0 + w * R;              // first y of this wavefront

    // edge coefficients: x edge i joins xl0+i and xl0+i+1; y edge k joins yw0+k-1 and yw0+k
    float cx[V], cy[R + 1];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const int x = xl0 + i;
        cx[i] = (x >= 0 && x + 1 < nx) ? P.coef[0] : P.closed;
    }
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        const int y = yw0 + k - 1;
        cy[k] = (y >= 0 && y + 1 < ny) ? P.coef[1] : P.closed;
    }

    // x offsets of the lane's voxels clamped into the cube (halo lanes read
    // real, finite data; their results are never used)
    const bool vec = g.vec;
    const int xv = min(max(xl0, 0), nx - V);  // vector path: whole chunk inside
    int xs[V];
#pragma unroll
    for (int i = 0; i < V; ++i) xs[i] = min(max(xl0 + i, 0), nx - 1);

    auto load_plane = [&](int z, float (&o)[R][V]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = min(max(yw0 + r, 0), ny - 1);
            const ST* row = src + ((long)z * ny + y) * nx;
            if (vec) {
                Vec<ST, V>::load(row + xv, o[r]);
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) o[r][i] = Store<ST>::load(row[xs[i]]);
            }
        }
    };

    float cur[T][R][V];   // level t: current plane of level t-1 (awaiting its z+ neighbour)
    float fzm[T][R][V];   // level t: edge term to the plane below
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < V; ++i) { cur[t][r][i] = 0.0f; fzm[t][r][i] = 0.0f; }

    float pf[R][V];
    if (nin > 0) load_plane(zin0, pf);

    float* lds_lvl = lds;  // base
    const int row_stride = RX;
    auto lds_row = [&](int t, int wave, int side) -> float* {
        return lds_lvl + ((t * W + wave) * 2 + side) * row_stride;
    };

    const int nsteps = nin + T;
    for (int s = 0; s < nsteps; ++s) {
        float nxt[R][V];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < V; ++i) nxt[r][i] = pf[r][i];
        if (s + 1 < nin) load_plane(zin0 + s + 1, pf);

#pragma unroll
        for (int t = 0; t < T; ++t) {
            // level t+1 of the pass; `nxt` holds plane zin0+s-t of level t (if any)
            const bool has_nxt = (s - t >= 0) && (s - t < nin);
            const bool compute = (s - t - 1 >= 0) && (s - t - 1 < nin);
            const int p = zin0 + s - t - 1;   // plane computed by this level
            float outv[R][V];
            if (compute) {
                const int L = t + 1;          // level number
                const int lo = ry0 <= 0 ? 0 : ry0 + L;
                const int hi = ry0 + RY >= ny ? ny : ry0 + RY - L;
                const float czp = (p + 1 < nz && has_nxt) ? P.coef[2] : P.closed;
                // rows next to this wavefront, from its neighbours (same level, same plane)
                float dn[V], up[V];
                if (w > 0) {
                    const float* q = lds_row(t, w - 1, 1) + lane * V;
#pragma unroll
                    for (int i = 0; i < V; ++i) dn[i] = q[i];
                } else {
#pragma unroll
                    for (int i = 0; i < V; ++i) dn[i] = cur[t][0][i];
                }
                if (w + 1 < W) {
                    const float* q = lds_row(t, w + 1, 0) + lane * V;
#pragma unroll
                    for (int i = 0; i < V; ++i) up[i] = q[i];
                } else {
#pragma unroll
                    for (int i = 0; i < V; ++i) up[i] = cur[t][R - 1][i];
                }
                // y edge terms: ey[k] joins row k-1 and row k (row -1 = dn, row R = up)
                float ey[R + 1][V];
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    ey[0][i] = edge_term<COND>(cur[t][0][i] - dn[i], cy[0], P.kap);
#pragma unroll
                    for (int k = 1; k < R; ++k)
                        ey[k][i] = edge_term<COND>(cur[t][k][i] - cur[t][k - 1][i], cy[k], P.kap);
                    ey[R][i] = edge_term<COND>(up[i] - cur[t][R - 1][i], cy[R], P.kap);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int y = yw0 + r;
                    if (y < lo || y >= hi) {
#pragma unroll
                        for (int i = 0; i < V; ++i) outv[r][i] = cur[t][r][i];
                        continue;
                    }
                    float ex[V];
#pragma unroll
                    for (int i = 0; i < V - 1; ++i)
                        ex[i] = edge_term<COND>(cur[t][r][i + 1] - cur[t][r][i], cx[i], P.kap);
                    const float right = lane_shl1(cur[t][r][0]);
                    ex[V - 1] = edge_term<COND>(right - cur[t][r][V - 1], cx[V - 1], P.kap);
                    const float exm0 = lane_shr1(ex[V - 1]);
#pragma unroll
                    for (int i = 0; i < V; ++i) {
                        const float n_up = has_nxt ? nxt[r][i] : cur[t][r][i];
                        const float ezp = edge_term<COND>(n_up - cur[t][r][i], czp, P.kap);
                        const float exm = i == 0 ? exm0 : ex[i - 1];
                        const float o = combine<COND>(cur[t][r][i], exm, ex[i], ey[r][i], ey[r + 1][i],
                                                      fzm[t][r][i], ezp, P.kap, P.tau);
                        outv[r][i] = Store<ST>::quant(o);
                        fzm[t][r][i] = ezp;
                    }
                }
            }
            if (has_nxt) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int i = 0; i < V; ++i) cur[t][r][i] = nxt[r][i];
            }
            if (compute) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int i = 0; i < V; ++i) nxt[r][i] = outv[r][i];
            }
            if (t == T - 1 && compute && p >= oz0 && p < oz1) {
                // write the last level's plane: rows [oy0, oy1), columns [ox0, ox1)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int y = yw0 + r;
                    if (y < oy0 || y >= oy1) continue;
                    ST* row = dst + ((long)p * ny + y) * nx;
                    if (vec && xl0 >= ox0 && xl0 + V <= ox1) {
                        Vec<ST, V>::store(row + xl0, outv[r]);
                    } else {
#pragma unroll
                        for (int i = 0; i < V; ++i) {
                            const int x = xl0 + i;
                            if (x >= ox0 && x < ox1) row[x] = Store<ST>::store(outv[r][i]);
                        }
                    }
                }
            }
        }
        // publish the new current planes' edge rows for the next step
        __syncthreads();
#pragma unroll
        for (int t = 0; t < T; ++t) {
            float* q0 = lds_row(t, w, 0) + lane * V;
            float* q1 = lds_row(t, w, 1) + lane * V;
#pragma unroll
            for (int i = 0; i < V; ++i) { q0[i] = cur[t][0][i]; q1[i] = cur[t][R - 1][i]; }
        }
        __syncthreads();
    }
}

}  // namespace igk
