// The host planner of the filter's streaming kernel and the validation of
// its parameters: plain C++ (no GPU headers), so it can also be built and
// checked on its own (with the sanitizers, in the CPU tests).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "igfilter.h"

namespace igk {

// Work split of one pass of the streaming kernel (k_stream): the tile grid of
// the cube and the piece table (x tile, y tile, output planes).
struct BlockGeom {
    int nx, ny, nz;
    int ntx, nty;         // tile counts in x, y
    int ox, oy;           // output extent of a tile in x, y
    int W;                // wavefronts per workgroup (== blockDim.y)
    int vec;              // 1: lane chunks are whole and aligned (vector I/O)
    int R;                // rows per wavefront (1, 2 or 4); a tile has W * R rows
    int hx;               // x halo of a tile when ntx > 1 (t_block rounded up to whole lane chunks)
};

struct Piece {
    int tx, ty, z0, z1;
};

// LDS bytes of the streaming kernel: two regions of T levels, each level
// W + 2 row slots of 64 V floats (current rows and up-edge terms).
inline size_t stream_lds_bytes(int V, int T, int W) { return (size_t)2 * T * (W + 2) * 64 * V * sizeof(float); }
constexpr size_t kMaxLds = 160 * 1024;

}  // namespace igk

// One pass of the streaming kernel, fully planned: geometry and piece table.
struct PassPlan {
    igk::BlockGeom g{};
    std::vector<igk::Piece> pieces;
    int V = 0, T = 0;
};
void auto_vec_rows(int64_t nx, int* V, int* R);
int resident_per_cu(int W, size_t lds);
// nullptr on success, else the reason schedule s cannot serve p at depth T
const char* plan_pass(const ig_params& p, const ig_schedule& s, int T, int ncu, PassPlan* pp);
ig_status igk_validate_params(const ig_params* p);
// The library's schedule for p when the caller sets none.
ig_schedule igk_auto_schedule(const ig_params* p);
// Record a thread-local message for ig_last_error() and return s.
ig_status igk_fail(ig_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
size_t dtype_size(int dt);
