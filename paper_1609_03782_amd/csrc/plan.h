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
    int ox, oy;           // largest output extent of a tile in x, y (the split below keeps every tile within it)
    int W;                // wavefronts per workgroup (== blockDim.y)
    int vec;              // 1: lane chunks are whole and aligned (vector I/O)
    int R;                // rows per wavefront (1, 2 or 4); a tile has W * R rows
    int hx;               // x halo of a tile when ntx > 1 (t_block rounded up to whole lane chunks)
    int npieces;          // pieces in the table
    int grouped;          // 1: workgroup b runs pieces [first[b], first[b+1]) (the ints after the table); 0: piece b
};

struct Piece {
    int tx, ty, z0, z1;
};

// Output extent of tile k: rows [k ny / nty, (k+1) ny / nty); columns from
// k nx / ntx rounded up to a multiple of V to the next tile's start (nx for
// the last).  The streaming kernel computes the same bounds.
inline void tile_rows(const BlockGeom& g, int k, int* y0, int* y1) {
    *y0 = (int)((long)k * g.ny / g.nty);
    *y1 = (int)((long)(k + 1) * g.ny / g.nty);
}
inline void tile_cols(const BlockGeom& g, int V, int k, int* x0, int* x1) {
    const long q = (long)g.ntx * V;
    *x0 = V * (int)(((long)k * g.nx + q - 1) / q);
    *x1 = k + 1 == g.ntx ? g.nx : V * (int)(((long)(k + 1) * g.nx + q - 1) / q);
}

// LDS bytes of the streaming kernel: two regions of T levels, each level
// W + 2 row slots of 64 V floats (current rows and up-edge terms).
inline size_t stream_lds_bytes(int V, int T, int W) { return (size_t)2 * T * (W + 2) * 64 * V * sizeof(float); }
constexpr size_t kMaxLds = 160 * 1024;

}  // namespace igk

// One pass of the streaming kernel, fully planned: geometry and piece table;
// with `first` non-empty, workgroup b runs pieces [first[b], first[b+1]) in
// turn (the device table holds the pieces, then `first` as ints).
struct PassPlan {
    igk::BlockGeom g{};
    std::vector<igk::Piece> pieces;
    std::vector<int> first;
    int V = 0, T = 0;
    int workgroups() const { return first.empty() ? (int)pieces.size() : (int)first.size() - 1; }
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
