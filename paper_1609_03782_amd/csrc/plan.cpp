// Host planner and parameter validation of the filter (see plan.h).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

using namespace igk;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

ig_status igk_fail(ig_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}


extern "C" const char* ig_last_error(void) { return g_last_error.c_str(); }

#define fail igk_fail

namespace {
bool finite_f(float v) { return std::isfinite(v); }
}  // namespace

size_t dtype_size(int dt) { return dt == IG_F32 ? 4 : 2; }

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
// Automatic x layout: 8 voxels per lane for 256 < nx <= 512 (one tile), 4
// per lane in 256-voxel x tiles above 512; up to 256, 4 voxels per lane and as
// many rows per wavefront as keep one row's lanes covering nx, so narrow cubes
// still give every lane 4 voxels.
void auto_vec_rows(int64_t nx, int* V, int* R) {
    // 8 voxels per lane while one 512-voxel tile holds the row; wider rows
    // need x tiles, and 256-voxel tiles waste fewer lanes on the last, partly
    // filled tile (measured on gfx950: 731 against 495 Gvoxel-iter/s at
    // nx = 1024, 860 against 648 at 2048, 574 against 344 at 600)
    if (nx > 512) { *V = 4; *R = 1; return; }
    if (nx > 256) { *V = 8; *R = 1; return; }
    if (nx < 4) { *V = nx >= 2 ? 2 : 1; *R = 1; return; }   // a lane's chunk never exceeds the row
    *V = 4;
    *R = nx <= 64 ? 4 : nx <= 128 ? 2 : 1;
}

// Workgroups of the streaming kernel one CU holds at once: 16 wavefronts of
// at most 128 VGPRs each (launch bound of 1024 threads) and 160 KB of LDS.
int resident_per_cu(int W, size_t lds) {
    const int by_waves = 16 / W;
    const int by_lds = (int)(kMaxLds / std::max<size_t>(lds, 1));
    return std::max(1, std::min(by_waves, by_lds));
}

// Equal shares of work per workgroup: the sequence tile 0 planes 0..nz-1,
// tile 1 planes 0..nz-1, ... (tiles in y-then-x order, every tile-plane one
// unit of work) is cut into G contiguous ranges of equal cost, and range b
// becomes the pieces of workgroup b (one, or two where it crosses a tile
// boundary).  Every piece refills the pipeline (its 2T halo planes and T
// extra steps), so each tile boundary inside the sequence counts 3T units:
// a range that takes a second piece takes fewer planes.  (Cutting each XCD's
// z-band separately, to keep neighbouring tiles on one L2, gave every
// workgroup two or three short pieces and measured slower.)
static void group_split(const BlockGeom& g, long ntiles, long G, int T, PassPlan* pp) {
    const int64_t nz = g.nz, F = 3 * T;
    const int64_t unit = nz + F;                 // a tile's cost with the refill that starts it
    const int64_t tot = ntiles * unit - F;       // the first tile's fill is paid by every range alike
    // position of cost x: (tile, plane); inside a refill it is plane 0 of that tile
    auto pos = [&](int64_t x, long* ti, int64_t* pl) {
        if (x >= tot) { *ti = ntiles; *pl = 0; return; }
        const int64_t y = x + F;                 // tile t spans [t unit, (t + 1) unit), its planes after F
        *ti = (long)(y / unit);
        *pl = std::max<int64_t>(0, y % unit - F);
    };
    pp->pieces.clear();
    pp->first.assign(1, 0);
    for (long b = 0; b < G; ++b) {
        long ta, tb;
        int64_t pa, pb;
        pos(tot * b / G, &ta, &pa);
        pos(b + 1 == G ? tot : tot * (b + 1) / G, &tb, &pb);
        for (long t = ta; t <= tb && t < ntiles; ++t) {
            const int64_t p0 = t == ta ? pa : 0, p1 = t == tb ? pb : nz;
            if (p1 > p0) pp->pieces.push_back(Piece{(int)(t % g.ntx), (int)(t / g.ntx), (int)p0, (int)p1});
        }
        pp->first.push_back((int)pp->pieces.size());
    }
    pp->g.npieces = (int)pp->pieces.size();
    pp->g.grouped = 1;
}

// Plan the pass of depth T for schedule s; returns nullptr or the reason it
// cannot serve the shape.
const char* plan_pass(const ig_params& p, const ig_schedule& s, int T, int ncu, PassPlan* pp) {
    const int nx = (int)p.nx, ny = (int)p.ny, nz = (int)p.nz;
    int V = s.vec, R = s.rows;
    if (V == 0) {
        int av, ar;
        auto_vec_rows(p.nx, &av, &ar);
        V = av;
        if (R == 0) R = ar;
    }
    if (R == 0) R = 1;
    const int W = s.waves;
    if (!(V == 1 || V == 2 || V == 4 || V == 8)) return "vec must be 1, 2, 4 or 8";
    if (V > nx) return "vec must not exceed nx";
    // a tile's rows of one plane are addressed with 32-bit byte offsets below 2^30
    if ((long)s.waves * std::max(R, 1) * nx * (long)dtype_size(p.dtype) >= (1L << 30))
        return "rows too long for the blocked schedule (use naive)";
    if (!(R == 1 || R == 2 || R == 4)) return "rows must be 1, 2 or 4";
    if (R > 1 && (V != 4 || (64 / R) * V < nx)) return "rows > 1 needs vec 4 and nx <= 256 / rows";
    if (W < 1 || W > 16) return "waves must be in 1..16";
    if (T < 1 || T > 4) return "t_block must be in 1..4";
    if (s.zchunk < 0 || s.rounds < 0) return "zchunk and rounds must be >= 0";
    const size_t lds = stream_lds_bytes(V, T, W);
    if (lds > kMaxLds) return "tile needs more LDS than a CU has (reduce waves, vec or t_block)";
    BlockGeom& g = pp->g;
    g.nx = nx; g.ny = ny; g.nz = nz; g.W = W; g.R = R;
    const int RX = 64 * V;
    if (nx <= RX) { g.ntx = 1; g.ox = nx; g.hx = 0; }
    else {
        // halo of whole lane chunks, so every tile starts at a multiple of V
        // and the vector path serves cubes wider than one tile
        g.hx = (T + V - 1) / V * V;
        g.ox = RX - 2 * g.hx;
        if (g.ox < 1) return "x tile too narrow for t_block";
        g.ntx = (nx + g.ox - 1) / g.ox;
    }
    if (ny <= W * R) { g.nty = 1; g.oy = ny; }
    else {
        g.oy = W * R - 2 * T;
        if (g.oy < 1) return "too few rows for t_block (need waves * rows > 2 * t_block)";
        g.nty = (ny + g.oy - 1) / g.oy;
    }
    for (int k = 0; k < g.ntx; ++k) {
        int a, b;
        tile_cols(g, V, k, &a, &b);
        if (a % V || b <= a || b - a > g.ox) return "x tile split out of range";
    }
    for (int k = 0; k < g.nty; ++k) {
        int a, b;
        tile_rows(g, k, &a, &b);
        if (b <= a || b - a > g.oy) return "y tile split out of range";
    }
    // vector I/O: whole lane chunks (nx a multiple of V) and a tile's rows of
    // one plane below 2^30 bytes (the buffer offsets of the 16-bit kernels)
    g.vec = (nx % V == 0 && (long)W * R * nx * (long)dtype_size(p.dtype) < (1L << 30)) ? 1 : 0;
    pp->V = V;
    pp->T = T;
    auto& pcs = pp->pieces;
    pcs.clear();
    pp->first.clear();
    g.grouped = 0;
    const long ntiles = (long)g.ntx * g.nty;
    if (s.zchunk > 0) {
        const int nzc = (nz + s.zchunk - 1) / s.zchunk;
        if (ntiles * nzc > (1L << 30)) return "too many pieces";
        for (int tz = 0; tz < nzc; ++tz)
            for (int ty = 0; ty < g.nty; ++ty)
                for (int tx = 0; tx < g.ntx; ++tx)
                    pcs.push_back(Piece{tx, ty, tz * s.zchunk, std::min(nz, (tz + 1) * s.zchunk)});
        g.npieces = (int)pcs.size();
        return nullptr;
    }
    // balanced split: G pieces of (nearly) equal work, G a whole number of
    // rounds of the resident workgroups.  Every tile costs the same per plane
    // step: its wavefronts step through the planes together, a step takes as
    // long as its busiest SIMD, and tiles differ only by the few halo rows or
    // columns that fall outside the cube at its faces (a tile there computes
    // no fewer levels per step on its other rows).  So a piece's work is its
    // plane count, whatever its tile's outputs.
    const long slots = (long)ncu * resident_per_cu(W, lds);
    long rounds = s.rounds > 0 ? s.rounds : std::max<long>(1, (ntiles + slots - 1) / slots);
    long G = std::min<long>(slots * rounds, ntiles * (long)nz);
    if (G > (1L << 24)) return "too many pieces";
    std::vector<double> area(ntiles, 1.0);
    const double total = (double)ntiles;
    std::vector<int> cnt(ntiles);
    long used = 0;
    for (long i = 0; i < ntiles; ++i) {
        cnt[i] = (int)std::max<double>(1.0, std::min<double>(nz, std::floor(G * area[i] / total)));
        used += cnt[i];
    }
    while (used < G) {   // give the next piece to the tile with the most work per piece
        long best = -1;
        double bw = -1.0;
        for (long i = 0; i < ntiles; ++i)
            if (cnt[i] < nz && area[i] / cnt[i] > bw) { bw = area[i] / cnt[i]; best = i; }
        if (best < 0) break;
        ++cnt[best];
        ++used;
    }
    // When the tile count does not divide the workgroups (512 rows in 43
    // tiles of 16-row workgroups over 256 compute units: some tiles get 5
    // pieces of 102 planes, the others 6 of 85), the longest piece sets the
    // pass time.  Then each workgroup takes an equal share of the (tile,
    // plane) sequence instead, one or two pieces in turn, if that is cheaper
    // counting the halo planes every piece reloads.
    {
        double old_cost = 0.0, amax = 0.0;
        for (long i = 0; i < ntiles; ++i) {
            old_cost = std::max(old_cost, area[i] * ((nz + cnt[i] - 1) / cnt[i] + 3 * T));
            amax = std::max(amax, area[i]);
        }
        const double new_cost = (total * (nz + 3.0 * T) - 3.0 * T) / (double)G + 3.0 * T * amax;
        // grouped kernels exist for depths 1 and 2; cubes wider than one
        // tile keep the one-piece split, whose order keeps x neighbours'
        // halos on one L2 (grouping them measured slower)
        if (T <= 2 && g.ntx == 1 && used == G && new_cost < 0.97 * old_cost) {
            group_split(g, ntiles, G, T, pp);
            return nullptr;
        }
    }
    struct Item { Piece pc; double key; };
    std::vector<Item> items;
    items.reserve(used);
    for (long i = 0; i < ntiles; ++i) {
        const int tx = (int)(i % g.ntx), ty = (int)(i / g.ntx);
        for (int k = 0; k < cnt[i]; ++k) {
            const int z0 = (int)((long)k * nz / cnt[i]), z1 = (int)((long)(k + 1) * nz / cnt[i]);
            items.push_back(Item{Piece{tx, ty, z0, z1}, 0.5 * (z0 + z1)});
        }
    }
    // neighbouring pieces (same z range, adjacent tiles) next to each other ...
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
        const double qa = std::floor(a.key * 8.0 / nz), qb = std::floor(b.key * 8.0 / nz);
        if (qa != qb) return qa < qb;
        if (a.pc.ty != b.pc.ty) return a.pc.ty < b.pc.ty;
        return a.pc.tx < b.pc.tx;
    });
    // ... and each contiguous eighth of that order on one XCD: workgroups are
    // dispatched to the 8 XCDs round-robin, so XCD j runs workgroups j, j+8, ...
    const long n = (long)items.size();
    pcs.resize(n);
    if (n % 8 == 0) {
        const long per = n / 8;
        for (long j = 0; j < 8; ++j)
            for (long k = 0; k < per; ++k) pcs[8 * k + j] = items[j * per + k].pc;
    } else {
        for (long k = 0; k < n; ++k) pcs[k] = items[k].pc;
    }
    g.npieces = (int)pcs.size();
    return nullptr;
}

// Heuristic schedule when no tuned entry exists.
ig_schedule igk_auto_schedule(const ig_params* p) {
    ig_schedule s{};
    s.kind = IG_SCHED_BLOCKED;
    auto_vec_rows(p->nx, &s.vec, &s.rows);
    s.t_block = std::max(1, std::min(2, p->n_iter));
    // 12 wavefronts and one round of pieces: the fastest on gfx950 for the
    // 512^3 cube in every conductance and storage type (measured over
    // T 1..3, 8..16 wavefronts, 0..2 rounds)
    s.waves = 12;
    if (stream_lds_bytes(s.vec, s.t_block, s.waves) > kMaxLds) s.waves = 8;
    s.zchunk = 0;
    s.rounds = 1;
    // 16 wavefronts (four per SIMD, 12 output rows per tile) when their
    // workgroups take equal shares of the planes (grouped plan) and the
    // longest share, in plane steps times the measured cost of a 16-wave step
    // (2.96 us against 2.13 us for a 12-wave step on the 512^3 cube, T = 2,
    // 8 voxels per lane), is shorter: 512^3 runs 93 such steps against 134.
    // FP32 storage only: with 16-bit storage the 16-wave grouped pass measured
    // slower than 12 waves (bf16 840 against 871, fp16 851 against 873
    // Gvoxel-iter/s on the 512^3 cube).
    if (p->dtype == IG_F32 && s.t_block == 2 && s.vec == 8 && s.rows == 1 && p->nx % 8 == 0 && p->nx <= 512 &&
        (long)16 * p->nx * (long)dtype_size(p->dtype) < (1L << 30)) {
        auto longest = [&](int W, bool* grouped) -> double {
            ig_schedule t = s;
            t.waves = W;
            PassPlan pp;
            if (plan_pass(*p, t, 2, 256, &pp)) return 1e300;
            *grouped = !pp.first.empty();
            double m = 0.0;
            for (int b = 0; b < pp.workgroups(); ++b) {
                const int k0 = pp.first.empty() ? b : pp.first[b], k1 = pp.first.empty() ? b + 1 : pp.first[b + 1];
                double steps = 0.0;
                for (int k = k0; k < k1; ++k) steps += pp.pieces[k].z1 - pp.pieces[k].z0 + 6;
                m = std::max(m, steps);
            }
            return m;
        };
        bool g12 = false, g16 = false;
        const double t12 = longest(12, &g12), t16 = longest(16, &g16);
        if (g16 && 2.96 * t16 < 2.13 * t12) s.waves = 16;
    }
    if ((long)s.waves * s.rows * p->nx * (long)dtype_size(p->dtype) >= (1L << 30)) {   // absurdly long rows
        ig_schedule n{};
        n.kind = IG_SCHED_NAIVE;
        return n;
    }
    return s;
}

