// Randomised exercise of the library's host planner and parameter validation
// (paper_1609_03782_amd/csrc/plan.cpp), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_cpu.py.  Besides running
// clean under the sanitizers, every plan must cover each output plane of each
// tile exactly once, and every rejected request must say why.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "plan.h"

static int failures = 0;
#define CHECK(cond, ...)                        \
    do {                                        \
        if (!(cond)) {                          \
            std::fprintf(stderr, __VA_ARGS__);  \
            std::fprintf(stderr, "\n");         \
            ++failures;                         \
        }                                       \
    } while (0)

static ig_params random_params(std::mt19937_64& rng, bool valid) {
    std::uniform_int_distribution<int> small(1, 300), tiny(1, 9), kind(0, 9);
    ig_params p{};
    p.struct_size = sizeof(ig_params);
    p.dtype = (int)(rng() % 3);
    p.cond = (int)(rng() % 3);
    p.n_iter = (int)(rng() % 60);
    const int shape_kind = kind(rng);
    p.nx = shape_kind < 3 ? tiny(rng) : small(rng) * (shape_kind == 9 ? 7 : 1);
    p.ny = shape_kind == 4 ? tiny(rng) : small(rng);
    p.nz = shape_kind == 5 ? tiny(rng) : small(rng) / 2 + 1;
    p.K = 0.25f + (float)(rng() % 1000) / 100.0f;
    p.tau = (float)(rng() % 100) / 1000.0f;
    for (int a = 0; a < 3; ++a) p.C[a] = (float)(rng() % 60) / 10.0f;
    p.rms = (rng() % 2) ? 0.0 : 1.5;
    if (!valid) {
        switch (rng() % 10) {
            case 0: p.nx = -(int64_t)(rng() % 5); break;
            case 1: p.K = NAN; break;
            case 2: p.tau = -1.0f; break;
            case 3: p.C[rng() % 3] = INFINITY; break;
            case 4: p.struct_size = 3; break;
            case 5: p.dtype = 9; break;
            case 6: p.cond = -2; break;
            case 7: p.n_iter = -3; break;
            case 8: p.reserved0 = 1.0f; break;
            default: p.nx = p.ny = p.nz = 1 << 11; break;   // 2^33 voxels
        }
    }
    return p;
}

// Every plane [0, nz) of every tile of the grid output by exactly one piece.
static void check_cover(const ig_params& p, const PassPlan& pp, const char* what) {
    const igk::BlockGeom& g = pp.g;
    CHECK(g.ntx >= 1 && g.nty >= 1 && g.ox >= 1 && g.oy >= 1, "%s: empty grid", what);
    CHECK((long)g.ntx * g.ox >= p.nx && (long)(g.ntx - 1) * g.ox < p.nx, "%s: x tiles %d x %d for nx %lld", what,
          g.ntx, g.ox, (long long)p.nx);
    CHECK((long)g.nty * g.oy >= p.ny && (long)(g.nty - 1) * g.oy < p.ny, "%s: y tiles %d x %d for ny %lld", what,
          g.nty, g.oy, (long long)p.ny);
    std::vector<int> seen((size_t)g.ntx * g.nty * p.nz, 0);
    for (const igk::Piece& pc : pp.pieces) {
        CHECK(pc.tx >= 0 && pc.tx < g.ntx && pc.ty >= 0 && pc.ty < g.nty && pc.z0 >= 0 && pc.z0 < pc.z1 &&
                  pc.z1 <= p.nz,
              "%s: bad piece (%d %d %d %d)", what, pc.tx, pc.ty, pc.z0, pc.z1);
        if (!(pc.tx >= 0 && pc.tx < g.ntx && pc.ty >= 0 && pc.ty < g.nty && pc.z0 >= 0 && pc.z1 <= p.nz)) continue;
        for (int z = pc.z0; z < pc.z1; ++z) ++seen[((size_t)z * g.nty + pc.ty) * g.ntx + pc.tx];
    }
    for (size_t i = 0; i < seen.size(); ++i)
        if (seen[i] != 1) {
            CHECK(false, "%s: plane-tile %zu covered %d times", what, i, seen[i]);
            break;
        }
}

int main(int argc, char** argv) {
    const unsigned long long seed = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1;
    const int iters = argc > 2 ? std::atoi(argv[2]) : 2000;
    std::mt19937_64 rng(seed);
    int planned = 0, rejected = 0;
    for (int it = 0; it < iters; ++it) {
        const bool valid = rng() % 4 != 0;
        ig_params p = random_params(rng, valid);
        const ig_status st = igk_validate_params(&p);
        if (!valid) {
            CHECK(st == IG_ERR_INVALID_ARG, "invalid params accepted (iteration %d)", it);
            CHECK(std::strlen(ig_last_error()) > 0, "rejection without a message");
            continue;
        }
        CHECK(st == IG_OK, "valid params rejected: %s", ig_last_error());
        if (st != IG_OK || p.nx * p.ny * p.nz > 4000000) continue;
        const ig_schedule a = igk_auto_schedule(&p);
        CHECK(a.kind == IG_SCHED_BLOCKED || a.kind == IG_SCHED_NAIVE, "auto schedule kind %d", a.kind);
        ig_schedule s{};
        s.kind = IG_SCHED_BLOCKED;
        s.t_block = 1 + (int)(rng() % 4);
        s.waves = 1 + (int)(rng() % 16);
        s.zchunk = (rng() % 2) ? 0 : 1 + (int)(rng() % 70);
        s.vec = (int)(rng() % 5) == 4 ? 0 : 1 << (rng() % 4);
        s.rounds = (int)(rng() % 3);
        s.rows = (int)(rng() % 3) == 2 ? 0 : 1 << (rng() % 3);
        const int ncu = 1 + (int)(rng() % 300);
        for (int T = 1; T <= s.t_block; ++T) {
            PassPlan pp;
            const char* why = plan_pass(p, s, T, ncu, &pp);
            if (why) {
                CHECK(std::strlen(why) > 0, "empty reason");
                ++rejected;
                break;
            }
            ++planned;
            check_cover(p, pp, "plan_pass");
        }
        if (a.kind == IG_SCHED_BLOCKED) {
            PassPlan pp;
            const char* why = plan_pass(p, a, a.t_block, 256, &pp);
            CHECK(!why, "automatic schedule cannot plan: %s", why ? why : "");
            if (!why) check_cover(p, pp, "auto");
        }
    }
    std::printf("host_fuzz seed %llu: %d iterations, %d passes planned, %d schedules rejected, %d failures\n", seed,
                iters, planned, rejected, failures);
    return failures ? 1 : 0;
}
