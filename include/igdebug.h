/*
 * igdebug.h - test hooks of libigfilter: injected allocation failures and a
 * count of the library's live allocations, for checking that every entry
 * point that allocates reports IG_ERR_OUT_OF_MEMORY when an allocation fails
 * and leaks nothing.  Not for production use.
 *
 * Every device allocation of the library (and the pinned host table of a
 * batch plan) goes through one counting wrapper.  The environment variable
 * IG_FAULT_INJECT=alloc[:N] makes the N-th such allocation after the library
 * loads fail (N = 1 when omitted), as ig_debug_fail_alloc(N) does at run time.
 */
#ifndef IGDEBUG_H
#define IGDEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The nth allocation from now (1 = the next one) fails with out-of-memory,
 * once; nth <= 0 cancels a pending failure.  Host only; process-wide. */
void ig_debug_fail_alloc(int64_t nth);

/* Allocations of the library alive now (made and not yet freed).  Host only. */
int64_t ig_debug_live_allocations(void);

/* Free the library's process-lifetime caches (the reduction scratch of
 * ig_compare / ig_reduce of the calling thread, the per-device scratch of
 * ig_quality, every cached batch plan) after the work using them has
 * finished; later calls allocate them again. */
void ig_debug_release_caches(void);

/* Largest piece ig_surrogate_infer runs in one pass, in voxels (larger cubes
 * are cut into slabs or tiles with a halo of the network's depth, which gives
 * the same result bit for bit); voxels <= 0 restores the default, 2^28.
 * Returns the previous limit.  Host only; process-wide: lets tests exercise
 * the tiled path on small cubes. */
int64_t ig_debug_set_infer_piece_limit(int64_t voxels);

#ifdef __cplusplus
}
#endif
#endif /* IGDEBUG_H */
