// Batched filter entry points (persistent launch); see include/igfilter.h.
#include <hip/hip_runtime.h>

#include "igfilter.h"

extern "C" ig_status ig_filter_batch(const ig_batch_item*, int32_t, int, void*, ig_stats*, double*) {
    return IG_ERR_UNSUPPORTED;
}
extern "C" void ig_batch_cache_clear(void) {}
