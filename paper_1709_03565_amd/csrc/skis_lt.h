// skis_lt.h -- the IIS sampler of the linear threshold model (Sec. 6).
#pragma once
#include "skis_internal.h"

namespace skis {

struct LtIo {
    uint32_t count = 0;                 // samples 0..count-1 of the build
    uint64_t first_id = 0;              // sample i is sample id first_id + i of the stream
    uint32_t seed_lo = 0, seed_hi = 0;
    int4 *rec = nullptr;                // rec[i].x = root of sample i
    uint32_t *out_size = nullptr;       // |R_i|
    unsigned long long *out_off = nullptr;    // R_i's nodes (walk order) at staging[out_off[i]]
    unsigned long long *out_probed = nullptr; // sum of the in-degrees of R_i's nodes
    uint32_t *medium = nullptr;         // samples above small_sort nodes, listed for compaction
    unsigned long long *n_medium = nullptr;
    int small_sort = 0;
    DevBuf<int32_t> *staging = nullptr; // (re)allocated here
    uint64_t staging_entries = 0;       // first capacity (0: from count)
};

struct LtStats {
    uint64_t walk_samples = 0, walk_entries = 0, walk_probed = 0, walk_picks = 0;
    uint64_t long_samples = 0, long_entries = 0, long_probed = 0, long_picks = 0;
    float ms_walk = 0, ms_long = 0;
};

// Samples the count LT-IIS samples of io into staging, with their sizes, offsets, probed
// counts and roots; prep must come from preprocess(..., MODEL_LT) with its alias table.
void sample_lt(Arena &arena, const Prep &prep, int32_t n, const LtIo &io, LtStats &st, hipStream_t s);

} // namespace skis
