// skis_plain.h -- the plain (one launch per BFS level) form of the sampler.
#pragma once
#include "skis_internal.h"

namespace skis {

struct PlainInputs {
    uint32_t count;                 // samples 0..count-1
    const int32_t *row_ptr;
    const uint4 *pairs;             // edge records two at a time, padded to whole quads
    int64_t nquads;
    const uint32_t *wbits;          // w bits per edge
    const int4 *rec;
    const int32_t *u1;
    uint32_t seed_lo, seed_hi;
    uint64_t first_id;              // sample i of the chunk series is sample id first_id + i
    uint64_t expected_size;         // expected |R_j|, sizes the chunk buffers
    DevBuf<int32_t> *staging;       // grown (contents kept) when a chunk does not fit
    uint32_t *out_size;
    unsigned long long *out_off;
    unsigned long long *out_probed;
    uint32_t *medium;
    unsigned long long *n_medium;
    int small_sort;
};

struct PlainOutputs {
    uint64_t entries = 0;
    uint32_t levels = 0;            // BFS levels launched, over all chunks
};

void sample_plain(Arena &arena, const PlainInputs &in, PlainOutputs &out, hipStream_t s);

} // namespace skis
