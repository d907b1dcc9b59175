// skis_query.h -- declarations of the query kernels' host launchers.
#pragma once
#include "skis_internal.h"

namespace skis {

constexpr int EST_BLOCK = 256;    // threads per query in k_estimate
constexpr int EST_MAX_SET = 4096; // largest seed set one estimate workgroup holds in LDS

constexpr int GREEDY_HOT = 2048;  // hot nodes decremented in LDS

struct GreedyState {
    unsigned done;              // blocks of k_greedy_argmax that have finished
    int32_t vstar;              // this round's pick (-1: none left)
    unsigned long long listed;  // samples newly covered this round
    unsigned long long cov;     // coverage of the picks so far
    double est;
};

// Per-sketch scratch for estimate: one bitmap of T bits per query in flight.
struct QueryScratch {
    DevBuf<uint32_t> bitmaps;
    uint64_t bitmap_words = 0;
    DevBuf<int> err;
};

void estimate_batch(const Sketch &sk, QueryScratch &qs, int32_t Q, const int64_t *set_ptr, const int32_t *set_nodes,
                    uint64_t *cov, double *est, hipStream_t s);
void greedy(const Sketch &sk, QueryScratch &qs, int32_t k, int32_t *seeds, uint64_t *marg, uint64_t *cov_out,
            double *est_out, hipStream_t s);

} // namespace skis
