// skis_query.h -- declarations of the query kernels' host launchers.
#pragma once
#include <mutex>

#include "skis_internal.h"

namespace skis {

constexpr int EST_BLOCK = 1024;   // threads per query in k_estimate
constexpr int EST_MAX_SET = 4096; // largest seed set one estimate workgroup holds in LDS
constexpr int EST_WALK = 4;       // sample-list entries a thread walks per round, loads issued together

constexpr int GREEDY_HOT = 2048;  // hot nodes decremented in LDS

struct GreedyState {
    unsigned done;              // blocks of k_greedy_argmax that have finished
    int32_t vstar;              // this round's pick (-1: none left)
    unsigned shrunk;            // a heavy round has cut the lists down (they are in the work copy)
    int32_t cur;                // which of the two delta buffers holds the current counts
    unsigned long long dstar;   // delta of this round's pick: the samples it newly covers
    unsigned long long cov;     // coverage of the picks so far
    double est;
};

// One recount work item: entries [p0, p0 + len) of node v's list.
struct RecountItem {
    int64_t p0;
    int32_t len;
    int32_t v;
};

// Per-sketch scratch for estimate: one bitmap of T bits per query in flight.
struct QueryScratch {
    DevBuf<uint32_t> bitmaps;
    uint64_t bitmap_words = 0;
    DevBuf<int> err;
};

void estimate_batch(const Sketch &sk, QueryScratch &qs, int32_t Q, const int64_t *set_ptr, const int32_t *set_nodes,
                    uint64_t *cov, double *est, hipStream_t s);
// One launch pair for nq sets in CSR form on the device (set_ptr from 0): the sets of at
// most EST_MAX_SET entries take a workgroup each; the nlarge sets listed in large[] (device
// indexes into the CSR) take the chunked path with one node bitmap of n bits each in
// nodebits.  bitmaps holds a zeroed bitmap of bitmap_words words for every workgroup
// (max(nq, nlarge) of them) and is left zeroed.  Stream-ordered; no host synchronisation.
void estimate_launch(const Sketch &sk, int32_t nq, const int64_t *set_ptr, const int32_t *set_nodes,
                     const int64_t *large, int32_t nlarge, uint32_t *bitmaps, uint64_t bitmap_words,
                     uint32_t *nodebits, unsigned long long *cov, double *est, int *err, hipStream_t s);
// The two launches of estimate_launch on their own: sets q0 .. q0+nq-1 of the CSR (those of
// at most EST_MAX_SET entries; set q0+b uses bitmap b), and the ng large sets listed in
// qlist[g0 .. g0+ng) (set qlist[g0+b] uses bitmap b and node bitmap b).  Stream-ordered.
void estimate_launch_small(const Sketch &sk, int64_t q0, int32_t nq, const int64_t *set_ptr,
                           const int32_t *set_nodes, uint32_t *bitmaps, uint64_t bitmap_words,
                           unsigned long long *cov, double *est, int *err, hipStream_t s);
void estimate_launch_large(const Sketch &sk, const int64_t *qlist, int64_t g0, int32_t ng, const int64_t *set_ptr,
                           const int32_t *set_nodes, uint32_t *bitmaps, uint64_t bitmap_words, uint32_t *nodebits,
                           unsigned long long *cov, double *est, int *err, hipStream_t s);
// Zero-fills count words with a kernel (capturable, unlike a memset node).
void fill_u32(uint32_t *p, uint64_t count, hipStream_t s);
void greedy(const Sketch &sk, QueryScratch &qs, int32_t k, int32_t *seeds, uint64_t *marg, uint64_t *cov_out,
            double *est_out, hipStream_t s);

} // namespace skis

// The opaque handle of the C ABI: the sketch, its estimate scratch, and a lock that
// serialises the calls that use that scratch.
struct skis_sketch {
    skis::Sketch core;
    skis::QueryScratch qs;
    std::mutex mu;
};
