// skis_internal.h -- host-side declarations shared by the libskis translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "skis.h"
#include "skis_device.h"

namespace skis {

// ---------------------------------------------------------------------------------
// Errors: every public entry point returns an int status and records a message.
// ---------------------------------------------------------------------------------
struct Error {
    int code;
    std::string msg;
};

void set_error(const std::string &msg);
const std::string &get_error();

#define SKIS_HIP_TRY(expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw ::skis::Error{SKIS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)};    \
    } while (0)

// ---------------------------------------------------------------------------------
// Device allocations, tracked against an optional byte cap.
// ---------------------------------------------------------------------------------
struct Arena {
    uint64_t cap = 0;   // 0 = unlimited (counts live and kept blocks)
    uint64_t used = 0;  // bytes currently held by live buffers
    uint64_t peak = 0;
    uint64_t kept = 0;  // bytes of released blocks kept for reuse
    hipStream_t stream = nullptr;              // allocations and releases are ordered on this stream
    std::unordered_map<void *, size_t> blocks; // every block the arena owns -> its size
    std::multimap<size_t, void *> free_blocks; // released blocks kept for reuse, by size
    std::unordered_set<void *> pooled_ptrs;    // blocks from the stream-ordered pool
    bool idle_on_destroy = false;              // set when no queued work can still use the blocks
    void *alloc(size_t bytes);
    void release(void *p, size_t bytes);
    // Gives the kept blocks back: with idle (no queued work on any stream can still touch
    // them) to the process-wide cache of idle device blocks, which later arenas reuse with no
    // driver call; otherwise to the device pool, in order on the arena's stream.
    void trim(bool idle = false);
    ~Arena();
};

template <typename T>
struct DevBuf {
    T *ptr = nullptr;
    size_t count = 0;
    Arena *arena = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { reset(); }
    void alloc(Arena &a, size_t n)
    {
        reset();
        arena = &a;
        count = n;
        ptr = (T *)a.alloc(sizeof(T) * (n ? n : 1));
    }
    void reset()
    {
        if (ptr && arena) arena->release(ptr, sizeof(T) * (count ? count : 1));
        ptr = nullptr;
        count = 0;
    }
    size_t bytes() const { return sizeof(T) * count; }
    void swap(DevBuf &o)
    {
        T *p = ptr;
        size_t c = count;
        Arena *a = arena;
        ptr = o.ptr;
        count = o.count;
        arena = o.arena;
        o.ptr = p;
        o.count = c;
        o.arena = a;
    }
};

// ---------------------------------------------------------------------------------
// The sketch object.
// ---------------------------------------------------------------------------------
struct Sketch {
    Arena arena;
    int32_t n = 0;
    uint64_t T = 0;
    uint64_t entries = 0;
    uint64_t probed_total = 0;
    uint64_t deferred = 0;
    uint64_t C = 0;
    double Gamma = 0.0;
    bool has_inverse = false;
    bool ris = false;             // plain RIS samples: estimates n * Cov / T, no q term
    DevBuf<double> q;             // [n]
    DevBuf<int64_t> sample_ptr;   // [T+1]
    DevBuf<int32_t> nodes;        // [entries]
    DevBuf<int32_t> roots;        // [T]
    DevBuf<uint64_t> probed;      // [T]
    DevBuf<int64_t> node_ptr;     // [n+1]
    DevBuf<int32_t> node_samples; // [entries]
    DevBuf<int32_t> owner;        // [entries] sample id of each entry; built for and consumed by the transpose
    DevBuf<int32_t> hot_id;       // [n] index in hot_node, or -1 (frequent nodes of the sketch)
    DevBuf<int32_t> hot_node;     // [nhot]
    int nhot = 0;
    double ms_preprocess = 0, ms_roots = 0, ms_sample = 0, ms_compact = 0, ms_inverse = 0;
    double ms_tier0 = 0, ms_tier1 = 0, ms_tier2 = 0, ms_tier3 = 0; // the sampler launches alone
    uint64_t deferred_global = 0;                    // samples that reached the HBM hash tier
    uint64_t deferred_bitmap = 0;                    // samples that reached the HBM bitmap tier
    uint32_t plain_levels = 0;                       // BFS level launches of the plain form
    uint32_t graph_replays = 0;                      // replays of the captured chain (captured form)
    uint64_t tier_stats[4][5] = {};                  // per sampler tier: samples, entries, edges probed,
                                                     // edges and nodes the tier's launch expanded
    // the estimator's scale and per-node term: Gamma and q for IIS (Eq. eq21), n and none
    // for RIS (Eq. ris_prob)
    double est_scale() const { return ris ? (double)n : Gamma; }
    const double *est_q() const { return ris ? nullptr : q.ptr; }
};

// ---------------------------------------------------------------------------------
// Preprocessing (rows a1-a3).
// ---------------------------------------------------------------------------------
// Diffusion models: independent cascade (Alg. 1) and linear threshold (Sec. 6)
enum : int { MODEL_IC = 0, MODEL_LT = 1 };

struct Prep {
    int model = MODEL_IC;
    DevBuf<int32_t> row_ptr;    // private copy [n+1]
    DevBuf<uint2> edges;        // interleaved (col, coin_threshold_hi(w)) per edge, padded with
                                // (0, 0) records to a multiple of four edges
    DevBuf<uint32_t> wbits;     // [m] w bits per edge (+0 for -0): coin ties and the roots' fallback
    DevBuf<double> P;           // [m] prefix products (IC) or running sums of w (LT)
    DevBuf<double> q;           // [n]
    DevBuf<uint64_t> W;         // [n]
    DevBuf<AliasEntry> alias;   // [n]
    uint64_t C = 0;
    double Gamma = 0.0;
};

// Validates the graph, copies row_ptr, interleaves (col, coin threshold), keeps the w bits,
// computes P, q, W, C, Gamma and (if build_alias) the alias table.  Throws Error on failure.
void preprocess(Arena &arena, int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                const float *w, bool build_alias, Prep &out, hipStream_t s, int model = MODEL_IC);

// ---------------------------------------------------------------------------------
// Sampling (rows a4-a7, a11) and compaction.
// ---------------------------------------------------------------------------------
struct SampleConfig {
    uint32_t form = 0;
    uint32_t threads = 64;
    uint32_t slots = 4;
    uint32_t visited = 192;
    uint32_t big_row = 16384;
    uint64_t staging_entries = 0;
    uint64_t chunk = 0; // captured form: samples per replay of the chain (0: 2^24)
    uint32_t qpl = 1;   // edge quads per lane per sweep in the first tier
    bool owners = false; // also write the sample id of every entry (Sketch::owner) for the transpose
    bool ris = false;    // plain RIS samples (uniform root, no conditioning) instead of IIS
    uint64_t first_id = 0; // sample i of the build is sample id first_id + i of the stream
    int model = MODEL_IC;  // MODEL_LT: the linear threshold sampler (Sec. 6); prep must match
};

void sample_and_compact(Arena &arena, const Prep &prep, int32_t n, int64_t m, uint64_t T, uint64_t seed,
                        const SampleConfig &cfg, Sketch &sk, hipStream_t s);

void build_inverse(Sketch &sk, hipStream_t s);

// Cuts a built sketch, before its transpose, to the smallest number of leading samples whose
// sizes sum to at least budget.
void truncate_to_budget(Sketch &sk, uint64_t budget, hipStream_t s);

// node_ptr[n+1] and node_samples[N] (each list ascending) of the N-entry sketch.
// owner: the sample id of every entry (written by the compaction), or null to have them
// computed here; its contents are overwritten.  deg[n] receives each node's entry count.
void radix_transpose(Arena &arena, const int64_t *sample_ptr, const int32_t *nodes, int32_t *owner, uint64_t T,
                     uint64_t N, int32_t n, int64_t *node_ptr, int32_t *node_samples, uint32_t *deg, hipStream_t s);

// ---------------------------------------------------------------------------------
// Device-wide scans (exclusive), T in {uint32_t, uint64_t, int64_t, u128}.
// ---------------------------------------------------------------------------------
template <typename T>
void excl_scan(Arena &arena, const T *in, T *out, int64_t n, T *d_total, hipStream_t s);
void excl_scan_u32_to_i64(Arena &arena, const uint32_t *in, int64_t *out, int64_t n, int64_t *d_total,
                          hipStream_t s);

// Launch-shape helper: number of compute units of the current device.
int device_cu_count();

// A second stream of the current device (non-blocking, default priority, created once and kept
// until the process ends) for work that runs beside the caller's stream between an event
// recorded on it and one the caller's stream waits on.
hipStream_t side_stream();

// Random-read probe (measurement aid): `reads` uniformly random rows of row_bytes bytes
// from a table of `rows` rows, stream-ordered on s; sink is one device word it almost never
// writes.
void probe_random_read(const void *table, uint64_t rows, uint32_t row_bytes, uint64_t reads, uint32_t seed,
                       uint32_t *sink, hipStream_t s);

} // namespace skis
