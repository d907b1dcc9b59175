// skis_api.cpp -- the extern "C" entry points of libskis (declared in include/skis.h):
// argument checks, allocation accounting, error reporting and the order of the stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "skis_internal.h"
#include "skis_query.h"


namespace skis {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
const std::string &get_error() { return g_err; }

// Limits on the memory kept for reuse (the pool's release threshold and the idle-block cache
// below).  Unless the caller sets them, each is half the device's memory: one build of 2^26
// samples at 1.4B edges allocates about 100 GB of transient buffers, and with smaller limits
// every build handed part of them back to the driver and mapped them again (150 ms a build
// once another process had used that memory, which the driver then clears first).
constexpr uint64_t KEEP_UNSET = ~0ull;
constexpr int CACHE_DEVICES = 64;
static std::atomic<uint64_t> g_pool_keep{KEEP_UNSET};
static std::atomic<uint64_t> g_cache_keep{KEEP_UNSET};

static uint64_t keep_limit(const std::atomic<uint64_t> &limit, int d)
{
    const uint64_t set = limit.load();
    if (set != KEEP_UNSET) return set;
    static std::atomic<uint64_t> half[CACHE_DEVICES];
    const int k = d >= 0 && d < CACHE_DEVICES ? d : 0;
    uint64_t h = half[k].load();
    if (h == 0) {
        size_t total = 0;
        if (hipDeviceTotalMem(&total, d) != hipSuccess || total == 0) total = 64ull << 30;
        (void)hipGetLastError();
        h = (uint64_t)total / 2;
        half[k].store(h);
    }
    return h;
}

// Stream-ordered allocation from the device's default memory pool, which keeps up to its
// release threshold of released memory for reuse: a build then takes its buffers from what the
// previous one released instead of going back to the driver.  Buffers are released on the
// arena's stream, after the work queued there that uses them.

static bool pool_ready()
{
    static thread_local int ready_dev = -1;
    static thread_local bool ok = false;
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return false;
    if (d != ready_dev) {
        ready_dev = d;
        int supported = 0;
        ok = hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, d) == hipSuccess && supported;
        if (ok) {
            hipMemPool_t pool = nullptr;
            uint64_t keep = keep_limit(g_pool_keep, d);
            ok = hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess &&
                 hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess;
        }
        (void)hipGetLastError();
    }
    return ok;
}

// Idle device blocks shared by every arena of the process (per device, up to the cache limit):
// a block enters only when no queued work can use it any more (after a stream or device
// synchronisation), so an arena on any stream may take it as it is.  Taking one costs no
// driver call; the stream-ordered free and allocation cost tens to hundreds of microseconds of
// host time each.

struct CachedBlock {
    void *p;
    bool pooled;
};

struct BlockCache {
    std::mutex mu;
    std::multimap<size_t, CachedBlock> blocks; // by size
    uint64_t bytes = 0;
};

static BlockCache &block_cache(int dev)
{
    static BlockCache caches[CACHE_DEVICES];
    return caches[dev >= 0 && dev < CACHE_DEVICES ? dev : 0];
}

static void free_block(void *p, bool pooled)
{
    if (pooled) (void)hipFreeAsync(p, nullptr);
    else (void)hipFree(p);
}

// an idle block of at least need and at most 2 * need bytes, or nullptr
static void *cache_take(size_t need, size_t *size, bool *pooled)
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= CACHE_DEVICES) return nullptr;
    BlockCache &c = block_cache(d);
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.blocks.lower_bound(need);
    if (it == c.blocks.end() || it->first > 2 * need) return nullptr;
    void *p = it->second.p;
    *size = it->first;
    *pooled = it->second.pooled;
    c.bytes -= it->first;
    c.blocks.erase(it);
    return p;
}

static void cache_put(void *p, size_t size, bool pooled)
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= CACHE_DEVICES) {
        free_block(p, pooled);
        return;
    }
    const uint64_t keep = keep_limit(g_cache_keep, d);
    if (size > keep) {
        free_block(p, pooled);
        return;
    }
    BlockCache &c = block_cache(d);
    std::lock_guard<std::mutex> lk(c.mu);
    c.blocks.emplace(size, CachedBlock{p, pooled});
    c.bytes += size;
    while (c.bytes > keep) { // the largest blocks leave first
        auto it = std::prev(c.blocks.end());
        c.bytes -= it->first;
        free_block(it->second.p, it->second.pooled);
        c.blocks.erase(it);
    }
}

// Frees idle blocks of the current device's cache, largest first, until it holds at most keep bytes.
static void trim_idle_cache(uint64_t keep)
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= CACHE_DEVICES) return;
    BlockCache &c = block_cache(d);
    std::lock_guard<std::mutex> lk(c.mu);
    while (c.bytes > keep && !c.blocks.empty()) {
        auto it = std::prev(c.blocks.end());
        c.bytes -= it->first;
        free_block(it->second.p, it->second.pooled);
        c.blocks.erase(it);
    }
}

// Under memory pressure: every idle block of this device's cache goes back, and the
// stream-ordered pool gives what it holds back to the device (after the device is idle), so
// that a failed allocation can be retried on memory the process is only keeping.
static void release_idle_memory()
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= CACHE_DEVICES) return;
    (void)hipDeviceSynchronize();
    {
        BlockCache &c = block_cache(d);
        std::lock_guard<std::mutex> lk(c.mu);
        for (auto &b : c.blocks) free_block(b.second.p, b.second.pooled);
        c.blocks.clear();
        c.bytes = 0;
    }
    (void)hipDeviceSynchronize();
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    (void)hipGetLastError();
}

// A released block is kept and handed to a later request of at least half its size: the
// stages of one build (sampler, compaction, transpose) allocate and release buffers of a few
// GB each, and reusing them avoids a driver call per buffer.  Kept blocks go back to the
// pool when the build ends (trim) and when the arena dies.
void *Arena::alloc(size_t bytes)
{
    const size_t need = bytes ? bytes : 1;
    auto it = free_blocks.lower_bound(need);
    if (it != free_blocks.end() && it->first <= 2 * need) {
        void *p = it->second;
        kept -= it->first;
        free_blocks.erase(it);
        used += bytes;
        peak = std::max(peak, used);
        return p;
    }
    if (cap && used + kept + need > cap) trim();
    if (cap && used + need > cap)
        throw Error{SKIS_ENOMEM, "max_device_bytes exceeded: " + std::to_string(used + need) + " > " +
                                     std::to_string(cap)};
    {
        size_t size = 0;
        bool pooled = false;
        if (void *p = cache_take(need, &size, &pooled)) {
            if (pooled) pooled_ptrs.insert(p);
            blocks[p] = size;
            used += bytes;
            peak = std::max(peak, used);
            return p;
        }
    }
    void *p = nullptr;
    const bool pooled = pool_ready();
    hipError_t e = pooled ? hipMallocAsync(&p, need, stream) : hipMalloc(&p, need);
    if (e != hipSuccess) { // give the kept and the idle blocks back and try once more
        (void)hipGetLastError();
        trim();
        release_idle_memory();
        e = pooled ? hipMallocAsync(&p, need, stream) : hipMalloc(&p, need);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{SKIS_ENOMEM, "device allocation of " + std::to_string(need) + " bytes failed: " +
                                     hipGetErrorString(e)};
    }
    if (pooled) pooled_ptrs.insert(p);
    blocks[p] = need;
    used += bytes;
    peak = std::max(peak, used);
    return p;
}

void Arena::release(void *p, size_t bytes)
{
    used -= bytes;
    auto it = blocks.find(p);
    if (it == blocks.end()) return;
    free_blocks.emplace(it->second, p);
    kept += it->second;
}

void Arena::trim(bool idle)
{
    for (auto &fb : free_blocks) {
        void *p = fb.second;
        const bool pooled = pooled_ptrs.erase(p) > 0;
        if (idle) cache_put(p, fb.first, pooled);
        else if (pooled) (void)hipFreeAsync(p, stream);
        else (void)hipFree(p);
        blocks.erase(p);
    }
    free_blocks.clear();
    kept = 0;
}

Arena::~Arena() { trim(idle_on_destroy); }

hipStream_t side_stream()
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int d = 0;
    SKIS_HIP_TRY(hipGetDevice(&d));
    if (d < 0 || d >= 64) throw Error{SKIS_EHIP, "device index out of range"};
    std::lock_guard<std::mutex> lk(mu);
    if (!streams[d]) SKIS_HIP_TRY(hipStreamCreateWithFlags(&streams[d], hipStreamNonBlocking));
    return streams[d];
}

int device_cu_count()
{
    static thread_local int cached_dev = -1, cached_cus = 0;
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return 1;
    if (d != cached_dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || cus < 1) cus = 1;
        cached_cus = cus;
        cached_dev = d;
    }
    return cached_cus;
}

} // namespace skis

template <class F>
static int guarded(F &&f)
{
    try {
        skis::set_error("");
        return f();
    } catch (const skis::Error &e) {
        skis::set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        skis::set_error("host allocation failed");
        return SKIS_ENOMEM;
    } catch (const std::exception &e) {
        skis::set_error(e.what());
        return SKIS_EHIP;
    }
}

static void check_graph_args(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w)
{
    if (n <= 0) throw skis::Error{SKIS_EINVAL, "n must be positive"};
    if (m < 0 || m > (int64_t)INT32_MAX) throw skis::Error{SKIS_EINVAL, "m must be in [0, 2^31)"};
    if (!row_ptr || (m > 0 && (!col || !w))) throw skis::Error{SKIS_EINVAL, "graph pointers must not be NULL"};
}

extern "C" {

void skis_default_options(skis_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->form = 0;
    opt->slots_per_block = 4;
    opt->visited_threshold = 192;
    opt->threads_per_block = 64;
    opt->big_row = 16384;
    opt->build_inverse_index = 1;
    opt->max_device_bytes = 0;
    opt->staging_entries = 0;
    opt->chunk_samples = 0;
    opt->quads_per_lane = 1;
}

static int preprocess_model(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                            double *P, double *q, uint64_t *W, uint64_t *thr, int32_t *alias, uint64_t *C_out,
                            double *Gamma_out, hipStream_t stream, int model)
{
    return guarded([&]() -> int {
        check_graph_args(n, m, row_ptr, col, w);
        skis::Arena arena;
        arena.stream = stream;
        skis::Prep prep;
        skis::preprocess(arena, n, m, row_ptr, col, w, thr || alias, prep, stream, model);
        if (P && m > 0)
            SKIS_HIP_TRY(hipMemcpyAsync(P, prep.P.ptr, sizeof(double) * (size_t)m, hipMemcpyDeviceToDevice, stream));
        if (q) SKIS_HIP_TRY(hipMemcpyAsync(q, prep.q.ptr, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, stream));
        if (W) SKIS_HIP_TRY(hipMemcpyAsync(W, prep.W.ptr, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, stream));
        if (prep.C > 0) {
            if (thr)
                SKIS_HIP_TRY(hipMemcpy2DAsync(thr, sizeof(uint64_t), prep.alias.ptr, sizeof(skis::AliasEntry),
                                              sizeof(uint64_t), (size_t)n, hipMemcpyDeviceToDevice, stream));
            if (alias)
                SKIS_HIP_TRY(hipMemcpy2DAsync(alias, sizeof(int32_t),
                                              reinterpret_cast<const char *>(prep.alias.ptr) + sizeof(uint64_t),
                                              sizeof(skis::AliasEntry), sizeof(int32_t), (size_t)n,
                                              hipMemcpyDeviceToDevice, stream));
        }
        SKIS_HIP_TRY(hipStreamSynchronize(stream));
        arena.idle_on_destroy = true; // the synchronisation above ended every use of the blocks
        if (C_out) *C_out = prep.C;
        if (Gamma_out) *Gamma_out = prep.Gamma;
        return prep.C == 0 ? SKIS_WDEGENERATE : SKIS_OK;
    });
}

int skis_preprocess(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w, double *P,
                    double *q, uint64_t *W, uint64_t *thr, int32_t *alias, uint64_t *C_out, double *Gamma_out,
                    hipStream_t stream)
{
    return preprocess_model(n, m, row_ptr, col, w, P, q, W, thr, alias, C_out, Gamma_out, stream, skis::MODEL_IC);
}

int skis_preprocess_lt(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w, double *S,
                       double *q, uint64_t *W, uint64_t *thr, int32_t *alias, uint64_t *C_out, double *Gamma_out,
                       hipStream_t stream)
{
    return preprocess_model(n, m, row_ptr, col, w, S, q, W, thr, alias, C_out, Gamma_out, stream, skis::MODEL_LT);
}

int skis_build_sketch(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                      uint64_t num_samples, uint64_t seed, const skis_options *opt_in, hipStream_t stream,
                      skis_sketch **out)
{
    return guarded([&]() -> int {
        if (!out) throw skis::Error{SKIS_EINVAL, "out must not be NULL"};
        *out = nullptr;
        check_graph_args(n, m, row_ptr, col, w);
        if (num_samples == 0) throw skis::Error{SKIS_EINVAL, "num_samples must be positive"};
        if (num_samples > (uint64_t)INT32_MAX)
            throw skis::Error{SKIS_EINVAL, "num_samples must be below 2^31 (sample ids are 32-bit)"};
        skis_options opt;
        skis_default_options(&opt);
        if (opt_in) {
            opt.form = opt_in->form;
            if (opt_in->slots_per_block) opt.slots_per_block = opt_in->slots_per_block;
            if (opt_in->visited_threshold) opt.visited_threshold = opt_in->visited_threshold;
            if (opt_in->big_row) opt.big_row = opt_in->big_row;
            if (opt_in->threads_per_block) opt.threads_per_block = opt_in->threads_per_block;
            opt.build_inverse_index = opt_in->build_inverse_index;
            opt.max_device_bytes = opt_in->max_device_bytes;
            opt.staging_entries = opt_in->staging_entries;
            opt.chunk_samples = opt_in->chunk_samples;
            if (opt_in->quads_per_lane) opt.quads_per_lane = opt_in->quads_per_lane;
            opt.ris_mode = opt_in->ris_mode;
            opt.entry_budget = opt_in->entry_budget;
            opt.model = opt_in->model;
        }
        if (opt.ris_mode > 1) throw skis::Error{SKIS_EINVAL, "ris_mode must be 0 or 1"};
        if (opt.model > 1) throw skis::Error{SKIS_EINVAL, "model must be 0 (independent cascade) or 1 (linear threshold)"};
        if (opt.model == 1 && (opt.ris_mode || opt.form != 0))
            throw skis::Error{SKIS_EINVAL, "the linear threshold sampler has the persistent form only and no RIS mode"};
        if (opt.form > 2) throw skis::Error{SKIS_EINVAL, "unknown sampler form"};
        skis_sketch *h = new skis_sketch;
        try {
            skis::Sketch &sk = h->core;
            sk.arena.cap = opt.max_device_bytes;
            sk.arena.stream = stream;
            sk.n = n;
            hipEvent_t e0, e1;
            SKIS_HIP_TRY(hipEventCreate(&e0));
            SKIS_HIP_TRY(hipEventCreate(&e1));
            SKIS_HIP_TRY(hipEventRecord(e0, stream));
            int status = SKIS_OK;
            {
                skis::Prep prep;
                skis::preprocess(sk.arena, n, m, row_ptr, col, w, true, prep, stream, (int)opt.model);
                SKIS_HIP_TRY(hipEventRecord(e1, stream));
                SKIS_HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                SKIS_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                sk.ms_preprocess = ms;
                sk.Gamma = prep.Gamma;
                sk.C = prep.C;
                sk.ris = opt.ris_mode != 0;
                if (prep.C == 0 && !sk.ris) {
                    status = SKIS_WDEGENERATE;
                    sk.T = 0;
                    sk.sample_ptr.alloc(sk.arena, 1);
                    SKIS_HIP_TRY(hipMemsetAsync(sk.sample_ptr.ptr, 0, sizeof(int64_t), stream));
                } else {
                    skis::SampleConfig cfg;
                    cfg.form = opt.form;
                    cfg.threads = opt.threads_per_block;
                    cfg.slots = opt.slots_per_block;
                    cfg.visited = opt.visited_threshold;
                    cfg.big_row = opt.big_row;
                    cfg.staging_entries = opt.staging_entries;
                    cfg.chunk = opt.chunk_samples;
                    cfg.qpl = opt.quads_per_lane;
                    cfg.owners = opt.build_inverse_index != 0;
                    cfg.ris = sk.ris;
                    cfg.model = (int)opt.model;
                    if (!opt.entry_budget) {
                        skis::sample_and_compact(sk.arena, prep, n, m, num_samples, seed, cfg, sk, stream);
                    } else {
                        // size-budgeted: rounds from a pilot of 2^16 ids, each sized from the mean
                        // sample size so far with 5 % to spare (at least doubling), until the
                        // samples hold the budget or the cap is reached; then the cut
                        uint64_t T_try = std::min<uint64_t>(num_samples, 1ull << 16);
                        for (;;) {
                            skis::sample_and_compact(sk.arena, prep, n, m, T_try, seed, cfg, sk, stream);
                            if (sk.entries >= opt.entry_budget || T_try == num_samples) break;
                            const double mean = std::max(1.0, (double)sk.entries / (double)T_try);
                            const double want = (double)opt.entry_budget / mean * 1.05 + 1024.0;
                            const uint64_t next = want >= (double)num_samples ? num_samples : (uint64_t)want;
                            T_try = std::min<uint64_t>(num_samples, std::max<uint64_t>(2 * T_try, next));
                        }
                        skis::truncate_to_budget(sk, opt.entry_budget, stream);
                    }
                }
                // q moves into the sketch only after every kernel that reads prep.q has run
                sk.q.swap(prep.q);
            } // preprocessing buffers released here
            if (opt.build_inverse_index) {
                SKIS_HIP_TRY(hipEventRecord(e0, stream));
                skis::build_inverse(sk, stream);
                SKIS_HIP_TRY(hipEventRecord(e1, stream));
                SKIS_HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                SKIS_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                sk.ms_inverse = ms;
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            SKIS_HIP_TRY(hipStreamSynchronize(stream));
            sk.arena.trim(true); // the stages' temporaries are idle: to the block cache
            *out = h;
            if (status == SKIS_WDEGENERATE) skis::set_error("Gamma = 0: no non-singular sample exists");
            return status;
        } catch (...) {
            delete h;
            throw;
        }
    });
}

int skis_sketch_info(const skis_sketch *h, skis_info *info)
{
    return guarded([&]() -> int {
        if (!h || !info) throw skis::Error{SKIS_EINVAL, "NULL argument"};
        const skis::Sketch &sk = h->core;
        std::memset(info, 0, sizeof(*info));
        info->n = sk.n;
        info->T = sk.T;
        info->entries = sk.entries;
        info->probed_total = sk.probed_total;
        info->deferred = sk.deferred;
        info->C = sk.C;
        info->Gamma = sk.Gamma;
        info->device_bytes = sk.arena.used;
        info->ms_preprocess = sk.ms_preprocess;
        info->ms_roots = sk.ms_roots;
        info->ms_sample = sk.ms_sample;
        info->ms_compact = sk.ms_compact;
        info->ms_inverse = sk.ms_inverse;
        info->ms_tier0 = sk.ms_tier0;
        info->ms_tier1 = sk.ms_tier1;
        info->ms_tier2 = sk.ms_tier2;
        info->ms_tier3 = sk.ms_tier3;
        info->deferred_global = sk.deferred_global;
        info->deferred_bitmap = sk.deferred_bitmap;
        info->plain_levels = sk.plain_levels;
        info->graph_replays = sk.graph_replays;
        for (int t = 0; t < 4; ++t) {
            info->tier_samples[t] = sk.tier_stats[t][0];
            info->tier_entries[t] = sk.tier_stats[t][1];
            info->tier_probed[t] = sk.tier_stats[t][2];
            info->tier_swept[t] = sk.tier_stats[t][3];
            info->tier_items[t] = sk.tier_stats[t][4];
        }
        return SKIS_OK;
    });
}

int skis_estimate(const skis_sketch *hc, int32_t num_sets, const int64_t *set_ptr, const int32_t *set_nodes,
                  uint64_t *cov, double *est, hipStream_t stream)
{
    return guarded([&]() -> int {
        if (!hc) throw skis::Error{SKIS_EINVAL, "NULL sketch"};
        skis_sketch *h = const_cast<skis_sketch *>(hc);
        if (num_sets < 0) throw skis::Error{SKIS_EINVAL, "num_sets must be >= 0"};
        if (num_sets == 0) return SKIS_OK;
        if (!set_ptr || !cov || !est) throw skis::Error{SKIS_EINVAL, "NULL argument"};
        if (!h->core.has_inverse) throw skis::Error{SKIS_EINVAL, "sketch was built without the inverse index"};
        std::lock_guard<std::mutex> lk(h->mu);
        h->core.arena.stream = stream; // this call's scratch is allocated and released in its order
        skis::estimate_batch(h->core, h->qs, num_sets, set_ptr, set_nodes, cov, est, stream);
        h->core.arena.trim();
        return SKIS_OK;
    });
}

int skis_greedy_max_cover(const skis_sketch *hc, int32_t k, int32_t *seeds, uint64_t *marg, uint64_t *cov_out,
                          double *est_out, hipStream_t stream)
{
    return guarded([&]() -> int {
        if (!hc) throw skis::Error{SKIS_EINVAL, "NULL sketch"};
        skis_sketch *h = const_cast<skis_sketch *>(hc);
        if (k < 1 || k > h->core.n) throw skis::Error{SKIS_EINVAL, "k must be in [1, n]"};
        if (!seeds || !marg || !cov_out || !est_out) throw skis::Error{SKIS_EINVAL, "NULL argument"};
        if (!h->core.has_inverse) throw skis::Error{SKIS_EINVAL, "sketch was built without the inverse index"};
        std::lock_guard<std::mutex> lk(h->mu);
        h->core.arena.stream = stream;
        skis::greedy(h->core, h->qs, k, seeds, marg, cov_out, est_out, stream);
        h->core.arena.trim(true); // greedy ends with a synchronisation of its stream
        return SKIS_OK;
    });
}

int skis_sketch_export(const skis_sketch *h, int64_t *sample_ptr, int32_t *nodes, int32_t *roots, uint64_t *probed,
                       hipStream_t stream)
{
    return guarded([&]() -> int {
        if (!h) throw skis::Error{SKIS_EINVAL, "NULL sketch"};
        const skis::Sketch &sk = h->core;
        if (sample_ptr)
            SKIS_HIP_TRY(hipMemcpyAsync(sample_ptr, sk.sample_ptr.ptr, sizeof(int64_t) * (sk.T + 1),
                                        hipMemcpyDeviceToDevice, stream));
        if (nodes && sk.entries)
            SKIS_HIP_TRY(hipMemcpyAsync(nodes, sk.nodes.ptr, sizeof(int32_t) * sk.entries, hipMemcpyDeviceToDevice,
                                        stream));
        if (roots && sk.T)
            SKIS_HIP_TRY(hipMemcpyAsync(roots, sk.roots.ptr, sizeof(int32_t) * sk.T, hipMemcpyDeviceToDevice, stream));
        if (probed && sk.T)
            SKIS_HIP_TRY(hipMemcpyAsync(probed, sk.probed.ptr, sizeof(uint64_t) * sk.T, hipMemcpyDeviceToDevice,
                                        stream));
        SKIS_HIP_TRY(hipStreamSynchronize(stream));
        return SKIS_OK;
    });
}

int skis_inverse_export(const skis_sketch *h, int64_t *node_ptr, int32_t *node_samples, hipStream_t stream)
{
    return guarded([&]() -> int {
        if (!h) throw skis::Error{SKIS_EINVAL, "NULL sketch"};
        const skis::Sketch &sk = h->core;
        if (!sk.has_inverse) throw skis::Error{SKIS_EINVAL, "sketch was built without the inverse index"};
        if (node_ptr)
            SKIS_HIP_TRY(hipMemcpyAsync(node_ptr, sk.node_ptr.ptr, sizeof(int64_t) * ((size_t)sk.n + 1),
                                        hipMemcpyDeviceToDevice, stream));
        if (node_samples && sk.entries)
            SKIS_HIP_TRY(hipMemcpyAsync(node_samples, sk.node_samples.ptr, sizeof(int32_t) * sk.entries,
                                        hipMemcpyDeviceToDevice, stream));
        SKIS_HIP_TRY(hipStreamSynchronize(stream));
        return SKIS_OK;
    });
}

int skis_node_q(const skis_sketch *h, double *q, hipStream_t stream)
{
    return guarded([&]() -> int {
        if (!h || !q) throw skis::Error{SKIS_EINVAL, "NULL argument"};
        SKIS_HIP_TRY(hipMemcpyAsync(q, h->core.q.ptr, sizeof(double) * (size_t)h->core.n, hipMemcpyDeviceToDevice,
                                    stream));
        SKIS_HIP_TRY(hipStreamSynchronize(stream));
        return SKIS_OK;
    });
}

void skis_sketch_free(skis_sketch *h)
{
    if (!h) return;
    // every call on the sketch has returned, but its buffers may have been used on any
    // stream: release them in order behind all work on the device
    (void)hipDeviceSynchronize();
    h->core.arena.stream = nullptr;
    h->core.arena.idle_on_destroy = true; // nothing queued uses the blocks any more
    delete h;
}

int skis_probe_random_read(const void *table, uint64_t rows, uint32_t row_bytes, uint64_t reads, uint32_t seed,
                           uint32_t *sink, hipStream_t stream)
{
    return guarded([&]() -> int {
        skis::probe_random_read(table, rows, row_bytes, reads, seed, sink, stream);
        return SKIS_OK;
    });
}

int skis_samples_for_estimate(int32_t n, double Gamma, double I_lower, double eps, double delta, uint64_t *T_out)
{
    return guarded([&]() -> int {
        if (!T_out) throw skis::Error{SKIS_EINVAL, "T_out must not be NULL"};
        if (n <= 0) throw skis::Error{SKIS_EINVAL, "n must be positive"};
        if (!(Gamma >= 0.0 && Gamma <= (double)n)) throw skis::Error{SKIS_EINVAL, "Gamma must be in [0, n]"};
        if (!(I_lower > 0.0)) throw skis::Error{SKIS_EINVAL, "I_lower must be positive"};
        if (!(eps > 0.0)) throw skis::Error{SKIS_EINVAL, "eps must be positive"};
        if (!(delta > 0.0 && delta < 1.0)) throw skis::Error{SKIS_EINVAL, "delta must be in (0, 1)"};
        // Lemma lem:monte: (2 Gamma / n + 2 eps / 3) ln(2 / delta) (n / I(S)) eps^-2 samples
        const double T = (2.0 * Gamma / (double)n + 2.0 * eps / 3.0) * std::log(2.0 / delta) * ((double)n / I_lower) /
                         (eps * eps);
        if (!(T < 9.2e18)) throw skis::Error{SKIS_EINVAL, "the sample count does not fit 63 bits"};
        *T_out = (uint64_t)std::ceil(T);
        return SKIS_OK;
    });
}

int skis_set_memory_limits(uint64_t cache_keep_bytes, uint64_t pool_keep_bytes)
{
    return guarded([&]() -> int {
        skis::g_cache_keep.store(cache_keep_bytes);
        skis::g_pool_keep.store(pool_keep_bytes);
        int d = 0;
        SKIS_HIP_TRY(hipGetDevice(&d));
        int supported = 0;
        if (hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, d) == hipSuccess && supported) {
            hipMemPool_t pool = nullptr;
            uint64_t keep = pool_keep_bytes;
            if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess)
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        (void)hipGetLastError();
        skis::trim_idle_cache(cache_keep_bytes);
        return SKIS_OK;
    });
}

int skis_release_cached_memory(void)
{
    return guarded([&]() -> int {
        skis::release_idle_memory();
        return SKIS_OK;
    });
}

const char *skis_last_error(void) { return skis::get_error().c_str(); }

} // extern "C"
