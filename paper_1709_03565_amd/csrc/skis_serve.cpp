// skis_serve.cpp -- an influence-estimate service over a resident sketch: the query phase
// of Alg. 2 (answer any seed set from the fixed sketch, Eq. eq21) under a stream of
// requests.
//
// Continuous batching: submitters append queries to a host queue; one worker thread owns
// `depth` pipeline slots, each with its own HIP stream, pinned host staging, device CSR
// buffers and zeroed bitmap scratch.  Whenever a slot is free and queries are waiting, the
// worker takes as many as the slot admits (by count, by total entries and by large sets),
// except that a heavy set (one whose members' sample lists hold more than HEAVY_WORK entries,
// a hub's set) runs in a batch of its own: a batch completes when its slowest set does, so a
// hub set among light ones would hold them all for milliseconds, while alone it holds one
// slot and the other slots keep serving.  It packs them into the slot's pinned CSR, and enqueues copy-in, the estimate kernels and
// copy-out on the slot's stream without waiting.  It polls the slots' completion events,
// and when a batch is done it stores each query's (Cov, I_hat) and completion time and
// wakes the waiters.  A query's result does not depend on the batch it ran in: each set
// takes its own workgroup and bitmap, and its sums run in a fixed order.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <memory>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "skis_internal.h"
#include "skis_query.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
    uint64_t ticket;
    std::vector<int32_t> nodes;
    uint64_t work = 0; // sum of |H(v)| over the members (from the inverse index's offsets)
    Clock::time_point arrive;
};

// A set whose members' lists hold more entries than this is batched alone (about a
// millisecond of walking for one workgroup; a set of 1000 uniform members on the 4M-node TRI
// sketch holds about 60 thousand, its top hub 3 million).
constexpr uint64_t HEAVY_WORK = 1ull << 18;

struct Done {
    uint64_t cov;
    double est;
    double latency_us;
};

template <typename T>
struct Pinned {
    T *ptr = nullptr;
    size_t count = 0;
    Pinned() = default;
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
    ~Pinned()
    {
        if (ptr) (void)hipHostFree(ptr);
    }
    void alloc(size_t n)
    {
        SKIS_HIP_TRY(hipHostMalloc((void **)&ptr, sizeof(T) * (n ? n : 1), hipHostMallocDefault));
        count = n;
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Pinned<int64_t> h_ptr;
    Pinned<int32_t> h_nodes;
    Pinned<int64_t> h_large;
    Pinned<unsigned long long> h_cov;
    Pinned<double> h_est;
    Pinned<int> h_err;
    skis::DevBuf<int64_t> d_ptr;
    skis::DevBuf<int32_t> d_nodes;
    skis::DevBuf<int64_t> d_large;
    skis::DevBuf<unsigned long long> d_cov;
    skis::DevBuf<double> d_est;
    skis::DevBuf<int> d_err;
    skis::DevBuf<uint32_t> bitmaps;  // max_batch_queries bitmaps of T bits
    skis::DevBuf<uint32_t> nodebits; // max_large node bitmaps of n bits
    std::vector<Pending> batch;
    bool busy = false;
};

} // namespace

struct skis_server {
    const skis_sketch *sk = nullptr;
    skis_server_options opt{};
    int device = 0;
    uint64_t wordsT = 1, wordsN = 1;
    skis::Arena arena;
    std::vector<int64_t> node_ptr; // host copy of the inverse index's offsets (n + 1), for the work of a set
    std::vector<std::unique_ptr<Slot>> slots;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, Done> results;
    std::unordered_set<uint64_t> outstanding; // submitted, not yet collected by a wait
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string fault; // set when the worker stopped on an error
    // statistics (under mu)
    uint64_t batches = 0, queries = 0, max_batch = 0;
    uint64_t hist[16] = {};

    void run();
    void launch(Slot &sl);
    void complete(Slot &sl);
    ~skis_server()
    {
        for (auto &p : slots) {
            if (p->stream) (void)hipStreamSynchronize(p->stream);
            if (p->done) (void)hipEventDestroy(p->done);
            if (p->stream) (void)hipStreamDestroy(p->stream);
        }
    }
};

void skis_server::launch(Slot &sl)
{
    const skis::Sketch &k = sk->core;
    const int32_t nq = (int32_t)sl.batch.size();
    int64_t off = 0;
    int32_t nl = 0;
    for (int32_t i = 0; i < nq; ++i) {
        const auto &v = sl.batch[i].nodes;
        sl.h_ptr.ptr[i] = off;
        if (!v.empty()) std::memcpy(sl.h_nodes.ptr + off, v.data(), sizeof(int32_t) * v.size());
        off += (int64_t)v.size();
        if ((int64_t)v.size() > skis::EST_MAX_SET) sl.h_large.ptr[nl++] = i;
    }
    sl.h_ptr.ptr[nq] = off;
    hipStream_t s = sl.stream;
    SKIS_HIP_TRY(hipMemcpyAsync(sl.d_ptr.ptr, sl.h_ptr.ptr, sizeof(int64_t) * (size_t)(nq + 1), hipMemcpyHostToDevice, s));
    if (off > 0)
        SKIS_HIP_TRY(hipMemcpyAsync(sl.d_nodes.ptr, sl.h_nodes.ptr, sizeof(int32_t) * (size_t)off,
                                    hipMemcpyHostToDevice, s));
    if (nl > 0)
        SKIS_HIP_TRY(hipMemcpyAsync(sl.d_large.ptr, sl.h_large.ptr, sizeof(int64_t) * (size_t)nl,
                                    hipMemcpyHostToDevice, s));
    skis::estimate_launch(k, nq, sl.d_ptr.ptr, sl.d_nodes.ptr, sl.d_large.ptr, nl, sl.bitmaps.ptr, wordsT,
                          sl.nodebits.ptr, sl.d_cov.ptr, sl.d_est.ptr, sl.d_err.ptr, s);
    SKIS_HIP_TRY(hipMemcpyAsync(sl.h_cov.ptr, sl.d_cov.ptr, sizeof(unsigned long long) * (size_t)nq,
                                hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipMemcpyAsync(sl.h_est.ptr, sl.d_est.ptr, sizeof(double) * (size_t)nq, hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipMemcpyAsync(sl.h_err.ptr, sl.d_err.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipEventRecord(sl.done, s));
    sl.busy = true;
}

void skis_server::complete(Slot &sl)
{
    if (*sl.h_err.ptr) {
        // ids were checked at submission, so this is an internal fault: scratch may hold bits
        throw skis::Error{SKIS_EHIP, "internal error in the estimate kernel (flags " + std::to_string(*sl.h_err.ptr) +
                                         ")"};
    }
    const auto now = Clock::now();
    const size_t nq = sl.batch.size();
    {
        std::lock_guard<std::mutex> g(mu);
        for (size_t i = 0; i < nq; ++i) {
            const double lat = std::chrono::duration<double, std::micro>(now - sl.batch[i].arrive).count();
            results[sl.batch[i].ticket] = Done{(uint64_t)sl.h_cov.ptr[i], sl.h_est.ptr[i], lat};
        }
        batches += 1;
        queries += nq;
        if (nq > max_batch) max_batch = nq;
        int b = 0;
        while (b < 15 && (1ull << (b + 1)) <= nq) ++b;
        hist[b] += 1;
    }
    sl.batch.clear();
    sl.busy = false;
    cv_done.notify_all();
}

void skis_server::run()
{
    try {
        SKIS_HIP_TRY(hipSetDevice(device));
        for (;;) {
            Slot *free_slot = nullptr;
            bool any_busy = false;
            {
                std::unique_lock<std::mutex> g(mu);
                for (auto &p : slots) any_busy |= p->busy;
                if (!any_busy) cv_work.wait(g, [&] { return stop || !queue.empty(); });
                if (stop && queue.empty() && !any_busy) return;
                for (auto &p : slots)
                    if (!p->busy) {
                        free_slot = p.get();
                        break;
                    }
                if (free_slot && !queue.empty()) {
                    // admission: by count, by entries (pinned staging) and by large sets
                    Slot &sl = *free_slot;
                    uint64_t entries = 0;
                    uint32_t large = 0;
                    while (!queue.empty() && sl.batch.size() < opt.max_batch_queries) {
                        const uint64_t e = queue.front().nodes.size();
                        const bool is_large = e > (uint64_t)skis::EST_MAX_SET;
                        const bool heavy = queue.front().work > HEAVY_WORK;
                        if (heavy && !sl.batch.empty()) break; // it goes alone, in the next free slot
                        if (entries + e > opt.max_batch_entries) break;
                        if (is_large && large >= opt.max_large_sets) break;
                        entries += e;
                        large += is_large ? 1u : 0u;
                        sl.batch.push_back(std::move(queue.front()));
                        queue.pop_front();
                        if (heavy) break;
                    }
                } else {
                    free_slot = nullptr;
                }
            }
            if (free_slot && !free_slot->batch.empty()) {
                launch(*free_slot);
                continue;
            }
            // nothing to launch now: finish every batch that is done (in any order, so a
            // slow batch holds only its own queries), else poll again
            bool progressed = false;
            for (auto &p : slots) {
                if (!p->busy) continue;
                const hipError_t q = hipEventQuery(p->done);
                if (q == hipSuccess) {
                    complete(*p);
                    progressed = true;
                } else if (q != hipErrorNotReady) {
                    SKIS_HIP_TRY(q);
                }
            }
            if (!progressed) std::this_thread::yield();
        }
    } catch (const skis::Error &e) {
        std::lock_guard<std::mutex> g(mu);
        fault = e.msg;
        stop = true;
        cv_done.notify_all();
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> g(mu);
        fault = e.what();
        stop = true;
        cv_done.notify_all();
    }
}

namespace {

template <typename F>
int serve_guarded(F &&f)
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

int submit_one(skis_server *sv, const int32_t *nodes, int32_t count, Clock::time_point arrive, uint64_t *ticket)
{
    if (count < 0) throw skis::Error{SKIS_EINVAL, "count must be >= 0"};
    if (count > 0 && !nodes) throw skis::Error{SKIS_EINVAL, "nodes must not be NULL"};
    if ((uint64_t)count > sv->opt.max_batch_entries)
        throw skis::Error{SKIS_EINVAL, "set larger than max_batch_entries"};
    const int32_t n = sv->sk->core.n;
    for (int32_t i = 0; i < count; ++i)
        if (nodes[i] < 0 || nodes[i] >= n) throw skis::Error{SKIS_EINVAL, "a seed set holds a node id outside [0, n)"};
    Pending p;
    p.nodes.assign(nodes, nodes + count);
    if (!sv->node_ptr.empty())
        for (int32_t i = 0; i < count; ++i) p.work += (uint64_t)(sv->node_ptr[nodes[i] + 1] - sv->node_ptr[nodes[i]]);
    p.arrive = arrive;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->stop) throw skis::Error{SKIS_EHIP, "server stopped: " + sv->fault};
        p.ticket = sv->next_ticket++;
        sv->outstanding.insert(p.ticket);
        if (ticket) *ticket = p.ticket;
        sv->queue.push_back(std::move(p));
    }
    sv->cv_work.notify_one();
    return SKIS_OK;
}

int wait_one(skis_server *sv, uint64_t ticket, uint64_t *cov, double *est, double *latency_us)
{
    std::unique_lock<std::mutex> g(sv->mu);
    if (!sv->outstanding.count(ticket)) throw skis::Error{SKIS_EINVAL, "unknown or already collected ticket"};
    sv->cv_done.wait(g, [&] { return sv->results.count(ticket) || sv->stop; });
    auto it = sv->results.find(ticket);
    if (it == sv->results.end()) throw skis::Error{SKIS_EHIP, "server stopped: " + sv->fault};
    if (cov) *cov = it->second.cov;
    if (est) *est = it->second.est;
    if (latency_us) *latency_us = it->second.latency_us;
    sv->results.erase(it);
    sv->outstanding.erase(ticket);
    return SKIS_OK;
}

} // namespace

extern "C" {

void skis_server_default_options(skis_server_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->pipeline_depth = 4;
    opt->max_batch_queries = 256;
    opt->max_batch_entries = 1u << 20;
    opt->max_large_sets = 4;
}

int skis_server_create(const skis_sketch *sk, const skis_server_options *opt_in, skis_server **out)
{
    return serve_guarded([&]() -> int {
        if (!out) throw skis::Error{SKIS_EINVAL, "out must not be NULL"};
        *out = nullptr;
        if (!sk) throw skis::Error{SKIS_EINVAL, "NULL sketch"};
        if (!sk->core.has_inverse && sk->core.T > 0)
            throw skis::Error{SKIS_EINVAL, "the sketch was built without the inverse index"};
        skis_server_options opt;
        skis_server_default_options(&opt);
        if (opt_in) {
            if (opt_in->pipeline_depth) opt.pipeline_depth = opt_in->pipeline_depth;
            if (opt_in->max_batch_queries) opt.max_batch_queries = opt_in->max_batch_queries;
            if (opt_in->max_batch_entries) opt.max_batch_entries = opt_in->max_batch_entries;
            if (opt_in->max_large_sets) opt.max_large_sets = opt_in->max_large_sets;
            opt.max_device_bytes = opt_in->max_device_bytes;
        }
        if (opt.pipeline_depth > 16 || opt.max_batch_queries > (1u << 20))
            throw skis::Error{SKIS_EINVAL, "pipeline_depth must be <= 16 and max_batch_queries <= 2^20"};
        auto sv = std::make_unique<skis_server>();
        sv->sk = sk;
        sv->opt = opt;
        SKIS_HIP_TRY(hipGetDevice(&sv->device));
        sv->arena.cap = opt.max_device_bytes;
        sv->wordsT = sk->core.T ? (sk->core.T + 31) / 32 : 1;
        sv->wordsN = ((uint64_t)sk->core.n + 31) / 32;
        if (sk->core.T > 0 && sk->core.node_ptr.ptr) {
            sv->node_ptr.resize((size_t)sk->core.n + 1);
            SKIS_HIP_TRY(hipMemcpy(sv->node_ptr.data(), sk->core.node_ptr.ptr, sizeof(int64_t) * ((size_t)sk->core.n + 1),
                                   hipMemcpyDeviceToHost));
        }
        const uint64_t nb = std::max<uint64_t>(opt.max_batch_queries, opt.max_large_sets);
        sv->arena.stream = nullptr; // allocations complete before any slot stream uses them (below)
        for (uint32_t i = 0; i < opt.pipeline_depth; ++i) {
            sv->slots.push_back(std::make_unique<Slot>());
            Slot &s = *sv->slots.back();
            SKIS_HIP_TRY(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
            SKIS_HIP_TRY(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
            s.h_ptr.alloc(opt.max_batch_queries + 1);
            s.h_nodes.alloc(opt.max_batch_entries);
            s.h_large.alloc(opt.max_large_sets);
            s.h_cov.alloc(opt.max_batch_queries);
            s.h_est.alloc(opt.max_batch_queries);
            s.h_err.alloc(1);
            s.d_ptr.alloc(sv->arena, opt.max_batch_queries + 1);
            s.d_nodes.alloc(sv->arena, opt.max_batch_entries);
            s.d_large.alloc(sv->arena, opt.max_large_sets);
            s.d_cov.alloc(sv->arena, opt.max_batch_queries);
            s.d_est.alloc(sv->arena, opt.max_batch_queries);
            s.d_err.alloc(sv->arena, 1);
            s.bitmaps.alloc(sv->arena, nb * sv->wordsT);
            s.nodebits.alloc(sv->arena, (uint64_t)opt.max_large_sets * sv->wordsN);
            SKIS_HIP_TRY(hipDeviceSynchronize());
            skis::fill_u32(s.bitmaps.ptr, nb * sv->wordsT, s.stream);
            skis::fill_u32(s.nodebits.ptr, (uint64_t)opt.max_large_sets * sv->wordsN, s.stream);
            skis::fill_u32(reinterpret_cast<uint32_t *>(s.d_err.ptr), 1, s.stream);
            SKIS_HIP_TRY(hipStreamSynchronize(s.stream));
        }
        skis_server *raw = sv.get();
        sv->worker = std::thread([raw] { raw->run(); });
        *out = sv.release();
        return SKIS_OK;
    });
}

int skis_server_submit(skis_server *sv, const int32_t *nodes, int32_t count, uint64_t *ticket)
{
    return serve_guarded([&]() -> int {
        if (!sv) throw skis::Error{SKIS_EINVAL, "NULL server"};
        return submit_one(sv, nodes, count, Clock::now(), ticket);
    });
}

int skis_server_wait(skis_server *sv, uint64_t ticket, uint64_t *cov, double *est, double *latency_us)
{
    return serve_guarded([&]() -> int {
        if (!sv) throw skis::Error{SKIS_EINVAL, "NULL server"};
        return wait_one(sv, ticket, cov, est, latency_us);
    });
}

int skis_server_replay(skis_server *sv, int32_t num_queries, const int64_t *set_ptr, const int32_t *set_nodes,
                       const double *arrival_us, uint64_t *cov, double *est, double *latency_us)
{
    return serve_guarded([&]() -> int {
        if (!sv) throw skis::Error{SKIS_EINVAL, "NULL server"};
        if (num_queries < 0 || (num_queries > 0 && (!set_ptr || !arrival_us)))
            throw skis::Error{SKIS_EINVAL, "bad replay arguments"};
        for (int32_t i = 0; i < num_queries; ++i) {
            if (set_ptr[i + 1] < set_ptr[i] || set_ptr[i] < 0 || set_ptr[i + 1] - set_ptr[i] > INT32_MAX)
                throw skis::Error{SKIS_EINVAL, "set_ptr must be nondecreasing from 0"};
            if (i > 0 && arrival_us[i] < arrival_us[i - 1])
                throw skis::Error{SKIS_EINVAL, "arrival times must be nondecreasing"};
        }
        std::vector<uint64_t> tickets((size_t)num_queries);
        const Clock::time_point t0 = Clock::now();
        for (int32_t i = 0; i < num_queries; ++i) {
            const auto due = t0 + std::chrono::duration_cast<Clock::duration>(
                                      std::chrono::duration<double, std::micro>(arrival_us[i]));
            while (Clock::now() < due) {
            } // open loop: submit at the scheduled time, whatever is still in flight
            submit_one(sv, set_nodes + set_ptr[i], (int32_t)(set_ptr[i + 1] - set_ptr[i]), due, &tickets[i]);
        }
        for (int32_t i = 0; i < num_queries; ++i) {
            uint64_t c = 0;
            double e = 0, l = 0;
            wait_one(sv, tickets[i], &c, &e, &l);
            if (cov) cov[i] = c;
            if (est) est[i] = e;
            if (latency_us) latency_us[i] = l;
        }
        return SKIS_OK;
    });
}

int skis_server_get_stats(skis_server *sv, skis_server_stats *st)
{
    return serve_guarded([&]() -> int {
        if (!sv || !st) throw skis::Error{SKIS_EINVAL, "NULL argument"};
        std::lock_guard<std::mutex> g(sv->mu);
        std::memset(st, 0, sizeof(*st));
        st->batches = sv->batches;
        st->queries = sv->queries;
        st->max_batch = sv->max_batch;
        st->device_bytes = sv->arena.used;
        for (int i = 0; i < 16; ++i) st->batch_hist[i] = sv->hist[i];
        return SKIS_OK;
    });
}

void skis_server_destroy(skis_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    delete sv;
}

} // extern "C"
