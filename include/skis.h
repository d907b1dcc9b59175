/*
 * skis.h -- C ABI of libskis: the SKIS hot path (importance sketching of influence
 * dynamics; Nguyen, Thai, Dinh, ICDM 2017) on AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Sec. 2, Definitions 1 and 2): given a probabilistic graph G=(V,E,w)
 * under the independent cascade model, estimate the influence I(S) of seed sets S
 * (influence estimation) and find k seeds of large influence (influence maximisation).
 * The library builds a sketch R = {R_1..R_T} of non-singular reverse-reachable samples
 * drawn by IIS (Alg. 1), keeps it on the device as a CSR hypergraph plus its transpose
 * (Alg. 2, preprocessing), and answers estimate queries by Eq. (eq21) and k-seed queries
 * by the greedy of Alg. 3.
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - Every call takes a hipStream_t and is ordered on it.  Calls that return results in
 *     host memory (marked "blocking") synchronise that stream before returning.
 *   - Return value: SKIS_OK (0), a positive warning, or a negative error code.  On error
 *     nothing is allocated or leaked, output buffers may be partly written, and
 *     skis_last_error() returns a message (thread-local, valid until the next call on
 *     the same thread).
 *   - Graph layout (in-CSR): row v lists the in-edges u->v of v.  row_ptr[n+1] int32,
 *     row_ptr[0] = 0, row_ptr[n] = m, nondecreasing; col[m] int32 holds the source u of
 *     each in-edge, u in [0,n), u != v; w[m] float32 in [0,1] is the edge probability.
 *     The order of edges within a row is the "fixed order" of N_in(v) in Sec. 3.1
 *     (component 3); it changes which sample a given seed produces, not the distribution.
 *     Repeated (u,v) pairs are independent edges.  The edge id of an in-edge is its
 *     position in col.
 *   - Randomness: sample j of a sketch is a pure function of (graph, seed, j) through a
 *     counter-based Philox4x32-10 stream (Salmon et al., SC'11), so results do not depend
 *     on launch shape, scheduling or the form of the sampler.
 */
#ifndef SKIS_H
#define SKIS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SKIS_OK 0
#define SKIS_WDEGENERATE 1 /* warning: Gamma = 0, no non-singular sample exists; empty sketch */
#define SKIS_EINVAL (-1)   /* invalid argument or malformed graph */
#define SKIS_ENOMEM (-2)   /* device allocation failed or max_device_bytes exceeded */
#define SKIS_EHIP (-3)     /* a HIP runtime call failed */

typedef struct skis_sketch skis_sketch; /* opaque; owns every device buffer it allocates */

/* Sampler and memory knobs.  Zero fields mean "default"; skis_default_options fills them. */
typedef struct skis_options {
    uint32_t form;                /* 0: persistent sampler (default); 1: plain form, one launch per BFS
                                     level; 2: captured form, the persistent sampler's whole chain
                                     (roots and the three tiers, with device-side work counts) captured
                                     once into a HIP graph and replayed per chunk of chunk_samples ids */
    uint32_t slots_per_block;     /* samples in flight per workgroup of the first sampler tier */
    uint32_t visited_threshold;   /* nodes per sample kept in LDS by the first tier before the sample
                                     moves to the next tier */
    uint32_t big_row;             /* in-degree above which the first tier hands a sample on */
    uint32_t build_inverse_index; /* 1 (default): build node->samples for estimate / greedy; 0: build only */
    uint32_t threads_per_block;   /* 64 (default: one wave per workgroup) or 256.  Supported
                                     (threads, slots, visited, quads_per_lane):
                                     (64,4,192,1) default, (64,4,192,2), (64,16,128,2),
                                     (64,4,256,2), (64,4,256,1), (64,2,256,1), (64,3,256,1),
                                     (64,2,384,1), (64,6,256,2), (64,8,128,2),
                                     (64,8,192,2), (64,8,192,1), (64,8,256,2), (64,12,192,2),
                                     (64,16,64,2), (256,16,128,2), (256,32,128,2), (256,16,256,2) */
    uint64_t max_device_bytes;    /* 0 = unlimited; larger total allocation -> SKIS_ENOMEM */
    uint64_t staging_entries;     /* initial staging capacity in node entries (0 = auto) */
    uint64_t chunk_samples;       /* captured form: sample ids per graph replay (0 = 2^24) */
    uint32_t quads_per_lane;      /* first tier: most edge quads (aligned groups of four edges)
                                     a lane takes per sweep, 1 (default: fewer registers, more
                                     workgroups resident) or 2 */
    uint64_t entry_budget;        /* 0 (default): num_samples samples.  Otherwise a size-budgeted sketch
                                     (the stopping rule of Sec. 7, samples until their total size
                                     reaches h * n * log n): the sketch holds samples 0 .. T-1 for the
                                     smallest T <= num_samples whose sizes sum to at least entry_budget
                                     (T = num_samples if none does).  Samples are drawn in rounds that
                                     overshoot and the sketch is then cut at T, so T and every sample are
                                     the same whatever the rounds; the tier and time counters of
                                     skis_info describe the last round */
    uint32_t ris_mode;            /* 0 (default): IIS samples (Alg. 1); 1: plain RIS samples of Sec. 2.3.1
                                     -- a root uniform over V, independent coins on all its in-edges,
                                     singular samples {root} kept -- for comparisons with IIS.  A RIS
                                     sketch answers estimate with n * Cov / T (Eq. ris_prob) and runs
                                     the greedy on gains n * Delta / T; it is built even when Gamma = 0 */
    uint32_t model;               /* diffusion model: 0 (default) independent cascade (Alg. 1); 1 linear
                                     threshold (Sec. 6): every node's in-weights must sum to at most 1 (up
                                     to 2^-20 of rounding), gamma_v = sum of v's in-weights, the root picks
                                     exactly one in-neighbour u with probability w(u, root) / gamma_root
                                     and the sample follows the model's reverse walk (the node added last
                                     picks at most one in-neighbour u with probability w(u, x)) until a node
                                     picks none or one already in the sample.  Persistent form only (form
                                     0), no RIS mode; skis_info's tier 0 is the walk kernel, tier 1 the
                                     kernel of walks longer than 32 nodes, *_swept count the picks drawn */
} skis_options;

/* Fills *opt with the defaults. */
void skis_default_options(skis_options *opt);

/*
 * Lemma lem:monte: a sketch of at least T = ceil((2 Gamma / n + 2 eps / 3) ln(2 / delta) n /
 * (I_lower eps^2)) samples gives an (eps, delta)-estimate of I(S) for every set S with
 * I(S) >= I_lower (the Lemma states it for I(S); any lower bound of it, such as |S|, keeps the
 * guarantee).  Host arithmetic only (binary64), no device work.  *T_out (host) receives T.
 * Errors: SKIS_EINVAL for n <= 0, Gamma outside [0, n], I_lower <= 0, eps <= 0, delta outside
 * (0, 1), or a T of 2^63 or more.
 */
int skis_samples_for_estimate(int32_t n, double Gamma, double I_lower, double eps, double delta,
                              uint64_t *T_out /* host */);

/*
 * Preprocessing alone (rows a1-a3 of the hot path), into caller buffers:
 *   Eq. (gamma_v):  P[e] = prod of (1 - w) over row v up to and including edge e, in row
 *                   order, left to right, fp64, one rounding per product (the bucket
 *                   masses of Eq. probn are (P[e-1] - P[e]) / gamma_v);  q[v] = P of the last edge of
 *                   row v (1 for an empty row) = 1 - gamma_v.
 *   Eq. (probu):    root weights W[v] = ceil(gamma_v * 2^s), s = 62 - ceil(log2 n), so the
 *                   root is v with probability W[v]/C, C = sum W (*C_out, host);
 *                   Gamma = sum_v gamma_v, exactly rounded (*Gamma_out, host);
 *                   alias table (thr[v] uint64, alias[v] int32): a bucket b drawn
 *                   uniformly and r uniform in [0,C) give v = (r < thr[b]) ? b : alias[b].
 *                   The table is the unique one produced by the sequential sweep: light
 *                   nodes (n*W <= C) in id order are filled from the current heavy node
 *                   (heavy nodes in id order), and a heavy node whose remainder falls to
 *                   <= C becomes a bucket at once, filled from the next heavy node.
 * Any output pointer may be NULL.  Blocking.  Errors: SKIS_EINVAL for a malformed graph.
 */
int skis_preprocess(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                    double *P, double *q, uint64_t *W, uint64_t *thr, int32_t *alias,
                    uint64_t *C_out /* host */, double *Gamma_out /* host */, hipStream_t stream);

/*
 * skis_preprocess for the linear threshold model (Sec. 6): S[e] = the running sum of w over row
 * v up to and including edge e, left to right in fp64 (S before the row's first edge is 0);
 * q[v] = 1 - the row's sum (1 for an empty row, 0 when the sum rounds past 1), so gamma_v =
 * 1 - q[v] is the sum of v's in-weights; W, thr, alias, C and Gamma as for skis_preprocess.
 * Errors: SKIS_EINVAL also when a row's weights sum to more than 1 + 2^-20.
 */
int skis_preprocess_lt(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                       double *S, double *q, uint64_t *W, uint64_t *thr, int32_t *alias,
                       uint64_t *C_out /* host */, double *Gamma_out /* host */, hipStream_t stream);

/*
 * Builds the sketch of num_samples IIS samples (Alg. 1 repeated, Alg. 2 preprocessing).
 * Sample j (0 <= j < num_samples) draws its root by the alias table, its first live
 * in-edge i* by Eq. (probn) (theta = U * gamma_root, i* = first edge with 1-P[e] > theta),
 * flips independent coins for the root's later in-edges (earlier ones are dead by the
 * bucket definition), then runs the reverse BFS of Alg. 1.  Each R_j is stored
 * sorted ascending; the sketch also keeps root[j], probed[j] = sum_{x in R_j} indeg(x),
 * q[v] and Gamma.  Inputs are borrowed for the duration of the call only.
 * opt (host) may be NULL.  Blocking.  *out (host) receives the sketch.
 * Errors: SKIS_EINVAL (malformed graph, num_samples = 0 or >= 2^31, n <= 0, m < 0 or m >= 2^31),
 * SKIS_ENOMEM, SKIS_EHIP.  Returns SKIS_WDEGENERATE (and an empty sketch) when Gamma = 0.
 */
int skis_build_sketch(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                      uint64_t num_samples, uint64_t seed, const skis_options *opt, hipStream_t stream,
                      skis_sketch **out);

typedef struct skis_info {
    int32_t n;
    int32_t reserved;
    uint64_t T;                  /* samples in the sketch (0 when degenerate) */
    uint64_t entries;            /* sum_j |R_j| */
    uint64_t probed_total;       /* sum_j probed[j] (edges probed) */
    uint64_t deferred;           /* samples that outgrew the first sampler tier */
    uint64_t C;                  /* integer root-weight total */
    double Gamma;                /* sum of gamma_v */
    uint64_t device_bytes;       /* bytes the sketch holds on the device */
    double ms_preprocess, ms_roots, ms_sample, ms_compact, ms_inverse; /* stage times (events) */
    double ms_tier0, ms_tier1, ms_tier2, ms_tier3; /* the four sampler tiers' launches alone; the
                                            plain and the captured form report their whole sampler
                                            in ms_tier0 */
    uint64_t deferred_global;    /* samples that outgrew the second tier (reached the HBM hash tier) */
    uint64_t deferred_bitmap;    /* samples that outgrew the HBM hash tier (reached the bitmap tier) */
    uint32_t plain_levels;       /* plain form: BFS level launches (0 for the persistent form) */
    uint32_t graph_replays;      /* captured form: replays of the captured chain (0 otherwise) */
    uint64_t tier_samples[4];    /* samples finished by each sampler tier (LDS 192-ish, LDS 1024, HBM
                                    hash, HBM bitmap); the plain form counts everything in tier 0 */
    uint64_t tier_entries[4];    /* sum of |R_j| over those samples */
    uint64_t tier_probed[4];     /* edges probed for those samples */
    uint64_t tier_swept[4];      /* in-edges each tier's launch expanded (the work of that launch:
                                    a sample resumed from an earlier tier is not counted again for
                                    the nodes that tier expanded) */
    uint64_t tier_items[4];      /* nodes (and root items) each tier's launch expanded */
} skis_info;

/* Sketch facts (host out-param). */
int skis_sketch_info(const skis_sketch *sk, skis_info *info /* host */);

/*
 * Estimates of Eq. (eq21) for Q seed sets given in CSR form: set i is
 * set_nodes[set_ptr[i] .. set_ptr[i+1]) (device buffers; set_ptr int64[Q+1]).
 * Duplicate ids in a set count once; an empty set gives cov 0 and est 0.
 *   cov[i] = Cov(S_i) = #{ j : R_j meets S_i }                     (uint64, exact)
 *   est[i] = fl(fl(cov * Gamma) / T) + sum_{v in S_i} q_v            (fp64; the sum is
 *            compensated, so est agrees with an exactly rounded sum to ~1e-15 relative)
 * For a degenerate sketch (T = 0) the first term is 0.  Sets of any size are accepted
 * (sets above 4096 entries take a slower chunked path).  Blocking.
 * Errors: SKIS_EINVAL (node id out of range, set_ptr not nondecreasing from 0, Q < 0,
 * sketch built without the inverse index).
 */
int skis_estimate(const skis_sketch *sk, int32_t num_sets, const int64_t *set_ptr, const int32_t *set_nodes,
                  uint64_t *cov, double *est, hipStream_t stream);

/*
 * skis_estimate without device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same sets, the
 * same results bit for bit, the same errors as skis_estimate.  Its scratch (an error word,
 * the list of large sets and the per-set bitmaps) is one file-scope device array of 32 MiB
 * that every GPU the library runs on holds until the process ends; the call clears the part
 * it uses and allocates nothing.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (from several threads or streams) race and must be serialised by the
 * caller.  Sets are taken in rounds of 1024 (set_ptr read to the host, stack staging); each
 * launch holds as many T-bit bitmaps as fit in the array, so T may be at most about 2^28.
 * Sets above 4096 entries also need a node bitmap of n bits beside their T-bit bitmap;
 * SKIS_EINVAL when one of those does not fit, or when T-bit bitmaps alone do not.  Blocking.
 */
int skis_estimate_noalloc(const skis_sketch *sk, int32_t num_sets, const int64_t *set_ptr, const int32_t *set_nodes,
                          uint64_t *cov, double *est, hipStream_t stream);

/*
 * Greedy max-cover of Alg. 3: k rounds, each adding the node v outside the current set
 * with the largest gain fl(fl(Delta(v) * Gamma) / T) + q_v (Eq. margin), Delta(v) being
 * the number of samples containing v not yet covered; ties go to the smallest id.
 * seeds[k] int32 and marg[k] uint64 (Delta of each pick) are device buffers; *cov_out
 * and *est_out (host) receive Cov and I_hat of the final set (Eq. eq21).  Blocking.
 * Errors: SKIS_EINVAL (k < 1 or k > n, sketch built without the inverse index).
 */
int skis_greedy_max_cover(const skis_sketch *sk, int32_t k, int32_t *seeds, uint64_t *marg,
                          uint64_t *cov_out /* host */, double *est_out /* host */, hipStream_t stream);

/*
 * Influence maximisation with the SKIS sketch: D-SSA (stop-and-stare, doubling) run on IIS
 * samples, as the paper's Sec. 5 and its appendix on D-SSA with SKIS describe.  The graph is
 * preprocessed once.  Iteration t (t = 1, 2, ...) draws the sketch R of sample ids [0, T) and,
 * when needed, the check sketch R^c of ids [T, 2T) from the stream of `seed`; T starts at
 * ceil(Lambda) and doubles each iteration.  The seeds are the greedy of Alg. 3 on R; when
 * Cov_R(seeds) >= Lambda they are estimated on R^c by Eq. (eq21), and the run stops when
 *   eps_t = (eps1 + eps2 + eps1 eps2)(1 - 1/e - eps) + (1 - 1/e) eps3 <= eps, with
 *   eps1 = I_R / I_Rc - 1,  eps2 = eps sqrt(n (1 + eps) / (2^(t-1) I_Rc)),
 *   eps3 = eps sqrt(n (1 + eps)(1 - 1/e - eps) / ((1 + eps/3) 2^(t-1) I_Rc)),
 * or when T reaches N_max (then the last seeds are returned, stopped = 0).  The bounds are
 * D-SSA's with the SKIS coverage threshold of the appendix:
 *   Upsilon(eps, d) = (2 + 2 eps/3) ln(1/d) / eps^2,
 *   N_max = 8 (1 - 1/e) / (2 + 2 eps/3) Upsilon(eps, delta / (6 C(n, k))) n / k,
 *   t_max = ceil(log2(2 N_max / Upsilon(eps, delta / 3))),
 *   Lambda = 1 + (1 + eps)(2 Gamma/n + 2 eps/3) ln(3 t_max / delta) / eps^2.
 * Graph buffers as for skis_build_sketch; seeds (host) receives k node ids in pick order;
 * *info (host) the run's figures.  opt may be NULL (sampler shape, model and max_device_bytes are
 * used; form, inverse index, RIS and budget options are not).  Blocking.  Errors: SKIS_EINVAL
 * (k outside [1, n], eps outside (0, 1 - 1/e), delta outside (0, 1), a malformed graph, or
 * sketches that would need 2^31 ids), SKIS_ENOMEM, SKIS_EHIP.  Gamma = 0 returns
 * SKIS_WDEGENERATE with seeds 0 .. k-1 (I(S) = |S| for every S).
 */
typedef struct skis_dssa_info {
    uint64_t T;                 /* samples in R at the end (R^c holds as many more) */
    uint32_t iterations;        /* iterations run */
    uint32_t stopped;           /* 1: the error condition held; 0: T reached N_max */
    uint64_t cov_select;        /* Cov_R(seeds) */
    uint64_t cov_check;         /* Cov_Rc(seeds) of the last check (0 if none ran) */
    double est_select;          /* I_hat_R(seeds), Eq. eq21 */
    double est_check;           /* I_hat_Rc(seeds) of the last check */
    double eps1, eps2, eps3, eps_t; /* the last check's error terms */
    double Lambda, N_max, t_max; /* the bounds */
    double Gamma;
} skis_dssa_info;

int skis_im_dssa(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w, int32_t k,
                 double eps, double delta, uint64_t seed, const skis_options *opt, hipStream_t stream,
                 int32_t *seeds /* host [k] */, skis_dssa_info *info /* host */);

/* Copies the sketch into caller buffers: sample_ptr int64[T+1], nodes int32[entries],
 * roots int32[T], probed uint64[T].  Any pointer may be NULL. */
int skis_sketch_export(const skis_sketch *sk, int64_t *sample_ptr, int32_t *nodes, int32_t *roots,
                       uint64_t *probed, hipStream_t stream);

/* Copies the node->samples transpose: node_ptr int64[n+1] and node_samples int32[entries]
 * (each list holds the ids j with v in R_j in ascending order).  Either may be NULL. */
int skis_inverse_export(const skis_sketch *sk, int64_t *node_ptr, int32_t *node_samples, hipStream_t stream);

/* Copies q[v] = 1 - gamma_v (fp64, n entries). */
int skis_node_q(const skis_sketch *sk, double *q, hipStream_t stream);

/* Frees the sketch and every device buffer it owns (NULL is a no-op). */
void skis_sketch_free(skis_sketch *sk);

/* Device memory the library keeps for reuse, process-wide.  Blocks that a finished call no longer
 * uses go to a cache of idle blocks (per device, at most cache_keep_bytes; the largest leave first)
 * from which later calls take buffers without a driver call, and the device's stream-ordered pool
 * keeps up to pool_keep_bytes of released memory.  Until this is called each limit is half of the
 * device's memory (a build of 2^26 samples at 1.4B edges uses about 100 GB of transient buffers).
 * Lower limits leave more memory to other users of the GPU (a PyTorch caching allocator, another
 * library); the call trims the current device's cache to the new limit at once.  Sketches and
 * servers keep the buffers they own.  Errors: SKIS_EHIP. */
int skis_set_memory_limits(uint64_t cache_keep_bytes, uint64_t pool_keep_bytes);

/* Gives every idle cached block of the current device back and trims its stream-ordered pool to
 * nothing, after a device synchronisation.  Memory owned by live sketches and servers stays.
 * Errors: SKIS_EHIP. */
int skis_release_cached_memory(void);

/* Message for the last failing call on this thread ("" if none). */
const char *skis_last_error(void);

/* Measurement aid, not a step of the method: reads `reads` rows of `row_bytes` bytes (8, 16,
 * 32, 64 or 128) at uniformly random positions of a device table of `rows` rows
 * (1 <= rows < 2^32, the table 16-byte aligned and at least rows * row_bytes bytes;
 * reads < 2^32), stream-ordered on `stream` and asynchronous.  It measures the achievable
 * bandwidth of random reads of one size, the ceiling for the sampler's random row-bound (8 B)
 * and edge-quad (32 B) reads and for whole cache lines (64 and 128 B); the caller times it.
 * `sink` is one device uint32 that is written only if the folded row words equal a fixed
 * constant.  SKIS_EINVAL for NULL pointers, an unsupported row size or sizes out of range. */
int skis_probe_random_read(const void *table, uint64_t rows, uint32_t row_bytes, uint64_t reads, uint32_t seed,
                           uint32_t *sink, hipStream_t stream);

/*
 * Estimate service over a resident sketch: Alg. 2 answers any seed set from the one
 * sketch (Eq. eq21), so a stream of influence queries is served without touching the
 * graph.  One worker thread per server batches waiting queries continuously: whenever one
 * of pipeline_depth batch slots is free, every waiting query it admits (by count, by total
 * entries, and by sets above 4096 entries) is packed into pinned host memory and sent
 * through copy-in, the estimate kernels and copy-out on the slot's own HIP stream, while
 * the next batch is being formed.  A set whose members' sample lists hold more than 2^18
 * entries in all (a set with a hub) goes in a batch of its own, so that it does not hold
 * the light sets it would have been batched with.  Results are identical to skis_estimate's
 * for the same set, alone or in any mix: every set has its own workgroup, bitmap and
 * summation order.  The sketch must outlive the server; the server does not lock it, and
 * other calls on the sketch (estimate, greedy, export) may run at the same time.  Memory:
 * each slot holds max_batch_queries bitmaps of T bits and max_large_sets bitmaps of n bits
 * on the device; the host keeps a copy of the inverse index's n + 1 offsets.
 */
typedef struct skis_server skis_server;

typedef struct skis_server_options {
    uint32_t pipeline_depth;    /* batches in flight (default 4, one per hardware queue; at most 16) */
    uint32_t max_batch_queries; /* queries per batch (default 256) */
    uint32_t max_batch_entries; /* seed-set entries per batch; also the largest set accepted (default 2^20) */
    uint32_t max_large_sets;    /* sets above 4096 entries per batch (default 4) */
    uint64_t max_device_bytes;  /* 0 = unlimited; larger total allocation -> SKIS_ENOMEM */
} skis_server_options;

typedef struct skis_server_stats {
    uint64_t batches;           /* batches completed */
    uint64_t queries;           /* queries completed */
    uint64_t max_batch;         /* largest batch */
    uint64_t device_bytes;      /* device memory the server holds */
    uint64_t batch_hist[16];    /* batches by size: bucket b counts sizes in [2^b, 2^(b+1)) (b = 15: >= 2^15) */
} skis_server_stats;

/* Fills *opt with the defaults. */
void skis_server_default_options(skis_server_options *opt);

/* Starts a server on the current device over sk (built with the inverse index).
 * Errors: SKIS_EINVAL (NULL arguments, no inverse index, depth > 16), SKIS_ENOMEM. */
int skis_server_create(const skis_sketch *sk, const skis_server_options *opt /* host, may be NULL */,
                       skis_server **out /* host */);

/* Queues one seed set (host array of count node ids, copied before the call returns) and
 * returns its ticket.  Thread-safe.  Errors: SKIS_EINVAL (an id outside [0, n), count < 0
 * or above max_batch_entries), SKIS_EHIP if the worker has stopped on a device error. */
int skis_server_submit(skis_server *sv, const int32_t *nodes /* host */, int32_t count,
                       uint64_t *ticket /* host */);

/* Blocks until the ticket's result is in host memory; returns Cov and I_hat as
 * skis_estimate would, and the time from submission to completion in microseconds.  A
 * ticket can be waited for once.  Thread-safe. */
int skis_server_wait(skis_server *sv, uint64_t ticket, uint64_t *cov /* host */, double *est /* host */,
                     double *latency_us /* host */);

/* Open-loop replay of a query trace (all host arrays): query i (set_nodes[set_ptr[i] ..
 * set_ptr[i+1])) is submitted at arrival_us[i] microseconds after the call starts
 * (nondecreasing), whatever is still in flight; then every result is collected.
 * latency_us[i] runs from the scheduled arrival to the result in host memory, so a
 * submitter that falls behind is charged to the latency.  Output pointers may be NULL. */
int skis_server_replay(skis_server *sv, int32_t num_queries, const int64_t *set_ptr /* [Q+1] */,
                       const int32_t *set_nodes, const double *arrival_us /* [Q] */, uint64_t *cov /* [Q] */,
                       double *est /* [Q] */, double *latency_us /* [Q] */);

/* Counters since creation. */
int skis_server_get_stats(skis_server *sv, skis_server_stats *stats /* host */);

/* Drains the queued queries, stops the worker and frees the server (NULL is a no-op).
 * Results not yet waited for are dropped. */
void skis_server_destroy(skis_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* SKIS_H */
