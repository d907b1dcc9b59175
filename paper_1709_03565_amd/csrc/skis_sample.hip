// skis_sample.hip -- IIS sampling (Alg. 1) and compaction into the CSR sketch (Alg. 2).
//
//   k_roots        one thread per sample: root by the alias table (Eq. probu) and first
//                  live in-edge i* by Eq. (probn) (binary search over the prefix products)
//   k_sample<...>  persistent sampler: every workgroup keeps S samples in flight, each
//                  with its visited set and node list; the unexpanded nodes of all slots
//                  form one flat list of (slot, edge range) items, and the lanes sweep the
//                  edges of all items four at a time (two 16-byte loads and one Philox call
//                  per aligned edge quad).  Tiers 0 and 1 keep the visited set in LDS (an
//                  open-addressing hash) and hand a sample to the next tier when it outgrows
//                  the hash or meets an in-degree above big_row; tier 2 keeps a hash and a
//                  node list sized to the sample in HBM (one sample per one-wave workgroup,
//                  thousands in flight); tier 3 keeps a bitmap of n bits and a node list of
//                  n entries per sample in HBM (one sample per 1024-thread workgroup).
//   k_gather_*     sorts each sample's nodes and writes the CSR in sample order.
//
// Sample j is a pure function of (graph, seed, j): the order in which a sample's nodes are
// discovered changes nothing, because the coins are keyed by (j, edge id) and the sample
// is the set of nodes that reach the root through live edges.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "skis_internal.h"
#include "skis_lt.h"
#include "skis_plain.h"

namespace skis {

constexpr uint32_t DEFERRED = 0xFFFFFFFFu;
constexpr int SMALL_SORT = 1024;   // sizes up to this are sorted in registers by k_gather_sort
constexpr int SORT_LDS_MAX = 8192; // sizes up to this are sorted by k_gather_medium_regs and
                                   // k_gather_block, larger ones through a node bitmap by
                                   // k_gather_large
constexpr int VQ_CAP = 64;        // live edges a wave queues before visiting them
// sample ids taken from the global counter at a time: at least the slots of a workgroup
template <int S>
constexpr int id_batch() { return S <= 16 ? 16 : 32; }

// F_RESUME: admitted this pass from a handover (its nodes are put back in phase B1r)
enum : int { F_ACTIVE = 1, F_ROOTPEND = 2, F_DEFER = 4, F_CLEAR = 8, F_RESUME = 16 };

// ---------------------------------------------------------------------------------------
// Root and first live in-edge of every sample.
//   rec[i] = (root, i*, row begin, row end), u1[i] = col[i*], for sample j = j0 + i.
//   With ris set (plain RIS samples, Sec. 2.3.1): root = the bucket drawn uniformly,
//   rec[i] = (root, row begin - 1, row begin, row end) and u1[i] = -1 -- no first live
//   in-edge, every in-edge of the root flips its own coin.
// ---------------------------------------------------------------------------------------
//   range (device, may be null): {base, count} of a chunk read at launch; the thread then
//   covers i = base .. base+count-1 instead of 0 .. count-1.
__global__ __launch_bounds__(256) void k_roots(uint64_t j0, uint32_t count, const unsigned long long *range,
                                               uint32_t seed_lo, uint32_t seed_hi,
                                               int32_t n, uint64_t C, const AliasEntry *__restrict__ alias,
                                               const int32_t *__restrict__ row_ptr, const double *__restrict__ q,
                                               const double *__restrict__ P, const uint2 *__restrict__ edges,
                                               const uint32_t *__restrict__ wbits, int4 *__restrict__ rec, int32_t *__restrict__ u1, int *__restrict__ err,
                                               int ris)
{
    const uint32_t base = range ? (uint32_t)range[0] : 0u;
    const uint32_t cnt = range ? (uint32_t)range[1] : count;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
        const uint32_t i = base + t;
        const uint64_t j = j0 + i;
        const uint32_t jl = (uint32_t)j, jh = (uint32_t)(j >> 32);
        uint64_t X, Y;
        philox2x64(0u, jl, jh, TAG_ROOT, seed_lo, seed_hi, X, Y);
        const uint64_t b = __umul64hi(X, (uint64_t)n);
        if (ris) {
            const int32_t root = (int32_t)b; // b < n
            const int32_t rb = row_ptr[root], re = row_ptr[root + 1];
            rec[i] = make_int4(root, rb - 1, rb, re);
            u1[i] = -1;
            continue;
        }
        const uint64_t r = __umul64hi(Y, C);
        const AliasEntry ae = alias[b];
        const int32_t root = r < ae.thr ? (int32_t)b : ae.alias;
        if (root < 0 || root >= n) { // cannot happen for a valid table; never index with it
            atomicOr(err, 8);
            rec[i] = make_int4(0, 0, 0, 0);
            u1[i] = 0;
            continue;
        }
        const int32_t rb = row_ptr[root], re = row_ptr[root + 1];
        if (re <= rb) { // a root has gamma > 0, hence an in-edge
            atomicOr(err, 8);
            rec[i] = make_int4(root, rb, rb, rb);
            u1[i] = root;
            continue;
        }
        philox2x64(0u, jl, jh, TAG_FIRST, seed_lo, seed_hi, X, Y);
        const double U = (double)(X >> 11) * 0x1p-53;
        const double theta = __dmul_rn(U, __dsub_rn(1.0, q[root]));
        // first e in the row with 1 - P[e] > theta (1 - P is nondecreasing along the row)
        int32_t lo = rb, hi = re;
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if (__dsub_rn(1.0, P[mid]) > theta) hi = mid; else lo = mid + 1;
        }
        int32_t istar = lo;
        if (istar >= re) { // theta rounded up to gamma: last in-edge of positive probability
            istar = re - 1;
            while (istar > rb && wbits[istar] == 0u) --istar;
        }
        rec[i] = make_int4(root, istar, rb, re);
        u1[i] = (int32_t)edges[istar].x;
    }
}

// The state of a sample handed from one LDS tier to the next as of the start of the pass in
// which it outgrew its slot: its first `count` nodes in discovery order (in the node buffer),
// how many of them were expanded, whether the root's item was still pending, and the edges it
// had probed.  The next tier resumes from there and repeats that pass (the coins depend only
// on (sample, edge), so the set is the same).
struct __align__(16) Handover {
    int32_t count;
    int32_t cursor_rp;        // cursor * 2 + (root item pending)
    unsigned long long probed;
};

// The largest prime below 2^32: for every count below it k -> k * P mod count permutes
// [0, count) (P and count are coprime), and k * P fits in 64 bits for k < 2^32.
constexpr unsigned long long ID_PERM_PRIME = 4294967291ull;

struct SampleArgs {
    int32_t n;
    const int32_t *row_ptr;
    const uint4 *pairs;         // edge records two at a time: (col[2p], th[2p], col[2p+1], th[2p+1]),
                                // th = coin_threshold_hi(w); padded to whole quads of edges
    int64_t nquads;             // pairs holds 2 * nquads records
    const uint32_t *wbits;      // w bits per edge, read when a coin's high half ties th
    const int4 *rec;
    const int32_t *u1;
    uint64_t j0;
    uint32_t seed_lo, seed_hi;
    unsigned long long *next;   // id counter
    const uint32_t *id_list;    // nullptr: ids id_base..id_base+id_count-1; else id_list[0..id_count)
    uint64_t id_count;
    const unsigned long long *id_count_dev; // when set, id_count is read from here at launch
    const unsigned long long *id_base_dev;  // when set, id_base is read from here (else 0)
    // nonzero: the k-th id taken is id_list[(k * ID_PERM_PRIME) mod id_count], a fixed
    // scramble of the list's order (a bijection for counts below the prime); 0: id_list[k]
    uint32_t id_perm;
    uint32_t big_row;
    int32_t *staging;
    unsigned long long stage_cap;
    unsigned long long *stage_used;
    uint32_t *out_size;
    unsigned long long *out_off;
    unsigned long long *out_probed;
    uint32_t *deferred;
    unsigned long long *n_deferred;
    uint32_t *medium;
    unsigned long long *n_medium;
    int *overflow;
    unsigned long long *tier_stats; // [5]: samples finished by this launch, their entries, their edges
                                    // probed; the edges and the nodes (items) this launch expanded
    uint32_t *gbits;            // bitmap tier: [slots][words]
    int32_t *glist;             // bitmap tier: [slots][n]
    uint64_t words;
    int32_t *ghash;             // hash tier: [slots][HCAP], -1 = empty (every launch leaves it so)
    uint2 *glist2;              // hash tier: [slots][RCAP] (node id, its hash slot) in discovery order
    // handover to the next tier: sample k of `deferred` (k < ho_cap_out) leaves its state in
    // ho_state_out[k] and its nodes in ho_nodes_out[k * ho_stride_out ...]
    Handover *ho_state_out;
    int32_t *ho_nodes_out;
    uint64_t ho_cap_out;
    int32_t ho_stride_out;
    // handover from the previous tier: the id at position p of id_list resumes from record
    // ho_slot_in[p] (p itself when ho_slot_in is null) if that is below ho_cap_in
    const Handover *ho_state_in;
    const int32_t *ho_nodes_in;
    const uint32_t *ho_slot_in;
    uint64_t ho_cap_in;
    int32_t ho_stride_in;
};

// RCAP: nodes a slot holds before its sample moves on (the visited threshold); HCAP: size
// of the slot's open-addressing hash, any size above RCAP (about 4/3 RCAP keeps the load
// factor at most 3/4 while leaving LDS for more slots).
// ICAP: items (pending nodes over all slots) expanded per pass; QPL: most edge quads (aligned
// groups of four edges, one Philox call) a lane takes per sweep (2 keeps more loads in
// flight, 1 needs fewer registers).
// TIER: 0 the first LDS tier (hands its overflowing samples on with their state), 1 the
// second LDS tier (resumes them and hands its own on), 2 the HBM hash tier (a hash of HCAP
// slots and a list of RCAP nodes per sample in global memory; resumes and hands on), 3 the
// HBM bitmap tier (a bitmap of n bits and a list of n nodes per sample; finishes every sample).
// Arguments used once per pass or less are read from the argument segment where they are used
// (see karg_at); the ones the edge sweep uses every pass stay in scalar registers.  SampleArgs is
// k_sample's only parameter, so it starts the segment and a field's offset is its offsetof.
#define SKIS_KARG(f) karg_at<decltype(SampleArgs::f)>(offsetof(SampleArgs, f))
static_assert(std::is_standard_layout<SampleArgs>::value, "argument offsets need a standard layout");

// Five waves a SIMD for the default tier-0 shape: its registers fit in 96 (one value spilled,
// reloaded once a pass); left to itself the compiler takes 98 and four waves.  Six for the
// HBM hash tier, whose samples wait on memory more than on anything else: 80 registers and a
// few spilled values (59 ms at 1.4B edges against 62-65 with five waves, 61 with eight; with
// a half or a quarter of the workgroups in flight it took 98 and 148 ms).
template <int S, int RCAP, int QPL, int TIER> constexpr int sample_min_waves()
{
    return TIER == 0 && S <= 4 && RCAP <= 192 && QPL == 1 ? 5 : TIER == 2 ? 6 : 1;
}

template <int BLOCK, int S, int RCAP, int HCAP, int ICAP, int QPL, int TIER>
__global__ __launch_bounds__(BLOCK, (sample_min_waves<S, RCAP, QPL, TIER>())) void k_sample(SampleArgs a)
{
    constexpr bool GLOBAL = TIER == 3; // bitmap visited sets: a sample never outgrows them
    constexpr bool GHASH = TIER == 2;  // hash visited sets in global memory
    constexpr bool LDSV = TIER <= 1;   // hash visited sets in LDS
    constexpr bool HO_OUT = TIER <= 2, HO_IN = TIER >= 1;
    constexpr int IDBATCH = id_batch<S>();
    static_assert(GLOBAL || HCAP > RCAP, "the hash must be larger than the node list");
    static_assert(!LDSV || HCAP <= 65535, "list entries are 8- or 16-bit hash slot indexes");
    static_assert(!GHASH || BLOCK == 64, "the hash tier's workgroups are one wave");
    constexpr int HSZ = LDSV ? S * HCAP : 1;
    constexpr int LSZ = LDSV ? S * RCAP : 1;
    constexpr int IPT = (ICAP + BLOCK - 1) / BLOCK;
    static_assert(S <= 64, "slots are owned by the lanes of wave 0");
    static_assert(IDBATCH >= S, "one refill must cover every empty slot");

    __shared__ int32_t sh_hash[HSZ];
    // LDS tiers: the node list holds the hash slot of each node in discovery order (the
    // slot holds the node id), a quarter or half the bytes of a list of ids
    using LIdx = std::conditional_t<(HCAP <= 256), uint8_t, uint16_t>;
    __shared__ LIdx sh_lidx[LSZ];
    __shared__ uint32_t s_idx[S];
    __shared__ int32_t s_count[S], s_cursor[S], s_flags[S], s_rib[S], s_rie[S];
    __shared__ unsigned long long s_probed[S];
    // phase B1 work of a slot: s_wo_cnt >= 0 entries to write at s_wo_off, -1 a hand-on
    // without handover, -2 a hand-on whose nodes go to handover s_wo_off; a slot flagged
    // F_RESUME refills from handover s_wo_off
    __shared__ int32_t s_wo_cnt[S];
    __shared__ unsigned long long s_wo_off[S];
    __shared__ Handover s_snap[HO_OUT ? S : 1]; // each slot's state at the start of the pass
    __shared__ int32_t s_ibase[S + 1], s_ifirst[S], s_irp[S];
    __shared__ int32_t it_beg[ICAP], it_end[ICAP], it_pb[ICAP + 1];
    __shared__ uint8_t it_slot[ICAP];
    __shared__ int32_t s_nitems, s_alive;
    __shared__ unsigned long long s_idnext, s_idend;
    // the root records of the last two id batches, loaded when a batch is taken, so that
    // admitting a sample costs no global round trip: [buffer][id - base]
    __shared__ int4 s_crec[2][IDBATCH];
    __shared__ int32_t s_cu1[2][IDBATCH];
    __shared__ uint32_t s_cidx[2][IDBATCH];
    __shared__ unsigned long long s_cbase[2];
    __shared__ int s_ccur;
    __shared__ int32_t s_scan[BLOCK / 64 + 1];
    // one-wave workgroups find an item's slot (one item per lane) and, in every sweep, a lane's
    // item (lane i holding item i's quad range) by a prefix maximum over the lanes instead of
    // a binary search: s_imap[i] = slot + 1 of the slot whose items start at i, s_qmap[p] =
    // item + 1 of the non-empty item whose quads start at position p of the sweep (or before
    // it, at p = 0), 0 elsewhere
    constexpr bool WMAP_SLOT = BLOCK == 64 && IPT == 1;
    // (one quad a lane only: with two, the marks cost tier 1 more than its searches)
    constexpr bool WMAP_QUAD = BLOCK == 64 && ICAP <= 64 && QPL == 1;
    __shared__ uint32_t s_imap[WMAP_SLOT ? 64 : 1];
    __shared__ uint32_t s_qmap[WMAP_QUAD ? 64 : 1];
    // per wave: the live edges of the pass's sweeps not yet visited (node, slot)
    __shared__ int32_t s_vq_node[(BLOCK / 64) * VQ_CAP];
    __shared__ uint8_t s_vq_slot[(BLOCK / 64) * VQ_CAP];

    const int tid = threadIdx.x;
    const int32_t n = a.n;
    // the work of this launch; in a captured chain the previous kernel has written it
    const unsigned long long id_count = SKIS_KARG(id_count_dev) ? *SKIS_KARG(id_count_dev) : SKIS_KARG(id_count);
    // position in id_list (and in the handover records) of the k-th id taken
    const bool perm = SKIS_KARG(id_perm) && id_count < ID_PERM_PRIME;
    auto list_pos = [&](unsigned long long k) -> unsigned long long {
        return perm ? (k * ID_PERM_PRIME) % id_count : k;
    };
    const unsigned long long id_base = SKIS_KARG(id_base_dev) ? *SKIS_KARG(id_base_dev) : 0ull;

    auto list_ptr = [&](int s) -> int32_t * { return a.glist + ((size_t)blockIdx.x * S + s) * (size_t)n; };
    auto ghash_ptr = [&](int s) -> int32_t * { return a.ghash + ((size_t)blockIdx.x * S + s) * (size_t)HCAP; };
    auto glist2_ptr = [&](int s) -> uint2 * { return a.glist2 + ((size_t)blockIdx.x * S + s) * (size_t)RCAP; };
    // node at position t of slot s's list
    auto list_node = [&](int s, int t) -> int32_t {
        if constexpr (GLOBAL) return list_ptr(s)[t];
        else if constexpr (GHASH) return (int32_t)glist2_ptr(s)[t].x;
        else return sh_hash[s * HCAP + sh_lidx[s * RCAP + t]];
    };
    auto bits_ptr = [&](int s) -> uint32_t * { return a.gbits + ((size_t)blockIdx.x * S + s) * a.words; };
    // The hash tier keeps its visited sets and lists in global memory, written by some lanes
    // and read by others after a barrier: its barriers order global memory at workgroup scope
    // (the stores have completed before any lane goes on).  The LDS tiers need LDS order only.
    auto bsync = [&]() {
        if constexpr (GHASH) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        } else {
            block_sync<BLOCK>();
        }
    };

    // Home slot of node u in an HCAP-entry hash: multiplicative hashing, then the high
    // half of the product with HCAP maps the 32-bit hash onto [0, HCAP).
    auto hash_slot = [](int32_t u) -> uint32_t {
        return (uint32_t)(((uint64_t)((uint32_t)u * 0x9E3779B1u) * (uint64_t)HCAP) >> 32);
    };

    // Inserts u into an HCAP-slot hash in global memory (linear probing from its home slot);
    // returns the slot it took, -1 if u was there already, -2 if the hash is full.
    auto ghash_insert = [&](int32_t *H, int32_t u) -> int {
        uint32_t h = hash_slot(u);
#pragma unroll 1
        for (int k = 0; k < HCAP; ++k) {
            const int32_t old = atomicCAS(&H[h], -1, u);
            if (old == -1) return (int)h;
            if (old == u) return -1;
            h = h + 1 == (uint32_t)HCAP ? 0u : h + 1;
        }
        return -2;
    };

    // Adds u to slot s's sample if it is not there yet.
    auto visit = [&](int s, int32_t u) {
        if constexpr (GHASH) {
            // a sample already handed on restarts from its snapshot in the next tier
            if (s_flags[s] & F_DEFER) return;
            const int h = ghash_insert(ghash_ptr(s), u);
            if (h >= 0) {
                const int pos = atomicAdd(&s_count[s], 1);
                if (pos < RCAP) glist2_ptr(s)[pos] = make_uint2((uint32_t)u, (uint32_t)h);
                else atomicOr(&s_flags[s], F_DEFER);
            } else if (h == -2) {
                atomicOr(&s_flags[s], F_DEFER);
            }
        } else if constexpr (GLOBAL) {
            const uint32_t bit = 1u << (u & 31);
            const uint32_t old = atomicOr(bits_ptr(s) + (u >> 5), bit);
            if (!(old & bit)) {
                const int pos = atomicAdd(&s_count[s], 1);
                list_ptr(s)[pos] = u;
            }
        } else {
            int32_t *H = sh_hash + s * HCAP;
            uint32_t h = hash_slot(u);
#pragma unroll 1
            for (int k = 0; k < HCAP; ++k) {
                const int32_t old = atomicCAS(&H[h], -1, u);
                if (old == -1) {
                    const int pos = atomicAdd(&s_count[s], 1);
                    if (pos < RCAP) sh_lidx[s * RCAP + pos] = (LIdx)h;
                    else atomicOr(&s_flags[s], F_DEFER);
                    return;
                }
                if (old == u) return;
                h = h + 1 == (uint32_t)HCAP ? 0u : h + 1;
            }
            atomicOr(&s_flags[s], F_DEFER);
        }
    };

    // lane s of wave 0 counts what slot s finishes; summed once when the workgroup exits
    unsigned long long st_fin = 0, st_ent = 0, st_prb = 0;
    // every lane counts the edges and items it sets up (the work of this launch)
    unsigned long long st_swp = 0, st_itm = 0;
    if constexpr (!GLOBAL)
        for (int i = tid; i < HSZ; i += BLOCK) sh_hash[i] = -1;
    if (tid < S) {
        s_flags[tid] = 0;
        s_wo_cnt[tid] = 0;
    }
    if (tid == 0) {
        s_idnext = 0;
        s_idend = 0;
        s_cbase[0] = s_cbase[1] = ~0ull;
        s_ccur = 0;
    }
    // staging space is reserved STAGE_CHUNK entries at a time per workgroup (lane 0 of
    // wave 0 keeps the open chunk [st_base, st_end)); the HBM tiers reserve exactly
    constexpr unsigned long long STAGE_CHUNK = LDSV ? 8ull * S * RCAP : 0ull;
    unsigned long long st_base = 0, st_end = 0;
    bsync();

    for (;;) {
        // ---- A1: wave 0, lane s owns slot s: finished and handed-on samples -----------------
        if (tid < 64) {
            const int s = tid;
            const bool own = s < S;
            int f = own ? s_flags[s] : 0;
            if constexpr (HO_IN) {
                if (f & F_RESUME) { // refilled in the last pass's phase B1r
                    f &= ~F_RESUME;
                    s_flags[s] = f;
                }
            }
            // finished samples of this pass take their staging space from the workgroup's
            // open chunk, which is refilled with one atomic when it runs short
            const bool fin = own && (f & F_ACTIVE) && !(!GLOBAL && (f & F_DEFER)) && !(f & F_ROOTPEND) &&
                             s_cursor[s] >= s_count[s];
            // scans over the S slot lanes only (the others hold zeros); totals from lane S - 1
            const uint32_t fcnt = fin ? (uint32_t)s_count[s] : 0u;
            const uint32_t fincl = wave_incl_scan_n<S>(fcnt);
            const unsigned long long ftot = lane_value(fincl, S - 1);
            unsigned long long fbase = 0;
            if (s == 0 && ftot) {
                if (st_base + ftot > st_end) {
                    const unsigned long long want = ftot > STAGE_CHUNK ? ftot : STAGE_CHUNK;
                    st_base = atomicAdd(SKIS_KARG(stage_used), want);
                    st_end = st_base + want;
                }
                fbase = st_base;
                st_base += ftot;
            }
            fbase = first_lane_value64(fbase); // lane 0: every lane of the wave is active here
            if (own && (f & F_ACTIVE)) {
                if (!GLOBAL && (f & F_DEFER)) {
                    const uint32_t i = s_idx[s];
                    const unsigned long long k = atomicAdd(SKIS_KARG(n_deferred), 1ull);
                    SKIS_KARG(deferred)[k] = i;
                    SKIS_KARG(out_size)[i] = DEFERRED;
                    s_wo_cnt[s] = -1; // nothing to write; its hash may hold keys past the list
                    if constexpr (HO_OUT) {
                        if (SKIS_KARG(ho_state_out) && k < SKIS_KARG(ho_cap_out)) {
                            SKIS_KARG(ho_state_out)[k] = s_snap[s]; // its nodes follow in phase B1
                            s_wo_cnt[s] = -2;
                            s_wo_off[s] = k;
                        }
                    }
                    f = F_CLEAR;
                    s_flags[s] = f;
                } else if (fin) {
                    const uint32_t i = s_idx[s];
                    const int cnt = s_count[s];
                    const unsigned long long off = fbase + (unsigned long long)(fincl - fcnt);
                    SKIS_KARG(out_size)[i] = (uint32_t)cnt;
                    SKIS_KARG(out_off)[i] = off;
                    SKIS_KARG(out_probed)[i] = s_probed[s];
                    st_fin += 1;
                    st_ent += (unsigned long long)cnt;
                    st_prb += s_probed[s];
                    if (cnt > SMALL_SORT) {
                        const unsigned long long k = atomicAdd(SKIS_KARG(n_medium), 1ull);
                        SKIS_KARG(medium)[k] = i;
                    }
                    if (off + (unsigned long long)cnt <= SKIS_KARG(stage_cap)) {
                        s_wo_cnt[s] = cnt;
                        s_wo_off[s] = off;
                    } else {
                        s_wo_cnt[s] = 0;
                        atomicOr(SKIS_KARG(overflow), 1);
                    }
                    f = F_CLEAR;
                    s_flags[s] = f;
                }
            }
        }
        bsync();

        // ---- B1: write out finished samples, clear their visited sets ----------------------
        // (before admission, so that a slot finished in this pass takes its next sample now)
        for (int s = 0; s < S; ++s) {
            const int fs = s_flags[s];
            if (fs != F_CLEAR) continue;
            const int cnt = s_wo_cnt[s];
            const unsigned long long off = s_wo_off[s];
            if constexpr (GHASH) {
                int32_t *H = ghash_ptr(s);
                const uint2 *GL = glist2_ptr(s);
                if (cnt < 0) { // a sample handed on: its nodes to the handover, then a full clear
                    if (cnt == -2) {
                        const int c = s_snap[s].count;
                        int32_t *dst = SKIS_KARG(ho_nodes_out) + (size_t)off * (size_t)SKIS_KARG(ho_stride_out);
                        for (int t = tid; t < c; t += BLOCK) dst[t] = (int32_t)GL[t].x;
                    }
                    for (int t = tid; t < HCAP; t += BLOCK) H[t] = -1;
                } else {
                    // a finished sample holds every key in its list: write them and clear their slots
                    const int rc = s_count[s];
                    for (int t = tid; t < rc; t += BLOCK) {
                        const uint2 e = GL[t];
                        if (t < cnt) SKIS_KARG(staging)[off + t] = (int32_t)e.x;
                        H[e.y] = -1;
                    }
                }
            } else if constexpr (!GLOBAL) {
                if (cnt < 0) { // a sample handed on: its nodes to the handover, then a full clear
                    if (HO_OUT && cnt == -2) {
                        const int c = s_snap[s].count;
                        int32_t *dst = SKIS_KARG(ho_nodes_out) + (size_t)off * (size_t)SKIS_KARG(ho_stride_out);
                        for (int t = tid; t < c; t += BLOCK) dst[t] = sh_hash[s * HCAP + sh_lidx[s * RCAP + t]];
                        bsync();
                    }
                    for (int t = tid; t < HCAP; t += BLOCK) sh_hash[s * HCAP + t] = -1;
                } else {
                    // a finished sample has every key in its list: write the first cnt
                    // (all, unless staging overflowed) and clear exactly the slots it used
                    const int rc = s_count[s];
                    for (int t = tid; t < rc; t += BLOCK) {
                        const int h = sh_lidx[s * RCAP + t];
                        if (t < cnt) SKIS_KARG(staging)[off + t] = sh_hash[s * HCAP + h];
                        sh_hash[s * HCAP + h] = -1;
                    }
                }
            } else {
                int32_t *L = list_ptr(s);
                uint32_t *B = bits_ptr(s);
                for (int t = tid; t < cnt; t += BLOCK) SKIS_KARG(staging)[off + t] = L[t];
                const int rc = s_count[s];
                for (int t = tid; t < rc; t += BLOCK) B[L[t] >> 5] = 0u;
            }
        }
        bsync();
        if (tid < S && s_flags[tid] == F_CLEAR) {
            s_flags[tid] = 0;
            s_wo_cnt[tid] = 0;
        }

        // ---- A2: wave 0 again: admission, the handover snapshot, the pass's items -----------
        if (tid < 64) {
            const int s = tid;
            const bool own = s < S;
            int f = own ? s_flags[s] : 0;
            // admission into every empty slot, those finished above included
            const bool want = own && f == 0;
            const unsigned long long wmask = __ballot(want);
            const int nwant = __popcll(wmask);
            if (nwant > 0) {
                const int rank = __popcll(wmask & ((1ull << s) - 1ull));
                const unsigned long long idnext = s_idnext, idend = s_idend;
                const unsigned long long avail = idend - idnext;
                unsigned long long nb = 0;
                int cur = s_ccur;
                if (avail < (unsigned long long)nwant) {
                    if (s == 0) nb = atomicAdd(SKIS_KARG(next), (unsigned long long)IDBATCH);
                    nb = first_lane_value64(nb);
                    // load the new batch's records into the other buffer (lane l: id nb + l)
                    cur ^= 1;
                    if (s < IDBATCH) {
                        const unsigned long long id = nb + (unsigned long long)s;
                        if (id < id_count) {
                            const uint32_t i = SKIS_KARG(id_list) ? SKIS_KARG(id_list)[list_pos(id)] : (uint32_t)(id_base + id);
                            s_cidx[cur][s] = i;
                            s_crec[cur][s] = SKIS_KARG(rec)[i];
                            s_cu1[cur][s] = SKIS_KARG(u1)[i];
                        }
                    }
                    if (s == 0) {
                        s_cbase[cur] = nb;
                        s_ccur = cur;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                const unsigned long long myid =
                    (unsigned long long)rank < avail ? idnext + rank : nb + (rank - avail);
                if (s == 0) {
                    if (avail >= (unsigned long long)nwant) {
                        s_idnext = idnext + nwant;
                    } else {
                        s_idnext = nb + (nwant - avail);
                        s_idend = nb + IDBATCH;
                    }
                }
                if (want && myid < id_count) {
                    // the id is in the newest batch or in the remainder of the one before
                    const int b = (myid - s_cbase[cur] < (unsigned long long)IDBATCH) ? cur : (cur ^ 1);
                    const unsigned long long cd = myid - s_cbase[b];
                    const int c = cd < (unsigned long long)IDBATCH ? (int)cd : 0;
                    const uint32_t i = s_cidx[b][c];
                    const int4 r = s_crec[b][c];
                    const int32_t u = s_cu1[b][c];
                    // a RIS record has no first live in-edge: u = -1 and i* = row begin - 1
                    const bool ris_rec = u == -1;
                    if (cd >= (unsigned long long)IDBATCH || i >= (uint32_t)(id_base + (SKIS_KARG(id_list) ? 0x7FFFFFFFull : id_count)) ||
                        (uint32_t)r.x >= (uint32_t)n ||
                        (ris_rec ? (r.y != r.z - 1 || r.w < r.z) : ((uint32_t)u >= (uint32_t)n || r.y < r.z || r.w <= r.y)) ||
                        (int64_t)r.w > 4 * a.nquads) {
                        atomicOr(SKIS_KARG(overflow), 8); // bounds guard: the sample is left out
                    } else {
                    s_idx[s] = i;
                    s_rib[s] = r.y + 1;
                    s_rie[s] = r.w;
                    s_probed[s] = (unsigned long long)(r.w - r.z);
                    s_count[s] = ris_rec ? 1 : 2;
                    s_cursor[s] = 1;
                    int nf = F_ACTIVE | (r.y + 1 < r.w ? F_ROOTPEND : 0);
                    if (!GLOBAL && (uint32_t)(r.w - r.z) > a.big_row) nf |= F_DEFER;
                    bool resumed = false;
                    if constexpr (HO_IN) {
                        const uint32_t *hs = SKIS_KARG(ho_slot_in);
                        const unsigned long long rec_k = hs ? (unsigned long long)hs[myid] : list_pos(myid);
                        if (SKIS_KARG(ho_state_in) && rec_k < SKIS_KARG(ho_cap_in)) {
                            const Handover h = SKIS_KARG(ho_state_in)[rec_k];
                            const int cur = h.cursor_rp >> 1;
                            const int cap = GLOBAL ? n : RCAP; // the bitmap tier's list holds n nodes
                            if (h.count >= 1 && h.count <= cap && cur >= 1 && cur <= h.count) {
                                // its nodes are put back into the visited set and list in phase B1r
                                resumed = true;
                                s_count[s] = h.count;
                                s_cursor[s] = cur;
                                s_probed[s] = h.probed;
                                nf = F_ACTIVE | F_RESUME | ((h.cursor_rp & 1) ? F_ROOTPEND : 0);
                                if (!GLOBAL && (uint32_t)(r.w - r.z) > a.big_row) nf |= F_DEFER;
                                s_wo_off[s] = rec_k;
                            }
                        }
                    }
                    if (resumed) {
                    } else if constexpr (GHASH) {
                        // root and u1 differ (no self-loops), so they take two slots
                        int32_t *H = ghash_ptr(s);
                        uint2 *GL = glist2_ptr(s);
                        const int32_t keys[2] = {r.x, u};
                        for (int t = 0; t < (ris_rec ? 1 : 2); ++t)
                            GL[t] = make_uint2((uint32_t)keys[t], (uint32_t)ghash_insert(H, keys[t]));
                    } else if constexpr (GLOBAL) {
                        int32_t *L = list_ptr(s);
                        uint32_t *B = bits_ptr(s);
                        L[0] = r.x;
                        atomicOr(B + (r.x >> 5), 1u << (r.x & 31));
                        if (!ris_rec) {
                            L[1] = u;
                            atomicOr(B + (u >> 5), 1u << (u & 31));
                        }
                    } else {
                        // root and u1 differ (no self-loops), so they take two slots
                        int32_t *H = sh_hash + s * HCAP;
                        const int32_t keys[2] = {r.x, u};
                        for (int t = 0; t < (ris_rec ? 1 : 2); ++t) {
                            uint32_t h = hash_slot(keys[t]);
                            while (H[h] != -1) h = h + 1 == (uint32_t)HCAP ? 0u : h + 1;
                            H[h] = keys[t];
                            sh_lidx[s * RCAP + t] = (LIdx)h;
                        }
                    }
                    f = nf;
                    s_flags[s] = f;
                    }
                }
            }
            // the state a handover would carry if this pass outgrows the slot
            if constexpr (HO_OUT) {
                if (SKIS_KARG(ho_state_out) && own && (f & F_ACTIVE)) {
                    Handover h;
                    h.count = s_count[s];
                    h.cursor_rp = s_cursor[s] * 2 + ((f & F_ROOTPEND) ? 1 : 0);
                    h.probed = s_probed[s];
                    s_snap[s] = h;
                }
            }
            // items: the root item (edges after i*) and then unexpanded nodes, slot by slot
            int pend = 0, rp = 0;
            if (own && (f & F_ACTIVE) && !(f & F_DEFER)) {
                rp = (f & F_ROOTPEND) ? 1 : 0;
                int lim = s_count[s];
                if (!GLOBAL && lim > RCAP) lim = RCAP;
                const int rest = lim - s_cursor[s];
                pend = rp + (rest > 0 ? rest : 0);
            }
            const int incl = wave_incl_scan_n<S>(pend);
            const int base = incl - pend;
            int take = ICAP - base;
            take = take < 0 ? 0 : (take > pend ? pend : take);
            const int tincl = wave_incl_scan_n<S>(take);
            if constexpr (WMAP_SLOT) {
                s_imap[s] = 0u;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (own && take > 0) s_imap[tincl - take] = (uint32_t)s + 1u; // below nitems <= 64
            }
            if (own) {
                s_ibase[s] = tincl - take;
                s_ifirst[s] = s_cursor[s];
                const int trp = take > 0 ? rp : 0;
                s_irp[s] = trp;
                if (take > 0) {
                    s_cursor[s] += take - trp;
                    if (trp) {
                        f &= ~F_ROOTPEND;
                        s_flags[s] = f;
                    }
                }
            }
            const int total = (int)lane_value((uint32_t)tincl, S - 1);
            // the workgroup stays while a slot is active: admission has filled every empty
            // slot while ids remain, so an idle workgroup holds no id taken from the counter
            const unsigned long long amask = __ballot(own && (f & F_ACTIVE));
            if (s == 0) {
                s_ibase[S] = total;
                s_nitems = total;
                s_alive = amask != 0ull;
            }
        }
        bsync();

        // ---- B1r: resumed samples (admitted above) put their nodes back into hash and list ---
        if constexpr (HO_IN) {
            for (int s = 0; s < S; ++s) {
                if (!(s_flags[s] & F_RESUME)) continue;
                const int c = s_count[s];
                const int32_t *src = SKIS_KARG(ho_nodes_in) + (size_t)s_wo_off[s] * (size_t)SKIS_KARG(ho_stride_in);
                if constexpr (GLOBAL) {
                    int32_t *L = list_ptr(s);
                    uint32_t *B = bits_ptr(s);
                    for (int t = tid; t < c; t += BLOCK) {
                        const int32_t u = src[t];
                        L[t] = u;
                        atomicOr(B + (u >> 5), 1u << (u & 31));
                    }
                } else if constexpr (GHASH) {
                    // distinct nodes, fewer than HCAP: each finds an empty slot
                    int32_t *H = ghash_ptr(s);
                    uint2 *GL = glist2_ptr(s);
                    for (int t = tid; t < c; t += BLOCK) {
                        const int32_t u = src[t];
                        GL[t] = make_uint2((uint32_t)u, (uint32_t)ghash_insert(H, u));
                    }
                } else {
                    int32_t *H = sh_hash + s * HCAP;
                    for (int t = tid; t < c; t += BLOCK) {
                        const int32_t u = src[t];
                        uint32_t h = hash_slot(u);
                        for (int k = 0; k < HCAP && atomicCAS(&H[h], -1, u) != -1; ++k)
                            h = h + 1 == (uint32_t)HCAP ? 0u : h + 1;
                        sh_lidx[s * RCAP + t] = (LIdx)h;
                    }
                }
            }
            bsync();
        }

        // ---- B2: item edge ranges ----------------------------------------------------------
        const int nitems = s_nitems;
        if (nitems > 0) {
            // item it = k * BLOCK + tid (nitems <= ICAP <= IPT * BLOCK): first the node of each
            // item, then all row-bound loads unconditionally (node 0 stands in where there is
            // none), then the ranges
            const int mapped_sl = WMAP_SLOT ? (int)wave_incl_max_dpp(s_imap[tid]) - 1 : 0;
            int xs[IPT], ss[IPT];
            bool rootit[IPT];
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const int it = k * BLOCK + tid;
                ss[k] = -1;
                xs[k] = 0;
                rootit[k] = false;
                if (it < nitems) {
                    int sl = mapped_sl;
                    if constexpr (!WMAP_SLOT) {
                        int lo = 0, hi = S;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (s_ibase[mid] <= it) lo = mid + 1; else hi = mid;
                        }
                        sl = lo - 1;
                    }
                    const int t = it - s_ibase[sl];
                    ss[k] = sl;
                    if (s_irp[sl] && t == 0) {
                        rootit[k] = true;
                    } else {
                        const int32_t x = list_node(sl, s_ifirst[sl] + t - s_irp[sl]);
                        if ((uint32_t)x >= (uint32_t)n) { // bounds guard: report, never index
                            atomicOr(SKIS_KARG(overflow), 4);
                            xs[k] = -1;
                        } else {
                            xs[k] = x;
                        }
                    }
                }
            }
            int rb[IPT], re[IPT];
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const int32_t xc = xs[k] >= 0 ? xs[k] : 0;
                rb[k] = a.row_ptr[xc];
                re[k] = a.row_ptr[xc + 1];
            }
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const int it = k * BLOCK + tid;
                const int sl = ss[k];
                if (sl < 0) continue;
                int beg, end;
                if (rootit[k]) {
                    beg = s_rib[sl];
                    end = s_rie[sl];
                } else {
                    beg = xs[k] >= 0 ? rb[k] : 0;
                    end = xs[k] >= 0 ? re[k] : 0;
                    atomicAdd(&s_probed[sl], (unsigned long long)(end - beg));
                    if (!GLOBAL && (uint32_t)(end - beg) > a.big_row) {
                        atomicOr(&s_flags[sl], F_DEFER);
                        end = beg;
                    }
                }
                st_swp += (unsigned long long)(end - beg);
                st_itm += 1;
                it_slot[it] = (uint8_t)sl;
                it_beg[it] = beg;
                it_end[it] = end;
                it_pb[it] = end > beg ? ((end - 1) >> 2) - (beg >> 2) + 1 : 0;
            }
        }
        bsync();

        // ---- B3: prefix sum of edge quads over the items -----------------------------------
        {
            int loc[IPT], cnt[IPT];
            int acc = 0;
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const int idx = tid * IPT + k;
                const int v = idx < nitems ? it_pb[idx] : 0;
                loc[k] = acc;
                cnt[k] = v;
                acc += v;
            }
            int tot;
            const int ex = block_excl_scan<BLOCK, int>(acc, s_scan, &tot);
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const int idx = tid * IPT + k;
                if (idx < nitems) it_pb[idx] = ex + loc[k];
            }
            if (tid == 0) it_pb[nitems] = tot;
            if constexpr (WMAP_QUAD) s_qmap[tid] = 0u;
        }
        bsync();

        // ---- B4: live-edge coins for every edge quad, visits ------------------------------
        // Each lane takes qpl consecutive quads (qpl = the fewest, up to QPL, that cover the
        // pass in one sweep; uniform over the workgroup): one search for the first quad's
        // item, the next ones by stepping across item boundaries; all loads are issued
        // before the coins are drawn.  One Philox call gives the high halves of a quad's
        // four coins; a high half equal to the edge's threshold (probability 2^-32) is
        // settled on the whole coin after the sweep.
        const int total = it_pb[nitems];
        const int qpl = total >= BLOCK * QPL ? QPL : (total + BLOCK - 1) / BLOCK;
        // one-wave workgroups: this lane's item's quads [my_qb, my_qe) (empty past nitems)
        int my_qb = 0, my_qe = 0;
        if constexpr (WMAP_QUAD) {
            if (tid < nitems) {
                my_qb = it_pb[tid];
                my_qe = it_pb[tid + 1];
            }
        }
        // The live edges a sweep finds join the wave's queue, and the queue is visited (the
        // visited-set inserts, one entry a lane) when it could not take the next sweep's and
        // after the last sweep: the inserts run with most lanes busy instead of with the few
        // lanes that hold a live edge in a sweep.  The nodes a pass adds are expanded in later
        // passes only, so when they are inserted within the pass does not matter.  Every lane
        // of a wave runs the same number of sweeps (the wave-level scan needs them all).
        int32_t *const vq_node = s_vq_node + (tid >> 6) * VQ_CAP;
        uint8_t *const vq_slot = s_vq_slot + (tid >> 6) * VQ_CAP;
        uint32_t vq_n = 0; // entries in the wave's queue (the same in every lane)
        auto vq_flush = [&]() {
            if (vq_n == 0) return;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (uint32_t i = (uint32_t)(tid & 63); i < vq_n; i += 64) visit((int)vq_slot[i], vq_node[i]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            vq_n = 0;
        };
        for (int base0 = 0; base0 < total; base0 += BLOCK * qpl) {
            const int base = base0 + tid * qpl; // past total: no quad (the lane still takes part)
            int lo = 0; // last item whose first quad index is <= base
            if constexpr (WMAP_QUAD) {
                // every item that overlaps the sweep marks where it starts in it (0 if before);
                // the largest mark at or before a lane's quad is its item
                if (my_qe > my_qb && my_qb < base0 + 64 && my_qe > base0)
                    s_qmap[max(my_qb - base0, 0)] = (uint32_t)tid + 1u;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                lo = max((int)wave_incl_max_dpp(s_qmap[tid]) - 1, 0);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                s_qmap[tid] = 0u;
            } else {
                int hi = nitems - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (it_pb[mid] <= base) lo = mid; else hi = mid - 1;
                }
            }
            int pq[QPL], ps[QPL];
            uint32_t pin[QPL]; // edges of the quad inside the item's range, one bit each
#pragma unroll
            for (int g = 0; g < QPL; ++g) {
                const int idx = base + g;
                ps[g] = -1;
                pq[g] = 0;
                pin[g] = 0u;
                if (g >= qpl || idx >= total) continue;
                while (it_pb[lo + 1] <= idx) ++lo; // it_pb[nitems] = total > idx
                const int sl = it_slot[lo];
                if (!GLOBAL && (s_flags[sl] & F_DEFER)) continue;
                const int q = (it_beg[lo] >> 2) + (idx - it_pb[lo]);
                if (q < 0 || (int64_t)q >= a.nquads) { // bounds guard: report, never index
                    atomicOr(SKIS_KARG(overflow), 2);
                    continue;
                }
                ps[g] = sl;
                pq[g] = q;
                const int lead = max(it_beg[lo] - 4 * q, 0), tail = max(4 * q + 4 - it_end[lo], 0);
                pin[g] = (0xFu << lead) & (0xFu >> tail);
            }
            // every load is issued, unconditionally (a lane without a quad reads quad 0, which
            // exists whenever the pass has a quad at all), before any is used: a load under a
            // branch would make the compiler wait for it before the next one
            uint4 pr[2 * QPL];
#pragma unroll
            for (int g = 0; g < QPL; ++g) {
                pr[2 * g] = a.pairs[2 * pq[g]];
                pr[2 * g + 1] = a.pairs[2 * pq[g] + 1];
            }
            // coins first; the live edges (bit 4g + h: edge h of quad g) are then visited
            // through one call site, so the hash probing is not inlined 4 * QPL times
            uint32_t live = 0u, tie = 0u;
#pragma unroll
            for (int g = 0; g < QPL; ++g) {
                if (g >= qpl) break;
                if (ps[g] < 0) continue;
                const uint64_t j = a.j0 + s_idx[ps[g]];
                uint64_t X, Y;
                philox2x64((uint32_t)pq[g], (uint32_t)j, (uint32_t)(j >> 32), TAG_EDGE, a.seed_lo, a.seed_hi, X, Y);
                const uint32_t hw[4] = {(uint32_t)X, (uint32_t)(X >> 32), (uint32_t)Y, (uint32_t)(Y >> 32)};
                const uint32_t th[4] = {pr[2 * g].y, pr[2 * g].w, pr[2 * g + 1].y, pr[2 * g + 1].w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    live |= (uint32_t)(hw[h] < th[h]) << (4 * g + h);
                    tie |= (uint32_t)(hw[h] == th[h]) << (4 * g + h);
                }
                live &= ~(0xFu << (4 * g)) | (pin[g] << (4 * g));
                tie &= ~(0xFu << (4 * g)) | (pin[g] << (4 * g));
            }
            static_assert(QPL <= 2, "the live-edge switch covers up to 2 quads per lane");
            while (tie) { // almost never taken
                const int c = __ffs(tie) - 1;
                tie &= tie - 1u;
                uint4 q;
                switch (c >> 1) {
                case 0: q = pr[0]; break;
                case 1: q = pr[1]; break;
                case 2: q = pr[QPL > 1 ? 2 : 0]; break;
                default: q = pr[QPL > 1 ? 3 : 0]; break;
                }
                const bool g1 = QPL > 1 && c >= 4;
                const int e = 4 * (g1 ? pq[QPL - 1] : pq[0]) + (c & 3);
                const uint64_t j = a.j0 + s_idx[g1 ? ps[QPL - 1] : ps[0]];
                // the coin's high half equals the threshold's
                const uint32_t hw = (c & 1) ? q.w : q.y;
                if (coin_live(SKIS_KARG(wbits)[e], coin_with_low_half(hw, (uint32_t)e, j, a.seed_lo, a.seed_hi)))
                    live |= 1u << c;
            }
            // the sweep's live edges into the queue (visited at once when a sweep alone holds
            // more than the queue can)
            const uint32_t nl = (uint32_t)__popc(live);
            const uint32_t incl = wave_incl_scan(nl);
            const uint32_t tot = lane_value(incl, 63);
            const bool direct = tot > (uint32_t)VQ_CAP;
            if (tot && (direct || vq_n + tot > (uint32_t)VQ_CAP)) vq_flush();
            uint32_t pos = vq_n + incl - nl;
            while (live) {
                const int c = __ffs(live) - 1;
                live &= live - 1u;
                uint4 q;
                int sl;
                // a switch, not an index into pr[]: the arrays stay in registers
                switch (c >> 1) {
                case 0: q = pr[0]; sl = ps[0]; break;
                case 1: q = pr[1]; sl = ps[0]; break;
                case 2: q = pr[QPL > 1 ? 2 : 0]; sl = ps[QPL > 1 ? 1 : 0]; break;
                default: q = pr[QPL > 1 ? 3 : 0]; sl = ps[QPL > 1 ? 1 : 0]; break;
                }
                const int32_t u = (int32_t)((c & 1) ? q.z : q.x);
                if (direct) {
                    visit(sl, u);
                } else {
                    vq_node[pos] = u;
                    vq_slot[pos] = (uint8_t)sl;
                    ++pos;
                }
            }
            if (!direct) vq_n += tot;
        }
        vq_flush();
        bsync();
        if (!s_alive) break;
    }
    if (SKIS_KARG(tier_stats)) {
        if (tid < 64) {
            st_fin = wave_sum(st_fin);
            st_ent = wave_sum(st_ent);
            st_prb = wave_sum(st_prb);
            if (tid == 0 && st_fin) {
                atomicAdd(SKIS_KARG(tier_stats) + 0, st_fin);
                atomicAdd(SKIS_KARG(tier_stats) + 1, st_ent);
                atomicAdd(SKIS_KARG(tier_stats) + 2, st_prb);
            }
        }
        st_swp = wave_sum(st_swp);
        st_itm = wave_sum(st_itm);
        if ((tid & 63) == 0 && st_itm) {
            atomicAdd(SKIS_KARG(tier_stats) + 3, st_swp);
            atomicAdd(SKIS_KARG(tier_stats) + 4, st_itm);
        }
    }
}

// ---------------------------------------------------------------------------------------
#undef SKIS_KARG

// Compaction: sort each sample and write it at sample_ptr[i].
// ---------------------------------------------------------------------------------------
// Size classes for the segmented sorts: class c holds sizes up to 8 << c; classes 0 .. 3 use
// segments of 8, 16, 32 or 64 lanes with one node per lane, classes 4 .. 7 a whole wave with
// 2, 4, 8 or 16 nodes per lane (up to SMALL_SORT).
constexpr int GATHER_CLASSES = 8;

__device__ __forceinline__ int size_class(uint32_t sz)
{
    return sz <= 8 ? 0 : sz <= 16 ? 1 : sz <= 32 ? 2 : sz <= 64 ? 3 : sz <= 128 ? 4 : sz <= 256 ? 5 : sz <= 512 ? 6 : 7;
}

// counts[c] = samples of class c (samples above SMALL_SORT are listed by the sampler)
__global__ __launch_bounds__(256) void k_class_count(uint64_t T, const uint32_t *__restrict__ size,
                                                     unsigned long long *__restrict__ counts)
{
    __shared__ unsigned long long bc[GATHER_CLASSES];
    if (threadIdx.x < GATHER_CLASSES) bc[threadIdx.x] = 0ull;
    __syncthreads();
    unsigned long long c[GATHER_CLASSES] = {};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t sz = size[i];
        if (sz <= SMALL_SORT) c[size_class(sz)] += 1;
    }
#pragma unroll
    for (int k = 0; k < GATHER_CLASSES; ++k) {
        const unsigned long long t = wave_sum(c[k]);
        if ((threadIdx.x & 63) == 0 && t) atomicAdd(&bc[k], t);
    }
    __syncthreads();
    // one global atomic per class and workgroup: same-address atomics serialise in L2
    if (threadIdx.x < GATHER_CLASSES && bc[threadIdx.x]) atomicAdd(&counts[threadIdx.x], bc[threadIdx.x]);
}

// lists[base(c) + ...] = the samples of class c, base(c) = counts of the classes before c.
// Each workgroup takes CLASS_CHUNK consecutive samples, counts their classes in LDS,
// reserves its range of every class list with one atomic per class, then places them.
constexpr int CLASS_CHUNK = 4096;

__global__ __launch_bounds__(256) void k_class_fill(uint64_t T, const uint32_t *__restrict__ size,
                                                    const unsigned long long *__restrict__ counts,
                                                    unsigned long long *__restrict__ cursor,
                                                    uint32_t *__restrict__ lists)
{
    __shared__ uint32_t lc[GATHER_CLASSES];
    __shared__ unsigned long long lb[GATHER_CLASSES];
    unsigned long long base[GATHER_CLASSES];
    unsigned long long acc = 0;
#pragma unroll
    for (int k = 0; k < GATHER_CLASSES; ++k) {
        base[k] = acc;
        acc += counts[k];
    }
    for (uint64_t c0 = (uint64_t)blockIdx.x * CLASS_CHUNK; c0 < T; c0 += (uint64_t)gridDim.x * CLASS_CHUNK) {
        const uint64_t c1 = min(c0 + CLASS_CHUNK, T);
        if (threadIdx.x < GATHER_CLASSES) lc[threadIdx.x] = 0u;
        __syncthreads();
        for (uint64_t i = c0 + threadIdx.x; i < c1; i += 256) {
            const uint32_t sz = size[i];
            if (sz <= SMALL_SORT) atomicAdd(&lc[size_class(sz)], 1u);
        }
        __syncthreads();
        if (threadIdx.x < GATHER_CLASSES) {
            const uint32_t x = lc[threadIdx.x];
            lb[threadIdx.x] = x ? atomicAdd(&cursor[threadIdx.x], (unsigned long long)x) : 0ull;
            lc[threadIdx.x] = 0u;
        }
        __syncthreads();
        for (uint64_t i = c0 + threadIdx.x; i < c1; i += 256) {
            const uint32_t sz = size[i];
            if (sz <= SMALL_SORT) {
                const int c = size_class(sz);
                lists[base[c] + lb[c] + atomicAdd(&lc[c], 1u)] = (uint32_t)i;
            }
        }
        __syncthreads();
    }
}

// v of lane (this lane ^ ld) for ld < 64: lane distances 1 and 2 by a DPP quad permutation (a
// plain VALU move), the others through the LDS crossbar.  In the unrolled networks below ld is
// a constant, so the choice costs nothing; distances 1 and 2 are about half of their shuffles.
__device__ __forceinline__ int32_t shfl_xor_lanes(int32_t v, int ld)
{
    if (ld == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false); // quad_perm [1,0,3,2]
    if (ld == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false); // quad_perm [2,3,0,1]
    return __shfl_xor(v, ld, 64);
}

// Bitonic network over the W * R values of a segment of W lanes, element e = t * R + r in v[r]
// of lane t: exchanges at distance d < R stay in the lane, the others are shuffles at lane
// distance d / R within the segment.  Every lane of the wave runs it.
template <int W, int R>
__device__ __forceinline__ void bitonic_regs(int32_t (&v)[R], int t)
{
    constexpr int P = W * R;
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (int d = k >> 1; d > 0; d >>= 1) {
            if (d < R) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r & d) continue;
                    const bool asc = ((t * R + r) & k) == 0;
                    const int32_t x = v[r], y = v[r | d];
                    v[r] = asc ? min(x, y) : max(x, y);
                    v[r | d] = asc ? max(x, y) : min(x, y);
                }
            } else {
                const int ld = d / R;
                const bool low = (t & ld) == 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool asc = ((t * R + r) & k) == 0;
                    // (32 values a lane: the DPP form makes the network too large to unroll)
                    const int32_t y = R >= 32 ? __shfl_xor(v[r], ld, 64) : shfl_xor_lanes(v[r], ld);
                    v[r] = (low == asc) ? min(v[r], y) : max(v[r], y);
                }
            }
        }
    }
}

// Segments of W lanes each sort one sample of up to W * R nodes in registers (64 / W samples
// per wave and step).  Node slot r * W + t of the sample is loaded by lane t of the segment
// into v[r] (coalesced; padding INT32_MAX), then a bitonic network sorts the W * R values
// with element e = t * R + r living in v[r] of lane t: exchanges at distance d < R stay
// in the lane, the others are shuffles at lane distance d / R within the segment.  The
// next step's list entry and sample bounds are loaded before the current sort.
template <int W, int R>
__global__ __launch_bounds__(64) void k_gather_sort(int cls, const unsigned long long *__restrict__ counts,
                                                    const uint32_t *__restrict__ lists,
                                                    const uint32_t *__restrict__ size,
                                                    const unsigned long long *__restrict__ off,
                                                    const int64_t *__restrict__ sptr,
                                                    const int32_t *__restrict__ staging, int32_t *__restrict__ nodes,
                                                    int32_t *__restrict__ owner)
{
    constexpr int G = 64 / W;
    const int lane = threadIdx.x, seg = lane / W, t = lane % W;
    unsigned long long base = 0;
    for (int k = 0; k < cls; ++k) base += counts[k];
    const unsigned long long cnt = counts[cls];
    const unsigned long long stride = (unsigned long long)gridDim.x * G;
    // a two-stage pipeline over this segment's samples g0 + seg, g0 + stride + seg, ...: the
    // list entry two samples ahead and the size, offset and position one sample ahead are
    // loaded while the current one is sorted.  Loads are unconditional (an index past the
    // class reads its last entry); a sample past the class has size 0 and writes nothing.
    auto entry = [&](unsigned long long g) -> uint32_t { return lists[base + (g < cnt ? g : cnt - 1)]; };
    unsigned long long g0 = (unsigned long long)blockIdx.x * G;
    if (g0 >= cnt) return;
    uint32_t id = entry(g0 + seg);
    const uint32_t sz0 = size[id];
    uint32_t sz = g0 + seg < cnt ? sz0 : 0u;
    unsigned long long o = off[id];
    int64_t dp = sptr[id];
    uint32_t id1 = entry(g0 + stride + seg);
    for (; g0 < cnt; g0 += stride) {
        const uint32_t id2 = entry(g0 + 2 * stride + seg);
        const uint32_t sz1 = size[id1];
        const uint32_t nsz = g0 + stride + seg < cnt ? sz1 : 0u;
        const unsigned long long no = off[id1];
        const int64_t ndp = sptr[id1];
        int32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int x = r * W + t;
            v[r] = staging[o + (x < (int)sz ? x : 0)];
            if (x >= (int)sz) v[r] = INT32_MAX;
        }
        bitonic_regs<W, R>(v, t);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = t * R + r;
            if (e < (int)sz) {
                nodes[dp + e] = v[r];
                if (owner) owner[dp + e] = (int32_t)id;
            }
        }
        sz = nsz;
        id = id1;
        o = no;
        dp = ndp;
        id1 = id2;
    }
}

// Listed samples of (32 R, 64 R] nodes, one per wave, sorted in registers by the network above
// (R nodes a lane); the next sample's list entry and bounds are loaded before the sort.
template <int R>
__global__ __launch_bounds__(64) void k_gather_medium_regs(uint64_t count, const uint32_t *__restrict__ list,
                                                           const uint32_t *__restrict__ size,
                                                           const unsigned long long *__restrict__ off,
                                                           const int64_t *__restrict__ sptr,
                                                           const int32_t *__restrict__ staging,
                                                           int32_t *__restrict__ nodes, int32_t *__restrict__ owner)
{
    constexpr int LO = 32 * R, HI = 64 * R;
    const int t = threadIdx.x;
    uint64_t k = blockIdx.x;
    if (k >= count) return;
    uint32_t id = list[k];
    uint32_t sz = size[id];
    for (; k < count; k += gridDim.x) {
        const uint64_t kn = k + gridDim.x < count ? k + gridDim.x : k;
        const uint32_t idn = list[kn];
        const uint32_t szn = size[idn];
        if (sz > (uint32_t)LO && sz <= (uint32_t)HI) {
            const unsigned long long o = off[id];
            const int64_t dp = sptr[id];
            int32_t v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int x = r * 64 + t;
                v[r] = x < (int)sz ? staging[o + x] : INT32_MAX;
            }
            bitonic_regs<64, R>(v, t);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = t * R + r;
                if (e < (int)sz) {
                    nodes[dp + e] = v[r];
                    if (owner) owner[dp + e] = (int32_t)id;
                }
            }
        }
        id = idn;
        sz = szn;
    }
}

constexpr int MEDIUM_REGS_MAX = 2048; // sizes up to this are sorted in registers by k_gather_medium_regs<32>
// (64 values a lane spill to scratch: the network is too large to unroll)

// Samples of MEDIUM_REGS_MAX + 1 .. SORT_LDS_MAX nodes, one at a time per workgroup of NT
// threads, in registers: element e = t * R + r of the padded sample (P = NT R values) lives in
// v[r] of thread t.  Bitonic stages at distance d < R stay in the thread, those with d < 64 R
// are shuffles within the wave, and only the d >= 64 R stages (three per sample at 4096
// values, six at 8192) exchange through LDS; the LDS network it replaces took a barrier at
// every one of its 78-91 stages.  R = 16 values a thread keeps the network fully unrolled (at
// 32 the compiler indexed the registers at run time); 256 threads take the samples up to 4096
// nodes, 512 the rest.  The load is coalesced (any assignment of the sample's nodes to
// elements sorts the same) and the sorted values go out coalesced through LDS, one pad word
// per R values keeping the strided writes free of bank conflicts.
constexpr int BLOCK_SORT_R = 16;
constexpr int BLOCK_SORT_BUF = SORT_LDS_MAX + SORT_LDS_MAX / BLOCK_SORT_R;
__device__ __forceinline__ int pad_idx(int e) { return e + e / BLOCK_SORT_R; }

template <int NT>
__global__ __launch_bounds__(NT) void k_gather_block(uint64_t count, const uint32_t *__restrict__ list,
                                                     const uint32_t *__restrict__ size,
                                                     const unsigned long long *__restrict__ off,
                                                     const int64_t *__restrict__ sptr,
                                                     const int32_t *__restrict__ staging,
                                                     int32_t *__restrict__ nodes, int32_t *__restrict__ owner)
{
    constexpr int R = BLOCK_SORT_R;
    constexpr int P = NT * R;
    constexpr int LO = NT == 256 ? MEDIUM_REGS_MAX : P / 2; // sizes in (LO, P] are this kernel's
    static_assert(P <= SORT_LDS_MAX && (NT == 256 || NT == 512), "one workgroup size per half of the range");
    __shared__ int32_t buf[BLOCK_SORT_BUF];
    const int t = threadIdx.x;
    for (uint64_t k = blockIdx.x; k < count; k += gridDim.x) {
        const uint32_t i = list[k];
        const int sz = (int)size[i];
        if (sz <= LO || sz > P) continue; // another kernel's sample
        const int32_t *src = staging + off[i];
        int32_t *dst = nodes + sptr[i];
        if (owner)
            for (int x = t; x < sz; x += NT) owner[sptr[i] + x] = (int32_t)i;
        int32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int x = r * NT + t;
            v[r] = x < sz ? src[x] : INT32_MAX;
        }
#pragma unroll
        for (int kk = 2; kk <= P; kk <<= 1) {
#pragma unroll
            for (int d = kk >> 1; d > 0; d >>= 1) {
                if (d < R) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (r & d) continue;
                        const bool asc = ((t * R + r) & kk) == 0;
                        const int32_t x = v[r], y = v[r | d];
                        v[r] = asc ? min(x, y) : max(x, y);
                        v[r | d] = asc ? max(x, y) : min(x, y);
                    }
                } else if (d < 64 * R) {
                    const int ld = d / R;
                    const bool low = (t & ld) == 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const bool asc = ((t * R + r) & kk) == 0;
                        // (at 512 threads the DPP form makes the network too large to unroll)
                        const int32_t y = NT == 512 ? __shfl_xor(v[r], ld, 64) : shfl_xor_lanes(v[r], ld);
                        v[r] = (low == asc) ? min(v[r], y) : max(v[r], y);
                    }
                } else { // partner in another wave: through LDS
                    const int ld = d / R;
                    const bool low = (t & ld) == 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[pad_idx(t * R + r)] = v[r];
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const bool asc = ((t * R + r) & kk) == 0;
                        const int32_t y = buf[pad_idx((t ^ ld) * R + r)];
                        v[r] = (low == asc) ? min(v[r], y) : max(v[r], y);
                    }
                    __syncthreads();
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pad_idx(t * R + r)] = v[r];
        __syncthreads();
        for (int x = t; x < sz; x += NT) dst[x] = buf[pad_idx(x)];
        __syncthreads();
    }
}

// Samples above SORT_LDS_MAX nodes, one at a time per workgroup: the sample's nodes set
// their bits in the workgroup's bitmap of n bits and in a summary of one bit per bitmap word;
// a walk over the summary, in node order, visits only the bitmap words that hold nodes,
// writes those nodes in ascending order and clears both levels (every sample leaves its
// bitmaps zero).  Work per sample: its nodes plus n / 1024 summary words.
constexpr int LARGE_BLOCK = 256;
constexpr uint64_t LARGE_BITMAP_BUDGET = 2ull << 30;

__global__ __launch_bounds__(LARGE_BLOCK) void k_gather_large(uint64_t count, const uint32_t *__restrict__ list,
                                                              const uint32_t *__restrict__ size,
                                                              const unsigned long long *__restrict__ off,
                                                              const int64_t *__restrict__ sptr,
                                                              const int32_t *__restrict__ staging,
                                                              int32_t *__restrict__ nodes, int32_t *__restrict__ owner,
                                                              uint32_t *__restrict__ bits, uint32_t *__restrict__ summ,
                                                              uint64_t words, uint64_t swords, int *err)
{
    __shared__ int32_t s_scan[LARGE_BLOCK / 64 + 1];
    uint32_t *B = bits + (size_t)blockIdx.x * words;
    uint32_t *Sm = summ + (size_t)blockIdx.x * swords;
    const int tid = threadIdx.x;
    for (uint64_t k = blockIdx.x; k < count; k += gridDim.x) {
        const uint32_t i = list[k];
        const int64_t sz = (int64_t)size[i];
        if (sz <= SORT_LDS_MAX) continue; // k_gather_block's
        const int32_t *src = staging + off[i];
        int32_t *dst = nodes + sptr[i];
        for (int64_t t = tid; t < sz; t += LARGE_BLOCK) {
            const uint32_t u = (uint32_t)src[t];
            if ((uint64_t)(u >> 5) >= words) { // bounds guard: report, never index
                atomicOr(err, 1);
                continue;
            }
            atomicOr(B + (u >> 5), 1u << (u & 31));
            atomicOr(Sm + (u >> 10), 1u << ((u >> 5) & 31));
            if (owner) owner[sptr[i] + t] = (int32_t)i;
        }
        __syncthreads();
        int64_t run = 0;
        for (uint64_t s0 = 0; s0 < swords; s0 += LARGE_BLOCK) {
            const uint64_t sw = s0 + tid;
            const uint32_t sm = sw < swords ? Sm[sw] : 0u;
            int c = 0;
            for (uint32_t x = sm; x; x &= x - 1u) c += __popc(B[sw * 32u + (uint64_t)(__ffs(x) - 1)]);
            int tot;
            const int ex = block_excl_scan<LARGE_BLOCK, int>(c, s_scan, &tot);
            int64_t pos = run + ex;
            for (uint32_t x = sm; x; x &= x - 1u) {
                const uint64_t wi = sw * 32u + (uint64_t)(__ffs(x) - 1);
                for (uint32_t y = B[wi]; y; y &= y - 1u) {
                    if (pos < sz) dst[pos] = (int32_t)(wi * 32u + (uint64_t)(__ffs(y) - 1));
                    ++pos;
                }
                B[wi] = 0u;
            }
            if (sm) Sm[sw] = 0u;
            run += tot;
        }
        if (tid == 0 && run != sz) atomicOr(err, 2); // a repeated node: the sample is broken
        __syncthreads();
    }
}

// Adds the sum of v over a 256-thread workgroup to *out with one global atomic.
__device__ __forceinline__ void block_add_to(unsigned long long v, unsigned long long *out)
{
    __shared__ unsigned long long part[4];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(out, t);
    }
}

__global__ __launch_bounds__(256) void k_count_value(uint64_t count, const uint32_t *__restrict__ x, uint32_t v,
                                                     unsigned long long *__restrict__ out)
{
    unsigned long long acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        acc += x[i] == v ? 1ull : 0ull;
    block_add_to(acc, out);
}

// *out += #{ k < count : x[list[k]] > v }
__global__ __launch_bounds__(256) void k_count_listed_above(uint64_t count, const uint32_t *__restrict__ list,
                                                            const uint32_t *__restrict__ x, uint32_t v,
                                                            unsigned long long *__restrict__ out)
{
    unsigned long long acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        acc += x[list[i]] > v ? 1ull : 0ull;
    block_add_to(acc, out);
}

__global__ __launch_bounds__(256) void k_roots_out(uint32_t count, const int4 *__restrict__ rec, int32_t *__restrict__ roots)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        roots[i] = rec[i].x;
}

__global__ __launch_bounds__(256) void k_sum_u64(uint64_t count, const unsigned long long *__restrict__ x,
                                                 unsigned long long *__restrict__ out)
{
    unsigned long long acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        acc += x[i];
    block_add_to(acc, out);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(uint64_t count, T *__restrict__ p, T v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------------------
// Chain control for the captured form: the graph [begin, roots, tier 0, tier 1, tier 2,
// end] is replayed once per chunk of sample ids, and everything that changes between
// replays lives in this record, so a replay needs nothing from the host.
// ---------------------------------------------------------------------------------------
struct ChainCtl {
    unsigned long long cursor;            // first sample id not yet handed to a chunk
    unsigned long long base, count;       // the current chunk: ids [base, base + count)
    unsigned long long next0, next1, next2, next3; // id counters of the four tiers
    unsigned long long nd0, nd1, nd2;     // samples handed on by tiers 0, 1, 2 in this chunk
    unsigned long long tot0, tot1, tot2;  // the same, summed over chunks
    unsigned long long replays;
};

__global__ __launch_bounds__(64) void k_chain_begin(ChainCtl *c, uint64_t T, uint64_t chunk)
{
    if (threadIdx.x != 0) return;
    const unsigned long long cur = c->cursor;
    const unsigned long long cnt = cur < T ? (T - cur < chunk ? T - cur : chunk) : 0ull;
    c->base = cur;
    c->count = cnt;
    c->cursor = cur + cnt;
    c->next0 = 0;
    c->next1 = 0;
    c->next2 = 0;
    c->next3 = 0;
    c->nd0 = 0;
    c->nd1 = 0;
    c->nd2 = 0;
}

__global__ __launch_bounds__(64) void k_chain_end(ChainCtl *c)
{
    if (threadIdx.x != 0) return;
    c->tot0 += c->nd0;
    c->tot1 += c->nd1;
    c->tot2 += c->nd2;
    c->replays += 1;
}

// out[0] = the smallest t in [1, T] with sptr[t] >= budget (T if there is none); one thread.
__global__ void k_first_reaching(const int64_t *__restrict__ sptr, uint64_t T, int64_t budget,
                                 unsigned long long *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t lo = 1, hi = T;
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (sptr[mid] >= budget) hi = mid; else lo = mid + 1;
    }
    out[0] = lo;
}

// ---------------------------------------------------------------------------------------
// Host orchestration.
// ---------------------------------------------------------------------------------------
static unsigned grid_cap(uint64_t items, int block, int per_cu = 16)
{
    uint64_t g = (items + block - 1) / block;
    const uint64_t cap = (uint64_t)device_cu_count() * per_cu;
    if (g > cap) g = cap;
    return (unsigned)(g > 0 ? g : 1);
}

struct Counters {
    unsigned long long next;
    unsigned long long stage_used;
    unsigned long long n_deferred;
    unsigned long long n_medium;
    int overflow;
    int pad;
    unsigned long long tier[4][5]; // per tier: samples finished, their entries, their edges probed,
                                   // edges and nodes the launch expanded
};

typedef void (*SampleKernel)(SampleArgs);

struct Variant {
    uint32_t threads, slots, visited, qpl;
    SampleKernel fn;
};

// LDS-tier variants: (threads per workgroup, slots per workgroup, LDS visited capacity).
// With 64 threads a workgroup is one wave that owns its slots and LDS and never waits for
// another wave; with 256 threads four waves share the slots and meet at barriers.
static const Variant kTier0[] = {
    {64, 4, 192, 2, k_sample<64, 4, 192, 256, 128, 2, 0>},
    {64, 4, 192, 1, k_sample<64, 4, 192, 256, 64, 1, 0>},
    {64, 4, 256, 2, k_sample<64, 4, 256, 320, 128, 2, 0>},
    {64, 4, 256, 1, k_sample<64, 4, 256, 320, 64, 1, 0>},
    {64, 2, 256, 1, k_sample<64, 2, 256, 320, 64, 1, 0>},
    {64, 3, 256, 1, k_sample<64, 3, 256, 320, 64, 1, 0>},
    {64, 2, 384, 1, k_sample<64, 2, 384, 512, 64, 1, 0>},
    {64, 6, 256, 2, k_sample<64, 6, 256, 320, 192, 2, 0>},
    {64, 8, 128, 2, k_sample<64, 8, 128, 172, 256, 2, 0>},
    {64, 8, 192, 2, k_sample<64, 8, 192, 256, 256, 2, 0>},
    {64, 8, 192, 1, k_sample<64, 8, 192, 256, 256, 1, 0>},
    {64, 8, 256, 2, k_sample<64, 8, 256, 344, 256, 2, 0>},
    {64, 12, 192, 2, k_sample<64, 12, 192, 256, 384, 2, 0>},
    {64, 16, 128, 2, k_sample<64, 16, 128, 172, 512, 2, 0>},
    {64, 16, 64, 2, k_sample<64, 16, 64, 88, 512, 2, 0>},
    {256, 16, 128, 2, k_sample<256, 16, 128, 172, 1024, 2, 0>},
    {256, 32, 128, 2, k_sample<256, 32, 128, 172, 1024, 2, 0>},
    {256, 16, 256, 2, k_sample<256, 16, 256, 344, 1024, 2, 0>},
};
// second tier: samples that outgrew the first, slots of 1024 nodes in LDS
// (64 items a pass and two quads a lane: 341 ms at 1.4B edges against 350 with one quad,
// 345 with 128 items, 399 and 469 with 128 and 256 items and one quad)
static const Variant kTierMidV[] = {
    {64, 1, 1024, 2, k_sample<64, 1, 1024, 1368, 64, 2, 1>},
    {256, 8, 1024, 2, k_sample<256, 8, 1024, 1368, 1024, 2, 1>},
};
// Third tier: one sample per one-wave workgroup, its visited set a hash of TIERH_HCAP slots
// and its node list TIERH_RCAP entries in HBM, so that every compute unit holds as many
// samples as waves fit (the samples that outgrow 1024 nodes number about 1 % on the 1.4B-edge
// workload, and each takes many passes).  The hashes of the samples in flight (6,144 at six
// waves a SIMD) are the tier's working set: with five waves, at 16384 slots (335 MB) the tier
// took 67 ms at 1.4B edges, at 8192 62 ms, and at 4096 slots the samples sent on to the
// bitmap tier cost more than the hash saved (71 ms); the samples that leave it mostly meet a
// hub row rather than outgrow it.
constexpr int TIERH_RCAP = 6144;
constexpr int TIERH_HCAP = 8192;
// in-degree above which the hash tier hands a sample on: a hub row is swept faster by the
// bitmap tier's sixteen waves than by one
constexpr uint32_t TIERH_BIG_ROW = 65536;
static SampleKernel const kTierHash = k_sample<64, 1, TIERH_RCAP, TIERH_HCAP, 64, 1, 2>;
// Fourth tier: one sample per workgroup with a bitmap of n bits and a node list of n entries;
// the few samples that outgrow the hash tier or meet an in-degree above 2^20 take sixteen waves
// each; the HBM buffers of all slots are kept within TIERG_BUDGET bytes.
constexpr int TIERG_SLOTS = 1;
constexpr int TIERG_BLOCK = 1024;
constexpr int TIERG_PER_CU = TIERG_BLOCK >= 512 ? 1 : 512 / TIERG_BLOCK;
constexpr uint64_t TIERG_BUDGET = 32ull << 30;
// captured form: sample ids per graph replay unless the caller names another count (every chunk
// waits for its own largest samples, so fewer chunks finish sooner)
constexpr uint64_t CHAIN_CHUNK_DEFAULT = 1ull << 24;
static SampleKernel const kTierGlobal = k_sample<TIERG_BLOCK, TIERG_SLOTS, 1, 1, 8 * TIERG_BLOCK, 2, 3>;

static const Variant &pick_variant(const Variant *vs, size_t nv, uint32_t threads, uint32_t slots, uint32_t visited,
                                   uint32_t qpl)
{
    for (size_t i = 0; i < nv; ++i)
        if (vs[i].threads == threads && vs[i].slots == slots && vs[i].visited == visited && vs[i].qpl == qpl)
            return vs[i];
    throw Error{SKIS_EINVAL,
                "unsupported (threads_per_block, slots_per_block, visited_threshold, quads_per_lane) combination"};
}

static int occupancy_blocks(SampleKernel fn, int block)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(fn), block, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

// Entries per sample of the last build on a graph of the same (n, m), per process: sizes the
// next build's staging, so that a graph whose samples outgrow the default guess (48 entries
// a sample) pays the staging-overflow retry (a second sampling pass) only once.
static std::mutex g_hint_mu;
static std::map<std::pair<int32_t, int64_t>, double> g_entries_hint;

static double entries_per_sample_hint(int32_t n, int64_t m)
{
    std::lock_guard<std::mutex> lk(g_hint_mu);
    const auto it = g_entries_hint.find({n, m});
    return it == g_entries_hint.end() ? 48.0 : std::max(48.0, it->second * 1.05);
}

static void set_entries_per_sample_hint(int32_t n, int64_t m, double v)
{
    std::lock_guard<std::mutex> lk(g_hint_mu);
    g_entries_hint[{n, m}] = v;
}

void sample_and_compact(Arena &arena, const Prep &prep, int32_t n, int64_t m, uint64_t T, uint64_t seed,
                        const SampleConfig &cfg, Sketch &sk, hipStream_t s)
{
    (void)m;
    if (T >= (1ull << 31)) throw Error{SKIS_EINVAL, "num_samples must be below 2^31"};
    const uint32_t count = (uint32_t)T;
    const uint32_t seed_lo = (uint32_t)seed, seed_hi = (uint32_t)(seed >> 32);
    constexpr int NEV = 12;
    hipEvent_t ev[NEV];
    for (auto &e : ev) SKIS_HIP_TRY(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int i = 0; i < NEV; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    bool ran_mid = false, ran_hash = false, ran_global = false;

    // every device buffer a kernel below dereferences must exist (checked on the host)
    auto need = [](const void *p, const char *what) {
        if (!p) throw Error{SKIS_EHIP, std::string("internal error: null device buffer ") + what};
    };
    const bool lt = cfg.model == MODEL_LT;
    if (lt && (cfg.ris || cfg.form != 0))
        throw Error{SKIS_EINVAL, "the linear threshold sampler has the persistent form only and no RIS mode"};
    if (lt != (prep.model == MODEL_LT)) throw Error{SKIS_EHIP, "internal error: sampler and preprocessing models differ"};
    if (!cfg.ris) need(prep.alias.ptr, "alias");
    need(prep.row_ptr.ptr, "row_ptr");
    need(prep.q.ptr, "q");
    need(prep.P.ptr, "P");
    need(prep.edges.ptr, "edges");
    need(prep.wbits.ptr, "w bits");

    DevBuf<int4> rec;
    DevBuf<int32_t> u1;
    rec.alloc(arena, count);
    u1.alloc(arena, count);
    DevBuf<int> rerr;
    rerr.alloc(arena, 1);
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (uint64_t)1, rerr.ptr, 0);
    SKIS_HIP_TRY(hipEventRecord(ev[0], s));
    if (cfg.form != 2 && !lt) { // the captured form draws the roots inside its chain, chunk by chunk
        hipLaunchKernelGGL(k_roots, dim3(grid_cap(count, 256, 64)), dim3(256), 0, s, (uint64_t)cfg.first_id, count,
                           (const unsigned long long *)nullptr, seed_lo, seed_hi, n, prep.C, prep.alias.ptr,
                           prep.row_ptr.ptr, prep.q.ptr, prep.P.ptr, prep.edges.ptr, prep.wbits.ptr, rec.ptr, u1.ptr, rerr.ptr,
                           (int)cfg.ris);
        SKIS_HIP_TRY(hipGetLastError());
    }
    SKIS_HIP_TRY(hipEventRecord(ev[1], s));

    DevBuf<uint32_t> out_size, deferred, medium;
    DevBuf<unsigned long long> out_off;
    out_size.alloc(arena, count);
    out_off.alloc(arena, count);
    sk.probed.alloc(arena, count);
    deferred.alloc(arena, count);
    medium.alloc(arena, count);
    DevBuf<Counters> ctr;
    ctr.alloc(arena, 1);

    DevBuf<int32_t> staging;
    Counters hc{};
    const Variant &v0 =
        pick_variant(kTier0, sizeof(kTier0) / sizeof(kTier0[0]), cfg.threads, cfg.slots, cfg.visited, cfg.qpl);
    const Variant &vm = kTierMidV[cfg.threads == 64 ? 0 : 1];
    // handover from tier 0 to tier 1 for the first ho_cap samples a launch hands on (the rest
    // start over in tier 1): an eighth of the ids one tier-0 launch takes (784 B a record at the
    // default shape; 8.2 % of the samples outgrow tier 0 on the 1.4B-edge WC graph)
    const uint64_t per_launch0 =
        cfg.form == 2 ? std::min<uint64_t>(count, cfg.chunk ? cfg.chunk : CHAIN_CHUNK_DEFAULT) : count;
    const bool tiered = !lt && cfg.form != 1;
    const uint64_t ho_cap = tiered ? std::min<uint64_t>(per_launch0, std::max<uint64_t>(1024, per_launch0 / 8)) : 0;
    const int ho_stride = (int)v0.visited;
    if (v0.visited > vm.visited) throw Error{SKIS_EHIP, "internal error: tier 1 smaller than tier 0"};
    DevBuf<Handover> ho_state;
    DevBuf<int32_t> ho_nodes;
    ho_state.alloc(arena, ho_cap);
    ho_nodes.alloc(arena, ho_cap * (uint64_t)ho_stride);
    const int cus = device_cu_count();
    const int nb0 = occupancy_blocks(v0.fn, (int)v0.threads) * cus;
    const int nbm = occupancy_blocks(vm.fn, (int)vm.threads) * cus;
    // Staging: each LDS-tier workgroup reserves 8 * slots * visited entries at a time and
    // wastes less than one finished pass (slots * visited) per reservation plus its last
    // open chunk, so sum|R| * 8/7 + 2 chunks per workgroup bounds what a launch reserves.
    const uint64_t ch0 = 8ull * v0.slots * v0.visited, chm = 8ull * vm.slots * vm.visited;
    const uint64_t slack = (uint64_t)std::min<uint64_t>(nb0, count) * 2 * ch0 +
                           (uint64_t)std::min<uint64_t>(nbm, count) * 2 * chm;
    auto staging_bound = [&](uint64_t entries, uint64_t launches) {
        return entries + entries / 7 + 1 + launches * slack + (1ull << 20);
    };
    const double per_sample = entries_per_sample_hint(n, m);
    uint64_t cap = cfg.staging_entries ? cfg.staging_entries : staging_bound((uint64_t)((double)count * per_sample), 1);
    const uint64_t words = ((uint64_t)n + 31) / 32;
    // bitmap tier: every slot holds a bitmap of n bits and a node list of n entries
    const uint64_t slot_bytes = (uint64_t)n * 4ull + words * 4ull;
    uint64_t nbg_mem = TIERG_BUDGET / (slot_bytes * TIERG_SLOTS);
    if (nbg_mem < 1) nbg_mem = 1;
    const int nbg = (int)std::min<uint64_t>((uint64_t)TIERG_PER_CU * cus, nbg_mem);
    // hash tier: as many one-wave workgroups as are resident at once, each with its own hash
    // and list
    const int nbh = occupancy_blocks(kTierHash, 64) * cus;
    DevBuf<uint32_t> deferred2;
    deferred2.alloc(arena, count);
    const int ho2_stride = (int)vm.visited; // tier 1 -> hash tier records
    const int ho3_stride = TIERH_RCAP;      // hash tier -> bitmap tier records
    constexpr uint64_t HO3_MAX = 8192;      // records of the samples that outgrow the hash tier (192 MiB)

    auto read_counters = [&]() {
        SKIS_HIP_TRY(hipMemcpyAsync(&hc, ctr.ptr, sizeof(hc), hipMemcpyDeviceToHost, s));
        SKIS_HIP_TRY(hipStreamSynchronize(s));
    };
    auto reset_ids = [&]() {
        hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)1, &ctr.ptr->next, 0ull);
        hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)1, &ctr.ptr->n_deferred, 0ull);
    };
    // the hash tier's hashes start empty (-1) and every launch leaves them so
    DevBuf<int32_t> ghash;
    DevBuf<uint2> glist2;
    auto alloc_hash_tier = [&]() {
        ghash.alloc(arena, (uint64_t)nbh * TIERH_HCAP);
        glist2.alloc(arena, (uint64_t)nbh * TIERH_RCAP);
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_cap((uint64_t)nbh * TIERH_HCAP, 256)), dim3(256), 0, s,
                           (uint64_t)nbh * TIERH_HCAP, ghash.ptr, -1);
        SKIS_HIP_TRY(hipGetLastError());
        need(ghash.ptr, "hash tier hashes");
        need(glist2.ptr, "hash tier lists");
    };

    // Captured form: the whole chain for one chunk of ids -- chunk bounds, roots, the four
    // tiers, each reading its work count from device memory -- is captured once into a HIP
    // graph on a private stream and replayed ceil(T / chunk) times on s with no host
    // round trip in between.  The HBM tiers cannot be skipped on the host's word here, so
    // their buffers are always allocated (each slot clears what its sample used when the
    // sample leaves, so they stay clear across replays).
    auto sample_chain_graph = [&]() {
        // 2^24 ids by default: every chunk waits for its own largest samples, so fewer chunks
        // finish sooner (2^22 took 44 / 115 ms on the 1M-node WC / 4M-node TRI graphs, 2^24 37 / 67)
        const uint64_t chunk = std::min<uint64_t>(count, cfg.chunk ? cfg.chunk : CHAIN_CHUNK_DEFAULT);
        const uint64_t replays = (count + chunk - 1) / chunk;
        if (!cfg.staging_entries) cap = staging_bound((uint64_t)((double)count * per_sample), replays);
        DevBuf<ChainCtl> gc;
        gc.alloc(arena, 1);
        const uint64_t nbg_g = (uint64_t)nbg;
        const uint64_t gslots = nbg_g * TIERG_SLOTS;
        DevBuf<uint32_t> gbits;
        DevBuf<int32_t> glist;
        gbits.alloc(arena, gslots * words);
        glist.alloc(arena, gslots * (uint64_t)n);
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_cap(gslots * words, 256)), dim3(256), 0, s, gslots * words,
                           gbits.ptr, 0u);
        alloc_hash_tier();
        need(gc.ptr, "chain control");
        need(gbits.ptr, "gbits");
        need(glist.ptr, "glist");
        // handover from tier 1 to the hash tier for the first ho2_cap samples tier 1 hands on
        // in a chunk, and from the hash tier to the bitmap tier for the first ho3_cap; each
        // tier takes its list in a scrambled order, and position p resumes from record p
        const uint64_t ho2_cap = std::min<uint64_t>(chunk, std::max<uint64_t>(1024, chunk / 64));
        const uint64_t ho3_cap = std::min<uint64_t>(chunk, HO3_MAX);
        DevBuf<Handover> ho2_state, ho3_state;
        DevBuf<int32_t> ho2_nodes, ho3_nodes;
        ho2_state.alloc(arena, ho2_cap);
        ho2_nodes.alloc(arena, ho2_cap * (uint64_t)ho2_stride);
        ho3_state.alloc(arena, ho3_cap);
        ho3_nodes.alloc(arena, ho3_cap * (uint64_t)ho3_stride);
        need(ho2_state.ptr, "handover");
        need(ho2_nodes.ptr, "handover nodes");
        need(ho3_state.ptr, "handover");
        need(ho3_nodes.ptr, "handover nodes");
        struct GraphGuard {
            hipStream_t cs = nullptr;
            hipGraph_t g = nullptr;
            hipGraphExec_t x = nullptr;
            bool capturing = false;
            ~GraphGuard()
            {
                if (capturing) {
                    hipGraph_t tmp = nullptr;
                    (void)hipStreamEndCapture(cs, &tmp);
                    if (tmp) (void)hipGraphDestroy(tmp);
                }
                if (x) (void)hipGraphExecDestroy(x);
                if (g) (void)hipGraphDestroy(g);
                if (cs) (void)hipStreamDestroy(cs);
            }
        } gg;
        SKIS_HIP_TRY(hipStreamCreateWithFlags(&gg.cs, hipStreamNonBlocking));
        for (int attempt = 0; attempt < 2; ++attempt) {
            staging.alloc(arena, cap);
            hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, s, (uint64_t)sizeof(Counters),
                               reinterpret_cast<unsigned char *>(ctr.ptr), (unsigned char)0);
            hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, s, (uint64_t)sizeof(ChainCtl),
                               reinterpret_cast<unsigned char *>(gc.ptr), (unsigned char)0);
            SKIS_HIP_TRY(hipGetLastError());
            SampleArgs A{};
            A.n = n;
            A.row_ptr = prep.row_ptr.ptr;
            A.pairs = reinterpret_cast<const uint4 *>(prep.edges.ptr);
            A.nquads = (int64_t)(prep.edges.count / 4);
            A.wbits = prep.wbits.ptr;
            A.rec = rec.ptr;
            A.u1 = u1.ptr;
            A.j0 = cfg.first_id;
            A.seed_lo = seed_lo;
            A.seed_hi = seed_hi;
            A.staging = staging.ptr;
            A.stage_cap = cap;
            A.stage_used = &ctr.ptr->stage_used;
            A.out_size = out_size.ptr;
            A.out_off = out_off.ptr;
            A.out_probed = reinterpret_cast<unsigned long long *>(sk.probed.ptr);
            A.medium = medium.ptr;
            A.n_medium = &ctr.ptr->n_medium;
            A.overflow = &ctr.ptr->overflow;
            A.words = words;
            need(A.staging, "staging");
            SampleArgs A0 = A, A1 = A, A2 = A, A3 = A;
            A0.tier_stats = ctr.ptr->tier[0];
            A1.tier_stats = ctr.ptr->tier[1];
            A2.tier_stats = ctr.ptr->tier[2];
            A3.tier_stats = ctr.ptr->tier[3];
            A0.next = &gc.ptr->next0;
            A0.id_list = nullptr;
            A0.id_count_dev = &gc.ptr->count;
            A0.id_base_dev = &gc.ptr->base;
            A0.big_row = cfg.big_row;
            A0.deferred = deferred.ptr;
            A0.n_deferred = &gc.ptr->nd0;
            A1.next = &gc.ptr->next1;
            A1.id_list = deferred.ptr;
            A1.id_count_dev = &gc.ptr->nd0;
            A1.big_row = std::max<uint32_t>(cfg.big_row, 1u << 20);
            A1.deferred = deferred2.ptr;
            A1.n_deferred = &gc.ptr->nd1;
            A2.next = &gc.ptr->next2;
            A2.id_list = deferred2.ptr;
            A2.id_count_dev = &gc.ptr->nd1;
            A2.id_perm = 1; // the eager form shuffles on the host; here the order is scrambled in place
            A2.big_row = std::max<uint32_t>(cfg.big_row, TIERH_BIG_ROW);
            A2.deferred = deferred.ptr; // tier 1 has read tier 0's list by now
            A2.n_deferred = &gc.ptr->nd2;
            A2.ghash = ghash.ptr;
            A2.glist2 = glist2.ptr;
            A3.next = &gc.ptr->next3;
            A3.id_list = deferred.ptr;
            A3.id_count_dev = &gc.ptr->nd2;
            A3.id_perm = 1;
            A3.deferred = deferred2.ptr;          // unused: the bitmap tier finishes every sample
            A3.n_deferred = &ctr.ptr->n_deferred; // unused for the same reason
            A3.gbits = gbits.ptr;
            A3.glist = glist.ptr;
            A0.ho_state_out = ho_state.ptr; // tiers 0-2 hand over, tiers 1-3 resume
            A0.ho_nodes_out = ho_nodes.ptr;
            A0.ho_cap_out = ho_cap;
            A1.ho_state_in = ho_state.ptr;
            A1.ho_nodes_in = ho_nodes.ptr;
            A1.ho_cap_in = ho_cap;
            A0.ho_stride_out = A1.ho_stride_in = ho_stride;
            A1.ho_state_out = ho2_state.ptr;
            A1.ho_nodes_out = ho2_nodes.ptr;
            A1.ho_cap_out = ho2_cap;
            A2.ho_state_in = ho2_state.ptr;
            A2.ho_nodes_in = ho2_nodes.ptr;
            A2.ho_slot_in = nullptr;
            A2.ho_cap_in = ho2_cap;
            A1.ho_stride_out = A2.ho_stride_in = ho2_stride;
            A2.ho_state_out = ho3_state.ptr;
            A2.ho_nodes_out = ho3_nodes.ptr;
            A2.ho_cap_out = ho3_cap;
            A3.ho_state_in = ho3_state.ptr;
            A3.ho_nodes_in = ho3_nodes.ptr;
            A3.ho_slot_in = nullptr;
            A3.ho_cap_in = ho3_cap;
            A2.ho_stride_out = A3.ho_stride_in = ho3_stride;

            SKIS_HIP_TRY(hipStreamBeginCapture(gg.cs, hipStreamCaptureModeThreadLocal));
            gg.capturing = true;
            hipLaunchKernelGGL(k_chain_begin, dim3(1), dim3(64), 0, gg.cs, gc.ptr, (uint64_t)count, chunk);
            hipLaunchKernelGGL(k_roots, dim3(grid_cap(chunk, 256, 64)), dim3(256), 0, gg.cs, (uint64_t)cfg.first_id, 0u,
                               (const unsigned long long *)&gc.ptr->base, seed_lo, seed_hi, n, prep.C,
                               prep.alias.ptr, prep.row_ptr.ptr, prep.q.ptr, prep.P.ptr, prep.edges.ptr, prep.wbits.ptr, rec.ptr,
                               u1.ptr, rerr.ptr, (int)cfg.ris);
            hipLaunchKernelGGL(v0.fn, dim3(nb0), dim3(v0.threads), 0, gg.cs, A0);
            hipLaunchKernelGGL(vm.fn, dim3(nbm), dim3(vm.threads), 0, gg.cs, A1);
            hipLaunchKernelGGL(kTierHash, dim3((unsigned)nbh), dim3(64), 0, gg.cs, A2);
            hipLaunchKernelGGL(kTierGlobal, dim3((unsigned)nbg_g), dim3(TIERG_BLOCK), 0, gg.cs, A3);
            hipLaunchKernelGGL(k_chain_end, dim3(1), dim3(64), 0, gg.cs, gc.ptr);
            const hipError_t launch_err = hipGetLastError();
            gg.capturing = false;
            SKIS_HIP_TRY(hipStreamEndCapture(gg.cs, &gg.g));
            SKIS_HIP_TRY(launch_err);
            SKIS_HIP_TRY(hipGraphInstantiate(&gg.x, gg.g, nullptr, nullptr, 0));
            SKIS_HIP_TRY(hipEventRecord(ev[4], s));
            for (uint64_t r = 0; r < replays; ++r) SKIS_HIP_TRY(hipGraphLaunch(gg.x, s));
            SKIS_HIP_TRY(hipEventRecord(ev[5], s));
            ChainCtl hg{};
            SKIS_HIP_TRY(hipMemcpyAsync(&hg, gc.ptr, sizeof(hg), hipMemcpyDeviceToHost, s));
            read_counters();
            int herr = 0;
            SKIS_HIP_TRY(hipMemcpyAsync(&herr, rerr.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
            SKIS_HIP_TRY(hipStreamSynchronize(s));
            if ((hc.overflow & ~1) || herr)
                throw Error{SKIS_EHIP, "internal bounds check failed in the sampler (flags " +
                                           std::to_string(hc.overflow | herr) + ")"};
            if (hg.replays != replays || hg.cursor != count)
                throw Error{SKIS_EHIP, "internal error: the captured chain covered " + std::to_string(hg.cursor) +
                                           " of " + std::to_string(count) + " samples"};
            sk.deferred = hg.tot0;
            sk.deferred_global = hg.tot1;
            sk.deferred_bitmap = hg.tot2;
            sk.graph_replays = (uint32_t)replays;
            (void)hipGraphExecDestroy(gg.x);
            (void)hipGraphDestroy(gg.g);
            gg.x = nullptr;
            gg.g = nullptr;
            if (!hc.overflow) return;
            // every size is known now: a bound that holds whatever order the chunks took
            cap = staging_bound(hc.tier[0][1] + hc.tier[1][1] + hc.tier[2][1] + hc.tier[3][1], replays);
            staging.reset();
            if (attempt == 1) throw Error{SKIS_ENOMEM, "staging overflow after resize"};
        }
    };

    LtStats lts;
    if (lt) {
        // linear threshold model: the walk kernel and the long-walk kernel fill the same staging,
        // sizes, offsets and roots that the compaction below reads
        hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, s, (uint64_t)sizeof(Counters),
                           reinterpret_cast<unsigned char *>(ctr.ptr), (unsigned char)0);
        LtIo io;
        io.count = count;
        io.first_id = cfg.first_id;
        io.seed_lo = seed_lo;
        io.seed_hi = seed_hi;
        io.rec = rec.ptr;
        io.out_size = out_size.ptr;
        io.out_off = out_off.ptr;
        io.out_probed = reinterpret_cast<unsigned long long *>(sk.probed.ptr);
        io.medium = medium.ptr;
        io.n_medium = &ctr.ptr->n_medium;
        io.small_sort = SMALL_SORT;
        io.staging = &staging;
        io.staging_entries = cfg.staging_entries;
        SKIS_HIP_TRY(hipEventRecord(ev[4], s));
        sample_lt(arena, prep, n, io, lts, s);
        SKIS_HIP_TRY(hipEventRecord(ev[5], s));
        read_counters();
        sk.deferred = lts.long_samples;
        sk.deferred_global = 0;
        sk.deferred_bitmap = 0;
    }
    if (cfg.form == 1 && !lt) {
        // plain form: one launch per BFS level over all samples of a chunk
        staging.alloc(arena, cap);
        hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, s, (uint64_t)sizeof(Counters),
                           reinterpret_cast<unsigned char *>(ctr.ptr), (unsigned char)0);
        PlainInputs in{};
        in.count = count;
        in.row_ptr = prep.row_ptr.ptr;
        in.pairs = reinterpret_cast<const uint4 *>(prep.edges.ptr);
        in.nquads = (int64_t)(prep.edges.count / 4);
        in.wbits = prep.wbits.ptr;
        in.rec = rec.ptr;
        in.u1 = u1.ptr;
        in.seed_lo = seed_lo;
        in.seed_hi = seed_hi;
        in.first_id = cfg.first_id;
        in.expected_size = 48;
        in.staging = &staging;
        in.out_size = out_size.ptr;
        in.out_off = out_off.ptr;
        in.out_probed = reinterpret_cast<unsigned long long *>(sk.probed.ptr);
        in.medium = medium.ptr;
        in.n_medium = &ctr.ptr->n_medium;
        in.small_sort = SMALL_SORT;
        PlainOutputs po;
        SKIS_HIP_TRY(hipEventRecord(ev[4], s));
        sample_plain(arena, in, po, s);
        SKIS_HIP_TRY(hipEventRecord(ev[5], s));
        read_counters();
        sk.deferred = 0;
        sk.deferred_global = 0;
        sk.deferred_bitmap = 0;
        sk.plain_levels = po.levels;
    }
    if (cfg.form == 2) sample_chain_graph();
    for (int attempt = 0; attempt < 2 && cfg.form == 0 && !lt; ++attempt) {
        staging.alloc(arena, cap);
        hipLaunchKernelGGL(k_fill<unsigned char>, dim3(1), dim3(64), 0, s, (uint64_t)sizeof(Counters),
                           reinterpret_cast<unsigned char *>(ctr.ptr), (unsigned char)0);
        SampleArgs A{};
        A.n = n;
        A.row_ptr = prep.row_ptr.ptr;
        A.pairs = reinterpret_cast<const uint4 *>(prep.edges.ptr);
        A.nquads = (int64_t)(prep.edges.count / 4);
        A.wbits = prep.wbits.ptr;
        A.rec = rec.ptr;
        A.u1 = u1.ptr;
        A.j0 = cfg.first_id;
        A.seed_lo = seed_lo;
        A.seed_hi = seed_hi;
        A.next = &ctr.ptr->next;
        A.id_list = nullptr;
        A.id_count = count;
        A.big_row = cfg.big_row;
        A.staging = staging.ptr;
        A.stage_cap = cap;
        A.stage_used = &ctr.ptr->stage_used;
        A.out_size = out_size.ptr;
        A.out_off = out_off.ptr;
        A.out_probed = reinterpret_cast<unsigned long long *>(sk.probed.ptr);
        A.deferred = deferred.ptr;
        A.n_deferred = &ctr.ptr->n_deferred;
        A.medium = medium.ptr;
        A.n_medium = &ctr.ptr->n_medium;
        A.overflow = &ctr.ptr->overflow;
        A.words = words;
        A.tier_stats = ctr.ptr->tier[0];
        A.ho_state_out = ho_state.ptr;
        A.ho_nodes_out = ho_nodes.ptr;
        A.ho_cap_out = ho_cap;
        A.ho_stride_out = ho_stride;
        for (const void *p : {(const void *)A.row_ptr, (const void *)A.pairs, (const void *)A.rec, (const void *)A.u1,
                              (const void *)A.next, (const void *)A.staging, (const void *)A.stage_used,
                              (const void *)A.out_size, (const void *)A.out_off, (const void *)A.out_probed,
                              (const void *)A.deferred, (const void *)A.n_deferred, (const void *)A.medium,
                              (const void *)A.n_medium, (const void *)A.overflow, (const void *)deferred2.ptr})
            need(p, "sampler argument");
        // tier 0: every sample, LDS visited sets of cfg.visited nodes
        SKIS_HIP_TRY(hipEventRecord(ev[4], s));
        hipLaunchKernelGGL(v0.fn, dim3(nb0), dim3(v0.threads), 0, s, A);
        SKIS_HIP_TRY(hipGetLastError());
        SKIS_HIP_TRY(hipEventRecord(ev[5], s));
        read_counters();
        sk.deferred = hc.n_deferred;
        sk.deferred_global = 0;
        sk.deferred_bitmap = 0;
        ran_mid = ran_hash = ran_global = false;
        // handover from tier 1 to the hash tier, for a quarter of tier 1's samples (the first
        // ones it hands on; about 1 % of the samples outgrow tier 1 on the TRI and 1.4B-edge
        // workloads, 15 % of tier 1's)
        DevBuf<Handover> ho2_state, ho3_state;
        DevBuf<int32_t> ho2_nodes, ho3_nodes;
        DevBuf<uint32_t> ho2_slot;
        uint64_t ho2_cap = 0, ho3_cap = 0;
        if (hc.n_deferred > 0) {
            // tier 1: the samples that outgrew tier 0, LDS visited sets of 1024 nodes
            const uint64_t nd = hc.n_deferred;
            ho2_cap = std::min<uint64_t>(nd, std::max<uint64_t>(1024, nd / 4));
            ho2_state.alloc(arena, ho2_cap);
            ho2_nodes.alloc(arena, ho2_cap * (uint64_t)ho2_stride);
            reset_ids();
            A.id_list = deferred.ptr;
            A.id_count = nd;
            A.deferred = deferred2.ptr;
            A.big_row = std::max<uint32_t>(cfg.big_row, 1u << 20);
            A.tier_stats = ctr.ptr->tier[1];
            A.ho_state_out = ho2_state.ptr;
            A.ho_nodes_out = ho2_nodes.ptr;
            A.ho_cap_out = ho2_cap;
            A.ho_stride_out = ho2_stride;
            A.ho_state_in = ho_state.ptr;
            A.ho_nodes_in = ho_nodes.ptr;
            A.ho_cap_in = ho_cap;
            A.ho_stride_in = ho_stride;
            SKIS_HIP_TRY(hipEventRecord(ev[6], s));
            hipLaunchKernelGGL(vm.fn, dim3(nbm), dim3(vm.threads), 0, s, A);
            SKIS_HIP_TRY(hipGetLastError());
            SKIS_HIP_TRY(hipEventRecord(ev[7], s));
            ran_mid = true;
            read_counters();
        }
        if (ran_mid && hc.n_deferred > 0) {
            // tier 2: the samples that outgrew tier 1, hashes and lists sized to them in HBM
            const uint64_t nd = hc.n_deferred;
            if (nd > 1) {
                // a fixed pseudo-random order (Fisher-Yates, a 64-bit LCG): in tier 1's hand-on
                // order the largest samples can bunch up and start last.  Each sample keeps its
                // handover record: the record of new position q is the old position perm[q]
                // (records exist below ho2_cap).
                std::vector<uint32_t> ids(nd), perm(nd), moved(nd), slot(nd);
                SKIS_HIP_TRY(hipMemcpyAsync(ids.data(), deferred2.ptr, sizeof(uint32_t) * nd, hipMemcpyDeviceToHost, s));
                SKIS_HIP_TRY(hipStreamSynchronize(s));
                for (uint64_t k = 0; k < nd; ++k) perm[k] = (uint32_t)k;
                uint64_t x = 0x9E3779B97F4A7C15ull;
                for (uint64_t k = nd - 1; k > 0; --k) {
                    x = x * 6364136223846793005ull + 1442695040888963407ull;
                    const uint64_t r = (uint64_t)(((unsigned __int128)(x >> 11) * (k + 1)) >> 53);
                    std::swap(perm[k], perm[r]);
                }
                for (uint64_t q = 0; q < nd; ++q) {
                    moved[q] = ids[perm[q]];
                    slot[q] = perm[q] < ho2_cap ? perm[q] : 0xFFFFFFFFu;
                }
                ho2_slot.alloc(arena, nd);
                SKIS_HIP_TRY(hipMemcpyAsync(deferred2.ptr, moved.data(), sizeof(uint32_t) * nd, hipMemcpyHostToDevice, s));
                SKIS_HIP_TRY(hipMemcpyAsync(ho2_slot.ptr, slot.data(), sizeof(uint32_t) * nd, hipMemcpyHostToDevice, s));
                SKIS_HIP_TRY(hipStreamSynchronize(s));
            }
            sk.deferred_global = nd;
            alloc_hash_tier();
            ho3_cap = std::min<uint64_t>(nd, HO3_MAX);
            ho3_state.alloc(arena, ho3_cap);
            ho3_nodes.alloc(arena, ho3_cap * (uint64_t)ho3_stride);
            reset_ids();
            A.id_list = deferred2.ptr;
            A.id_count = nd;
            A.deferred = deferred.ptr; // tier 1 has read tier 0's list by now
            A.ghash = ghash.ptr;
            A.glist2 = glist2.ptr;
            A.big_row = std::max<uint32_t>(cfg.big_row, TIERH_BIG_ROW);
            A.tier_stats = ctr.ptr->tier[2];
            A.ho_state_out = ho3_state.ptr;
            A.ho_nodes_out = ho3_nodes.ptr;
            A.ho_cap_out = ho3_cap;
            A.ho_stride_out = ho3_stride;
            A.ho_state_in = ho2_state.ptr;
            A.ho_nodes_in = ho2_nodes.ptr;
            A.ho_slot_in = ho2_slot.ptr; // null when there was nothing to shuffle
            A.ho_cap_in = ho2_cap;
            A.ho_stride_in = ho2_stride;
            SKIS_HIP_TRY(hipEventRecord(ev[8], s));
            hipLaunchKernelGGL(kTierHash, dim3((unsigned)nbh), dim3(64), 0, s, A);
            SKIS_HIP_TRY(hipGetLastError());
            SKIS_HIP_TRY(hipEventRecord(ev[9], s));
            ran_hash = true;
            read_counters();
        }
        if (ran_hash && hc.n_deferred > 0) {
            // tier 3: what is left, a bitmap and a node list of n entries per slot in HBM
            const uint64_t nd = hc.n_deferred;
            sk.deferred_bitmap = nd;
            const uint64_t slots = (uint64_t)nbg * TIERG_SLOTS;
            DevBuf<uint32_t> gbits;
            DevBuf<int32_t> glist;
            gbits.alloc(arena, slots * words);
            glist.alloc(arena, slots * (uint64_t)n);
            hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_cap(slots * words, 256)), dim3(256), 0, s, slots * words,
                               gbits.ptr, 0u);
            reset_ids();
            A.id_list = deferred.ptr;
            A.id_count = nd;
            A.id_perm = 1;              // a fixed scramble of the hand-on order
            A.deferred = deferred2.ptr; // unused: the bitmap tier finishes every sample
            A.gbits = gbits.ptr;
            A.glist = glist.ptr;
            A.tier_stats = ctr.ptr->tier[3];
            A.ho_state_out = nullptr;
            A.ho_nodes_out = nullptr;
            A.ho_cap_out = 0;
            A.ho_state_in = ho3_state.ptr; // records follow the list position
            A.ho_nodes_in = ho3_nodes.ptr;
            A.ho_slot_in = nullptr;
            A.ho_cap_in = ho3_cap;
            A.ho_stride_in = ho3_stride;
            need(A.gbits, "gbits");
            need(A.glist, "glist");
            SKIS_HIP_TRY(hipEventRecord(ev[10], s));
            hipLaunchKernelGGL(kTierGlobal, dim3(nbg), dim3(TIERG_BLOCK), 0, s, A);
            SKIS_HIP_TRY(hipGetLastError());
            SKIS_HIP_TRY(hipEventRecord(ev[11], s));
            ran_global = true;
            read_counters();
        }
        int herr = 0;
        SKIS_HIP_TRY(hipMemcpyAsync(&herr, rerr.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        if ((hc.overflow & ~1) || herr)
            throw Error{SKIS_EHIP, "internal bounds check failed in the sampler (flags " +
                                       std::to_string(hc.overflow | herr) + ")"};
        if (!hc.overflow) break;
        // every size is known now: a bound that holds whatever order the chunks took
        cap = staging_bound(hc.tier[0][1] + hc.tier[1][1] + hc.tier[2][1] + hc.tier[3][1], 1);
        staging.reset();
        if (attempt == 1) throw Error{SKIS_ENOMEM, "staging overflow after resize"};
    }
    SKIS_HIP_TRY(hipEventRecord(ev[2], s));
    for (int t = 0; t < 4; ++t)
        for (int k = 0; k < 5; ++k) sk.tier_stats[t][k] = hc.tier[t][k];
    if (lt) { // stage 0: the walk kernel, stage 1: the long walks; picks drawn in place of swept edges
        const uint64_t ts[2][5] = {{lts.walk_samples, lts.walk_entries, lts.walk_probed, lts.walk_picks, lts.walk_entries},
                                   {lts.long_samples, lts.long_entries, lts.long_probed, lts.long_picks, lts.long_entries}};
        for (int t = 0; t < 4; ++t)
            for (int k = 0; k < 5; ++k) sk.tier_stats[t][k] = t < 2 ? ts[t][k] : 0;
    }

    // every sample must have finished in one of the tiers; the samples above SORT_LDS_MAX
    // nodes (all listed in `medium`) are counted for k_gather_large
    DevBuf<unsigned long long> tally;
    tally.alloc(arena, 2);
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)2, tally.ptr, 0ull);
    hipLaunchKernelGGL(k_count_value, dim3(grid_cap(count, 256, 1)), dim3(256), 0, s, (uint64_t)count, out_size.ptr,
                       DEFERRED, tally.ptr);
    if (hc.n_medium > 0)
        hipLaunchKernelGGL(k_count_listed_above, dim3(grid_cap(hc.n_medium, 256, 1)), dim3(256), 0, s,
                           (uint64_t)hc.n_medium, medium.ptr, out_size.ptr, (uint32_t)SORT_LDS_MAX, tally.ptr + 1);
    SKIS_HIP_TRY(hipGetLastError());
    unsigned long long htally[2] = {0, 0};
    SKIS_HIP_TRY(hipMemcpyAsync(htally, tally.ptr, sizeof(htally), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    if (htally[0])
        throw Error{SKIS_EHIP, "internal error: " + std::to_string(htally[0]) + " samples did not finish"};
    const uint64_t n_large = htally[1];

    // CSR: sample_ptr = exclusive scan of sizes, then sorted copies
    sk.T = count;
    sk.sample_ptr.alloc(arena, (size_t)count + 1);
    excl_scan_u32_to_i64(arena, out_size.ptr, sk.sample_ptr.ptr, count, sk.sample_ptr.ptr + count, s);
    int64_t total = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&total, sk.sample_ptr.ptr + count, sizeof(total), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    sk.entries = (uint64_t)total;
    if (count && !cfg.staging_entries) set_entries_per_sample_hint(n, m, (double)total / (double)count);
    sk.nodes.alloc(arena, (size_t)total);
    if (cfg.owners) sk.owner.alloc(arena, (size_t)total);
    else sk.owner.reset();
    int32_t *const owner_p = cfg.owners ? sk.owner.ptr : nullptr;
    // samples by size class (the lists live until the side stream below has joined)
    DevBuf<unsigned long long> cls;
    DevBuf<uint32_t> lists;
    // The register sorts of the 1025-8192-node samples (bound by their ALU work) run on a
    // second stream beside the size classes (bound by memory), dispatched first, and the
    // largest size class (513-1024 nodes) follows them there; the caller's stream waits for
    // them before the large samples and everything after (also when an error leaves this
    // function early: the buffers they use are released on that stream).
    const bool mid_side = hc.n_medium > n_large;
    hipEvent_t mfork = nullptr, mjoin = nullptr, mcls = nullptr;
    bool mid_pending = false;
    hipError_t mid_err = hipSuccess;
    struct MidEvents {
        hipStream_t s;
        hipEvent_t *a, *b, *c;
        bool *pending;
        ~MidEvents()
        {
            if (*pending) (void)hipStreamWaitEvent(s, *b, 0);
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
            if (*c) (void)hipEventDestroy(*c);
        }
    } mid_events{s, &mfork, &mjoin, &mcls, &mid_pending};
    if (mid_side) {
        hipStream_t s2 = side_stream();
        SKIS_HIP_TRY(hipEventCreateWithFlags(&mfork, hipEventDisableTiming));
        SKIS_HIP_TRY(hipEventCreateWithFlags(&mjoin, hipEventDisableTiming));
        SKIS_HIP_TRY(hipEventCreateWithFlags(&mcls, hipEventDisableTiming));
        SKIS_HIP_TRY(hipEventRecord(mfork, s));
        hipError_t e = hipStreamWaitEvent(s2, mfork, 0);
        if (e == hipSuccess) {
            const unsigned gm = grid_cap(hc.n_medium, 1, 16);
            hipLaunchKernelGGL((k_gather_medium_regs<32>), dim3(gm), dim3(64), 0, s2, (uint64_t)hc.n_medium,
                               medium.ptr, out_size.ptr, out_off.ptr, sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr,
                               owner_p);
            hipLaunchKernelGGL(k_gather_block<256>, dim3(grid_cap(hc.n_medium, 1, 4)), dim3(256), 0, s2,
                               (uint64_t)hc.n_medium, medium.ptr, out_size.ptr, out_off.ptr, sk.sample_ptr.ptr,
                               staging.ptr, sk.nodes.ptr, owner_p);
            hipLaunchKernelGGL(k_gather_block<512>, dim3(grid_cap(hc.n_medium, 1, 2)), dim3(512), 0, s2,
                               (uint64_t)hc.n_medium, medium.ptr, out_size.ptr, out_off.ptr, sk.sample_ptr.ptr,
                               staging.ptr, sk.nodes.ptr, owner_p);
            e = hipGetLastError();
        }
        const hipError_t rec = hipEventRecord(mjoin, s2);
        if (rec != hipSuccess) (void)hipStreamSynchronize(s2); // no event to wait on: drain it here
        SKIS_HIP_TRY(rec);
        mid_pending = true;
        mid_err = e;
    }
    {
        // one segmented sort per class
        cls.alloc(arena, 2 * GATHER_CLASSES);
        lists.alloc(arena, count);
        hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)(2 * GATHER_CLASSES),
                           cls.ptr, 0ull);
        hipLaunchKernelGGL(k_class_count, dim3(grid_cap(count, 256, 1)), dim3(256), 0, s, (uint64_t)count, out_size.ptr,
                           cls.ptr);
        hipLaunchKernelGGL(k_class_fill, dim3(grid_cap(count, CLASS_CHUNK, 8)), dim3(256), 0, s, (uint64_t)count,
                           out_size.ptr, cls.ptr, cls.ptr + GATHER_CLASSES, lists.ptr);
        const unsigned gg = grid_cap(count, 8, 64);
        const uint32_t *const sz_p = out_size.ptr;
        const unsigned long long *const off_p = out_off.ptr;
        bool last_class_side = false;
        if (mid_pending) {
            hipStream_t s2 = side_stream();
            SKIS_HIP_TRY(hipEventRecord(mcls, s));
            SKIS_HIP_TRY(hipStreamWaitEvent(s2, mcls, 0));
            hipLaunchKernelGGL((k_gather_sort<64, 16>), dim3(gg), dim3(64), 0, s2, 7, cls.ptr, lists.ptr, sz_p, off_p,
                               sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
            const hipError_t e7 = hipGetLastError();
            const hipError_t rec = hipEventRecord(mjoin, s2); // the join now follows this class too
            if (rec != hipSuccess) (void)hipStreamSynchronize(s2);
            SKIS_HIP_TRY(rec);
            if (mid_err == hipSuccess) mid_err = e7;
            last_class_side = true;
        }
        hipLaunchKernelGGL((k_gather_sort<8, 1>), dim3(gg), dim3(64), 0, s, 0, cls.ptr, lists.ptr, sz_p, off_p,
                           sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        hipLaunchKernelGGL((k_gather_sort<16, 1>), dim3(gg), dim3(64), 0, s, 1, cls.ptr, lists.ptr, sz_p, off_p,
                           sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        hipLaunchKernelGGL((k_gather_sort<32, 1>), dim3(gg), dim3(64), 0, s, 2, cls.ptr, lists.ptr, sz_p, off_p,
                           sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        hipLaunchKernelGGL((k_gather_sort<64, 1>), dim3(gg), dim3(64), 0, s, 3, cls.ptr, lists.ptr, sz_p, off_p,
                           sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        hipLaunchKernelGGL((k_gather_sort<64, 2>), dim3(gg), dim3(64), 0, s, 4, cls.ptr, lists.ptr, sz_p, off_p,
                           sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        hipLaunchKernelGGL((k_gather_sort<64, 4>), dim3(gg), dim3(64), 0, s, 5, cls.ptr, lists.ptr, sz_p, off_p,
                           sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        hipLaunchKernelGGL((k_gather_sort<64, 8>), dim3(gg), dim3(64), 0, s, 6, cls.ptr, lists.ptr, sz_p, off_p,
                           sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        if (!last_class_side)
            hipLaunchKernelGGL((k_gather_sort<64, 16>), dim3(gg), dim3(64), 0, s, 7, cls.ptr, lists.ptr, sz_p, off_p,
                               sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr, owner_p);
        SKIS_HIP_TRY(hipGetLastError());
    }
    if (mid_pending) {
        SKIS_HIP_TRY(hipStreamWaitEvent(s, mjoin, 0));
        mid_pending = false;
        SKIS_HIP_TRY(mid_err);
    }
    if (n_large > 0) {
        // one bitmap of n bits and one summary bit per bitmap word for each workgroup, at
        // most LARGE_BITMAP_BUDGET bytes of them
        const uint64_t words = ((uint64_t)n + 31) / 32, swords = (words + 31) / 32;
        const uint64_t per_wg = (words + swords) * 4;
        uint64_t g = std::min<uint64_t>({n_large, (uint64_t)device_cu_count() * 2,
                                         std::max<uint64_t>(1, LARGE_BITMAP_BUDGET / per_wg)});
        DevBuf<uint32_t> lbits, lsumm;
        DevBuf<int> lerr;
        lbits.alloc(arena, g * words);
        lsumm.alloc(arena, g * swords);
        lerr.alloc(arena, 1);
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_cap(g * words, 256)), dim3(256), 0, s, g * words, lbits.ptr, 0u);
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_cap(g * swords, 256)), dim3(256), 0, s, g * swords, lsumm.ptr, 0u);
        hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (uint64_t)1, lerr.ptr, 0);
        hipLaunchKernelGGL(k_gather_large, dim3((unsigned)g), dim3(LARGE_BLOCK), 0, s, (uint64_t)hc.n_medium,
                           medium.ptr, out_size.ptr, out_off.ptr, sk.sample_ptr.ptr, staging.ptr, sk.nodes.ptr,
                           owner_p, lbits.ptr, lsumm.ptr, words, swords, lerr.ptr);
        SKIS_HIP_TRY(hipGetLastError());
        int herr = 0;
        SKIS_HIP_TRY(hipMemcpyAsync(&herr, lerr.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        if (herr) throw Error{SKIS_EHIP, "internal error: a large sample failed its sort (flags " +
                                             std::to_string(herr) + ")"};
    }
    sk.roots.alloc(arena, count);
    hipLaunchKernelGGL(k_roots_out, dim3(grid_cap(count, 256)), dim3(256), 0, s, count, rec.ptr, sk.roots.ptr);
    SKIS_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)1, &ctr.ptr->next, 0ull);
    hipLaunchKernelGGL(k_sum_u64, dim3(grid_cap(count, 256, 1)), dim3(256), 0, s, (uint64_t)count,
                       reinterpret_cast<const unsigned long long *>(sk.probed.ptr), &ctr.ptr->next);
    SKIS_HIP_TRY(hipGetLastError());
    unsigned long long ptot = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&ptot, &ctr.ptr->next, sizeof(ptot), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipEventRecord(ev[3], s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    sk.probed_total = ptot;
    if (cfg.form == 1) { // the plain form is one stage
        sk.tier_stats[0][0] = count;
        sk.tier_stats[0][1] = (uint64_t)total;
        sk.tier_stats[0][2] = ptot;
        sk.tier_stats[0][3] = ptot;            // every probed edge is swept once
        sk.tier_stats[0][4] = (uint64_t)total; // and every node expanded once
    }
    float ms = 0;
    SKIS_HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
    sk.ms_roots = ms;
    SKIS_HIP_TRY(hipEventElapsedTime(&ms, ev[1], ev[2]));
    sk.ms_sample = ms;
    SKIS_HIP_TRY(hipEventElapsedTime(&ms, ev[2], ev[3]));
    sk.ms_compact = ms;
    SKIS_HIP_TRY(hipEventElapsedTime(&ms, ev[4], ev[5]));
    sk.ms_tier0 = lt ? lts.ms_walk : ms;
    sk.ms_tier1 = lt ? lts.ms_long : 0;
    sk.ms_tier2 = 0;
    sk.ms_tier3 = 0;
    if (ran_mid) {
        SKIS_HIP_TRY(hipEventElapsedTime(&ms, ev[6], ev[7]));
        sk.ms_tier1 = ms;
    }
    if (ran_hash) {
        SKIS_HIP_TRY(hipEventElapsedTime(&ms, ev[8], ev[9]));
        sk.ms_tier2 = ms;
    }
    if (ran_global) {
        SKIS_HIP_TRY(hipEventElapsedTime(&ms, ev[10], ev[11]));
        sk.ms_tier3 = ms;
    }
}

// Cuts a built sketch (before its transpose) to its first T' samples, T' the smallest count
// whose sizes sum to at least budget (T' = T when all of them together hold fewer entries).
void truncate_to_budget(Sketch &sk, uint64_t budget, hipStream_t s)
{
    if (sk.T == 0 || sk.entries < budget) return;
    DevBuf<unsigned long long> t;
    t.alloc(sk.arena, 2);
    hipLaunchKernelGGL(k_first_reaching, dim3(1), dim3(64), 0, s, sk.sample_ptr.ptr, (uint64_t)sk.T, (int64_t)budget,
                       t.ptr);
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (uint64_t)1, t.ptr + 1, 0ull);
    SKIS_HIP_TRY(hipGetLastError());
    unsigned long long T2 = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&T2, t.ptr, sizeof(T2), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    if (T2 < 1 || T2 > sk.T) throw Error{SKIS_EHIP, "internal error: budget cut outside the sketch"};
    hipLaunchKernelGGL(k_sum_u64, dim3(grid_cap(T2, 256, 1)), dim3(256), 0, s, (uint64_t)T2,
                       reinterpret_cast<const unsigned long long *>(sk.probed.ptr), t.ptr + 1);
    SKIS_HIP_TRY(hipGetLastError());
    int64_t ent = 0;
    unsigned long long ptot = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&ent, sk.sample_ptr.ptr + T2, sizeof(ent), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipMemcpyAsync(&ptot, t.ptr + 1, sizeof(ptot), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    sk.T = T2;
    sk.entries = (uint64_t)ent;
    sk.probed_total = ptot;
}

} // namespace skis
