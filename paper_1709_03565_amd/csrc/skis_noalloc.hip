// skis_noalloc.hip -- skis_estimate_noalloc: the estimates of skis_estimate (Eq. eq21) with no
// device allocation, for callers that cannot allocate.  Its scratch -- the error word, the
// list of large sets and the per-set bitmaps -- lives in one file-scope device array that
// every GPU the library runs on holds until the process ends.  Calls that overlap on one GPU
// share that array and race.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "skis_internal.h"
#include "skis_query.h"

namespace skis {

// Layout in 32-bit words: [0, NA_LIST) the error word (word 0); [NA_LIST, NA_BITS) the large
// sets of one host chunk as int64 set indexes; [NA_BITS, NA_WORDS) the bitmaps.
constexpr uint64_t NA_WORDS = (32ull << 20) / 4; // 32 MiB
constexpr int NA_CHUNK = 1024;                   // sets routed per host round
constexpr uint64_t NA_LIST = 64;
constexpr uint64_t NA_BITS = NA_LIST + 2 * NA_CHUNK;
static_assert(NA_BITS % 64 == 0, "the bitmaps start 256-byte aligned");

static __device__ __align__(256) uint32_t scratch[NA_WORDS];

namespace {

constexpr int NA_DEVICES = 64;
std::mutex g_na_mu;
uint32_t *g_na_ptr[NA_DEVICES] = {};

// The current device's copy of `scratch`, looked up once per device.
uint32_t *scratch_ptr()
{
    int d = 0;
    SKIS_HIP_TRY(hipGetDevice(&d));
    if (d < 0 || d >= NA_DEVICES) throw Error{SKIS_EHIP, "device index out of range for the no-alloc scratch"};
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[d]) {
        void *p = nullptr;
        SKIS_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error{SKIS_EHIP, "hipGetSymbolAddress returned no address for the scratch array"};
        g_na_ptr[d] = static_cast<uint32_t *>(p);
    }
    return g_na_ptr[d];
}

__global__ __launch_bounds__(256) void k_na_fill(uint64_t count, uint32_t *__restrict__ p, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void na_fill(uint32_t *p, uint64_t count, hipStream_t s)
{
    if (!count) return;
    uint64_t g = (count + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (g > cap) g = cap;
    hipLaunchKernelGGL(k_na_fill, dim3((unsigned)g), dim3(256), 0, s, count, p, 0u);
    SKIS_HIP_TRY(hipGetLastError());
}

} // namespace

void estimate_noalloc(const Sketch &sk, int32_t Q, const int64_t *set_ptr, const int32_t *set_nodes, uint64_t *cov,
                      double *est, hipStream_t s)
{
    const uint64_t wordsT = sk.T ? (sk.T + 31) / 32 : 1;
    const uint64_t wordsN = ((uint64_t)sk.n + 31) / 32;
    const uint64_t room = NA_WORDS - NA_BITS;
    if (wordsT > room)
        throw Error{SKIS_EINVAL, "the sketch's T-bit bitmap exceeds the no-alloc scratch (" +
                                     std::to_string(NA_WORDS * 4) + " bytes)"};
    uint32_t *base = scratch_ptr();
    int *err = reinterpret_cast<int *>(base);
    int64_t *qlist = reinterpret_cast<int64_t *>(base + NA_LIST);
    uint32_t *bits = base + NA_BITS;
    // sets per launch: one bitmap of T bits each (small sets); a bitmap and a node bitmap of n
    // bits each (large sets)
    const uint64_t nb = std::min<uint64_t>(room / wordsT, (uint64_t)NA_CHUNK);
    const uint64_t ng = std::min<uint64_t>(room / (wordsT + wordsN), (uint64_t)NA_CHUNK);
    // the array keeps the last call's contents: clear what this call uses
    na_fill(base, NA_LIST, s);
    na_fill(bits, std::max<uint64_t>(nb * wordsT, ng * (wordsT + wordsN)), s);
    int64_t hp[NA_CHUNK + 1];
    int64_t lg[NA_CHUNK];
    for (int64_t c0 = 0; c0 < Q; c0 += NA_CHUNK) {
        const int ch = (int)std::min<int64_t>(NA_CHUNK, Q - c0);
        SKIS_HIP_TRY(hipMemcpyAsync(hp, set_ptr + c0, sizeof(int64_t) * (size_t)(ch + 1), hipMemcpyDeviceToHost, s));
        SKIS_HIP_TRY(hipStreamSynchronize(s));
        int nl = 0;
        for (int i = 0; i < ch; ++i) {
            const int64_t k = hp[i + 1] - hp[i];
            if (k < 0 || hp[i] < 0) throw Error{SKIS_EINVAL, "set_ptr must be nondecreasing from 0"};
            if (k > EST_MAX_SET) lg[nl++] = c0 + i;
        }
        if (hp[ch] > hp[0] && !set_nodes) throw Error{SKIS_EINVAL, "set_nodes must not be NULL"};
        if (nl > 0 && ng == 0)
            throw Error{SKIS_EINVAL, "a set above " + std::to_string(EST_MAX_SET) +
                                         " entries needs more than the no-alloc scratch holds on this sketch"};
        for (int b0 = 0; b0 < ch; b0 += (int)nb)
            estimate_launch_small(sk, c0 + b0, (int32_t)std::min<int64_t>((int64_t)nb, ch - b0), set_ptr, set_nodes,
                                  bits, wordsT, reinterpret_cast<unsigned long long *>(cov), est, err, s);
        if (nl > 0) {
            SKIS_HIP_TRY(hipMemcpyAsync(qlist, lg, sizeof(int64_t) * (size_t)nl, hipMemcpyHostToDevice, s));
            for (int g0 = 0; g0 < nl; g0 += (int)ng)
                estimate_launch_large(sk, qlist, g0, (int32_t)std::min<int>((int)ng, nl - g0), set_ptr, set_nodes,
                                      bits, wordsT, bits + ng * wordsT, reinterpret_cast<unsigned long long *>(cov),
                                      est, err, s);
            SKIS_HIP_TRY(hipStreamSynchronize(s)); // lg is rewritten by the next chunk
        }
    }
    int herr = 0;
    SKIS_HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    if (herr & 1) throw Error{SKIS_EINVAL, "set_ptr must be nondecreasing"};
    if (herr & 4) throw Error{SKIS_EINVAL, "a seed set holds a node id outside [0, n)"};
    if (herr) throw Error{SKIS_EHIP, "internal error in the estimate kernel (flags " + std::to_string(herr) + ")"};
}

} // namespace skis

extern "C" int skis_estimate_noalloc(const skis_sketch *hc, int32_t num_sets, const int64_t *set_ptr,
                                     const int32_t *set_nodes, uint64_t *cov, double *est, hipStream_t stream)
{
    try {
        skis::set_error("");
        if (!hc) throw skis::Error{SKIS_EINVAL, "NULL sketch"};
        if (num_sets < 0) throw skis::Error{SKIS_EINVAL, "num_sets must be >= 0"};
        if (num_sets == 0) return SKIS_OK;
        if (!set_ptr || !cov || !est) throw skis::Error{SKIS_EINVAL, "NULL argument"};
        if (!hc->core.has_inverse && hc->core.T > 0)
            throw skis::Error{SKIS_EINVAL, "sketch was built without the inverse index"};
        skis::estimate_noalloc(hc->core, num_sets, set_ptr, set_nodes, cov, est, stream);
        return SKIS_OK;
    } catch (const skis::Error &e) {
        skis::set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        skis::set_error(e.what());
        return SKIS_EHIP;
    }
}
