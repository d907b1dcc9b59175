// skis_im.cpp -- influence maximisation with the SKIS sketch: the stop-and-stare driver D-SSA
// run on IIS samples (the paper's "SKIS-based IM algorithms", Sec. 5, and its appendix on
// D-SSA with SKIS).  The graph is preprocessed once; iteration t draws the sketch R of sample
// ids [0, T) and the check sketch R^c of ids [T, 2T) from the same stream, picks k seeds by the
// greedy of Alg. 3 on R, estimates them on R^c by Eq. (eq21), and stops when the coverage and
// error conditions of D-SSA hold; otherwise T doubles (R grows by R^c).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "skis_internal.h"
#include "skis_query.h"

namespace skis {
namespace {

// A sketch of sample ids [first, first + T) with its transpose, sharing the preprocessing.
std::unique_ptr<Sketch> range_sketch(const Prep &prep, int32_t n, int64_t m, uint64_t first, uint64_t T,
                                     uint64_t seed, const SampleConfig &base, hipStream_t s)
{
    auto sk = std::make_unique<Sketch>();
    sk->arena.stream = s;
    sk->n = n;
    sk->Gamma = prep.Gamma;
    sk->C = prep.C;
    SampleConfig cfg = base;
    cfg.first_id = first;
    cfg.owners = true;
    sample_and_compact(sk->arena, prep, n, m, T, seed, cfg, *sk, s);
    sk->q.alloc(sk->arena, (size_t)n);
    SKIS_HIP_TRY(hipMemcpyAsync(sk->q.ptr, prep.q.ptr, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    build_inverse(*sk, s);
    SKIS_HIP_TRY(hipStreamSynchronize(s));
    return sk;
}

} // namespace

// D-SSA's sample bounds with the SKIS coverage threshold (binary64, in this order; only libm's
// log, log2, exp and ceil are called).
//   Upsilon(eps, d) = (2 + 2 eps / 3) ln(1 / d) / eps^2
//   N_max = 8 (1 - 1/e) / (2 + 2 eps / 3) * Upsilon(eps, delta / (6 C(n, k))) * n / k
//   t_max = ceil(log2(2 N_max / Upsilon(eps, delta / 3)))
//   Lambda = 1 + (1 + eps) (2 Gamma / n + 2 eps / 3) ln(3 t_max / delta) / eps^2
void dssa_bounds(int32_t n, int32_t k, double Gamma, double eps, double delta, double *N_max, double *t_max,
                 double *Lambda)
{
    // ln C(n, k) as the sum of ln((n - k + i) / i), i = 1 .. k, each term ln(n - k + i) - ln(i)
    double lnC = 0.0;
    for (int32_t i = 1; i <= k; ++i) lnC += std::log((double)(n - k + i)) - std::log((double)i);
    const double a = 2.0 + 2.0 * eps / 3.0;
    const double ups_nk = a * (std::log(6.0 / delta) + lnC) / (eps * eps);
    const double ups_3 = a * std::log(3.0 / delta) / (eps * eps);
    const double e1 = 1.0 - 1.0 / std::exp(1.0);
    *N_max = 8.0 * e1 / a * ups_nk * (double)n / (double)k;
    *t_max = std::ceil(std::log2(2.0 * *N_max / ups_3));
    if (*t_max < 1.0) *t_max = 1.0;
    *Lambda = 1.0 + (1.0 + eps) * (2.0 * Gamma / (double)n + 2.0 * eps / 3.0) * std::log(3.0 * *t_max / delta) /
                        (eps * eps);
}

} // namespace skis

extern "C" int skis_im_dssa(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *w,
                            int32_t k, double eps, double delta, uint64_t seed, const skis_options *opt_in,
                            hipStream_t stream, int32_t *seeds_out, skis_dssa_info *info)
{
    try {
        skis::set_error("");
        if (n <= 0) throw skis::Error{SKIS_EINVAL, "n must be positive"};
        if (m < 0 || m > (int64_t)INT32_MAX) throw skis::Error{SKIS_EINVAL, "m must be in [0, 2^31)"};
        if (!row_ptr || (m > 0 && (!col || !w)) || !seeds_out || !info)
            throw skis::Error{SKIS_EINVAL, "NULL argument"};
        if (k < 1 || k > n) throw skis::Error{SKIS_EINVAL, "k must be in [1, n]"};
        const double e1 = 1.0 - 1.0 / std::exp(1.0);
        if (!(eps > 0.0 && eps < e1)) throw skis::Error{SKIS_EINVAL, "eps must be in (0, 1 - 1/e)"};
        if (!(delta > 0.0 && delta < 1.0)) throw skis::Error{SKIS_EINVAL, "delta must be in (0, 1)"};
        skis_options opt;
        skis_default_options(&opt);
        if (opt_in) {
            if (opt_in->slots_per_block) opt.slots_per_block = opt_in->slots_per_block;
            if (opt_in->visited_threshold) opt.visited_threshold = opt_in->visited_threshold;
            if (opt_in->big_row) opt.big_row = opt_in->big_row;
            if (opt_in->threads_per_block) opt.threads_per_block = opt_in->threads_per_block;
            if (opt_in->quads_per_lane) opt.quads_per_lane = opt_in->quads_per_lane;
            opt.max_device_bytes = opt_in->max_device_bytes;
            opt.model = opt_in->model;
        }
        if (opt.model > 1) throw skis::Error{SKIS_EINVAL, "model must be 0 (independent cascade) or 1 (linear threshold)"};
        std::memset(info, 0, sizeof(*info));
        skis::Arena arena;
        arena.cap = opt.max_device_bytes;
        arena.stream = stream;
        skis::Prep prep;
        skis::preprocess(arena, n, m, row_ptr, col, w, true, prep, stream, (int)opt.model);
        info->Gamma = prep.Gamma;
        if (prep.C == 0) {
            // Gamma = 0: no edge can be live, I(S) = |S| for every S; the greedy's tie rule picks 0..k-1
            for (int32_t i = 0; i < k; ++i) seeds_out[i] = i;
            info->est_select = info->est_check = (double)k;
            skis::set_error("Gamma = 0: no non-singular sample exists");
            return SKIS_WDEGENERATE;
        }
        double N_max, t_max, Lambda;
        skis::dssa_bounds(n, k, prep.Gamma, eps, delta, &N_max, &t_max, &Lambda);
        info->N_max = N_max;
        info->t_max = t_max;
        info->Lambda = Lambda;
        skis::SampleConfig cfg;
        cfg.threads = opt.threads_per_block;
        cfg.slots = opt.slots_per_block;
        cfg.visited = opt.visited_threshold;
        cfg.big_row = opt.big_row;
        cfg.qpl = opt.quads_per_lane;
        cfg.model = (int)opt.model;
        skis::DevBuf<int32_t> d_seeds;
        skis::DevBuf<uint64_t> d_marg;
        skis::DevBuf<int64_t> d_ptr;
        skis::DevBuf<unsigned long long> d_cov;
        skis::DevBuf<double> d_est;
        d_seeds.alloc(arena, (size_t)k);
        d_marg.alloc(arena, (size_t)k);
        d_ptr.alloc(arena, 2);
        d_cov.alloc(arena, 1);
        d_est.alloc(arena, 1);
        const int64_t hptr[2] = {0, k};
        SKIS_HIP_TRY(hipMemcpyAsync(d_ptr.ptr, hptr, sizeof(hptr), hipMemcpyHostToDevice, stream));
        SKIS_HIP_TRY(hipStreamSynchronize(stream));
        uint64_t T = (uint64_t)std::ceil(Lambda);
        if (T < 1) T = 1;
        for (uint32_t t = 1;; ++t) {
            if (2 * T >= (1ull << 31)) throw skis::Error{SKIS_EINVAL, "the sketches would need 2^31 sample ids or more"};
            uint64_t cov_R = 0;
            double est_R = 0.0;
            {
                auto R = skis::range_sketch(prep, n, m, 0, T, seed, cfg, stream);
                skis::QueryScratch qs;
                skis::greedy(*R, qs, k, d_seeds.ptr, d_marg.ptr, &cov_R, &est_R, stream);
                SKIS_HIP_TRY(hipStreamSynchronize(stream));
                R->arena.idle_on_destroy = true;
            }
            info->iterations = t;
            info->T = T;
            info->cov_select = cov_R;
            info->est_select = est_R;
            bool done = false;
            if ((double)cov_R >= Lambda) {
                unsigned long long cov_c = 0;
                double est_c = 0.0;
                {
                    auto Rc = skis::range_sketch(prep, n, m, T, T, seed, cfg, stream);
                    skis::QueryScratch qs;
                    skis::estimate_batch(*Rc, qs, 1, d_ptr.ptr, d_seeds.ptr, reinterpret_cast<uint64_t *>(d_cov.ptr),
                                         d_est.ptr, stream);
                    SKIS_HIP_TRY(hipMemcpyAsync(&cov_c, d_cov.ptr, sizeof(cov_c), hipMemcpyDeviceToHost, stream));
                    SKIS_HIP_TRY(hipMemcpyAsync(&est_c, d_est.ptr, sizeof(est_c), hipMemcpyDeviceToHost, stream));
                    SKIS_HIP_TRY(hipStreamSynchronize(stream));
                    Rc->arena.idle_on_destroy = true;
                }
                // D-SSA's error terms on the two sketches (the appendix's eps_1, eps_2, eps_3)
                const double p2 = (double)(1ull << (t - 1));
                const double eps1 = est_R / est_c - 1.0;
                const double eps2 = eps * std::sqrt((double)n * (1.0 + eps) / (p2 * est_c));
                const double eps3 = eps * std::sqrt((double)n * (1.0 + eps) * (e1 - eps) / ((1.0 + eps / 3.0) * p2 * est_c));
                const double eps_t = (eps1 + eps2 + eps1 * eps2) * (e1 - eps) + e1 * eps3;
                info->cov_check = cov_c;
                info->est_check = est_c;
                info->eps1 = eps1;
                info->eps2 = eps2;
                info->eps3 = eps3;
                info->eps_t = eps_t;
                if (eps_t <= eps) {
                    info->stopped = 1;
                    done = true;
                }
            }
            if (!done && (double)T >= N_max) done = true; // the cap: the last iteration's seeds
            if (done) break;
            T *= 2;
        }
        SKIS_HIP_TRY(hipMemcpyAsync(seeds_out, d_seeds.ptr, sizeof(int32_t) * (size_t)k, hipMemcpyDeviceToHost, stream));
        SKIS_HIP_TRY(hipStreamSynchronize(stream));
        arena.idle_on_destroy = true;
        return SKIS_OK;
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
