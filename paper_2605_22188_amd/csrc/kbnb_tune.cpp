// kbnb_tune.cpp -- batch-width and certificate-period autotuner (the batch
// size sweep of App. E.4, done as a timed search on the device at hand).
//
// Every candidate is a separate problem created from the caller's
// description with that batch width and certificate period; all candidates
// bound the same node sample through submit_nodes / poll_bounds, so the rate
// includes admission, the captured rounds, certificates and retirement --
// everything a caller of the library pays.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/kbnb.h"

namespace kbnb {
int set_error(int code, const char *fmt, ...);
}

namespace {

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014)
struct SplitMix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    int below(int n) { return (int)(next() % (uint64_t)n); }  // uniform enough for n << 2^64
};

struct SampleNode {
    std::vector<int32_t> in, out;
};

std::vector<SampleNode> make_sample(int p, int k, int count, uint64_t seed)
{
    SplitMix g{seed};
    std::vector<SampleNode> v(count);
    std::vector<int32_t> perm(p);
    for (auto &nd : v) {
        const int n1 = g.below(k / 2 + 1);
        int n0 = g.below(p / 10 + 1);
        n0 = std::min(n0, p - n1);
        for (int j = 0; j < p; ++j) perm[j] = j;
        for (int r = 0; r < n1 + n0; ++r) std::swap(perm[r], perm[r + g.below(p - r)]);
        nd.in.assign(perm.begin(), perm.begin() + n1);
        nd.out.assign(perm.begin() + n1, perm.begin() + n1 + n0);
        std::sort(nd.in.begin(), nd.in.end());
        std::sort(nd.out.begin(), nd.out.end());
    }
    return v;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// bound every node once; returns the wall time or a negative error code
double run_sample(kbnb_problem *P, std::vector<kbnb_node_desc> &nodes, int cap, int &rc)
{
    std::vector<kbnb_bound_result> out(cap);
    const double t0 = now_s();
    rc = submit_nodes(P, nodes.data(), (int32_t)nodes.size());
    if (rc) return -1.0;
    size_t got = 0;
    while (got < nodes.size()) {
        int32_t n = 0;
        rc = poll_bounds(P, out.data(), cap, &n, nullptr, nullptr, 1000000);
        if (rc < 0) return -1.0;
        if (n == 0 && rc == KBNB_TIMEOUT) continue;
        got += (size_t)n;
    }
    rc = 0;
    return now_s() - t0;
}

// Cache of choices per device and shape bucket.
typedef std::tuple<int, int, int, int, int, int> TuneKey;  // device, log2 n, log2 p, dtype, loss, iteration
std::mutex g_tune_mu;
std::map<TuneKey, kbnb_tune_result> g_tune_cache;

int ceil_log2(int64_t v)
{
    int r = 0;
    while ((int64_t)1 << r < v) ++r;
    return r;
}

}  // namespace

extern "C" int autotune(const kbnb_problem_desc *desc, const kbnb_node_desc *nodes, int32_t count,
                        const kbnb_tune_options *opts, kbnb_tune_result *result, double *rates)
{
    using kbnb::set_error;
    if (!desc || !result) return set_error(KBNB_E_INVALID_ARGUMENT, "NULL argument");
    if (count < 0 || (count > 0 && !nodes)) return set_error(KBNB_E_INVALID_ARGUMENT, "bad node sample");
    kbnb_tune_options o{};
    if (opts) o = *opts;
    static const int32_t dw[] = {64, 128, 256, 512, 1024, 2048};
    static const int32_t dp[] = {4, 8, 16};
    const int32_t *widths = o.widths ? o.widths : dw;
    const int nw = o.widths ? o.n_widths : 6;
    const int32_t *periods = o.periods ? o.periods : dp;
    const int np = o.periods ? o.n_periods : 3;
    if (nw <= 0 || np <= 0) return set_error(KBNB_E_INVALID_ARGUMENT, "no candidates");
    int wmax = 0;
    for (int i = 0; i < nw; ++i) {
        if (widths[i] <= 0 || widths[i] > 4096) return set_error(KBNB_E_INVALID_ARGUMENT, "width %d out of range", widths[i]);
        wmax = std::max(wmax, widths[i]);
    }
    for (int i = 0; i < np; ++i)
        if (periods[i] <= 0 || periods[i] > 1000) return set_error(KBNB_E_INVALID_ARGUMENT, "period %d out of range", periods[i]);
    const int max_it = o.max_iters > 0 ? o.max_iters : 2000;
    const double tol = o.rel_tol > 0 ? o.rel_tol : 1e-6;
    const double tlim = o.time_limit_s > 0 ? o.time_limit_s : 60.0;
    const double tie = o.tie_frac > 0 ? o.tie_frac : 0.03;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const int iter_key = desc->iter_dtype;
    const TuneKey key{dev, ceil_log2(desc->n), ceil_log2(desc->p), desc->x_dtype, desc->loss, iter_key};
    if (!o.refresh) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && (it->second.tile_trials > 0 || !o.tune_tiles)) {
            *result = it->second;
            result->cached = 1;
            result->seconds = 0.0;
            if (rates) std::fill(rates, rates + (size_t)nw * np, 0.0);
            return KBNB_OK;
        }
    }

    // the sample
    std::vector<SampleNode> gen;
    std::vector<kbnb_node_desc> sample;
    if (count > 0) {
        sample.assign(nodes, nodes + count);
    } else {
        const int cnt = o.sample_nodes > 0 ? o.sample_nodes : 2 * wmax;
        gen = make_sample(desc->p, desc->k, cnt, o.seed);
        sample.resize(cnt);
        for (int i = 0; i < cnt; ++i) {
            kbnb_node_desc d{};
            d.n_in = (int32_t)gen[i].in.size();
            d.fixed_in = gen[i].in.data();
            d.n_out = (int32_t)gen[i].out.size();
            d.fixed_out = gen[i].out.data();
            sample[i] = d;
        }
    }
    for (size_t i = 0; i < sample.size(); ++i) {
        sample[i].tag = i;
        sample[i].upper_bound = INFINITY;
        sample[i].rel_tol = tol;
        sample[i].max_iters = max_it;
    }

    if (rates) std::fill(rates, rates + (size_t)nw * np, 0.0);
    const double t_start = now_s();
    int trials = 0;
    std::vector<double> rate((size_t)nw * np, 0.0);
    for (int a = 0; a < nw; ++a) {
        bool over_budget = false;
        for (int b = 0; b < np && !over_budget; ++b) {
            if (now_s() - t_start > tlim) break;
            kbnb_problem_desc d = *desc;
            d.batch_width = widths[a];
            d.cert_period = periods[b];
            kbnb_problem *P = nullptr;
            int rc = create_problem(&d, &P);
            if (rc == KBNB_E_BUDGET_EXCEEDED) { over_budget = true; break; }
            if (rc) return rc;
            // warm-up: a few nodes, so one-time costs are not timed
            std::vector<kbnb_node_desc> warm(sample.begin(), sample.begin() + std::min<size_t>(8, sample.size()));
            run_sample(P, warm, widths[a], rc);
            double dt = rc ? -1.0 : run_sample(P, sample, widths[a], rc);
            destroy_problem(P);
            if (rc) return rc;
            rate[(size_t)a * np + b] = (double)sample.size() / dt;
            ++trials;
        }
    }
    // choice: smallest width whose best rate ties the overall best
    double best = 0.0;
    for (double r : rate) best = std::max(best, r);
    if (!(best > 0.0)) return set_error(KBNB_E_BUDGET_EXCEEDED, "no candidate could be measured");
    int cw = -1, cp = -1;
    int best_w = 1 << 30;
    for (int a = 0; a < nw; ++a) {
        for (int b = 0; b < np; ++b) {
            const double r = rate[(size_t)a * np + b];
            if (r >= (1.0 - tie) * best && widths[a] <= best_w) {
                if (widths[a] < best_w || r > rate[(size_t)cw * np + cp]) {
                    best_w = widths[a];
                    cw = a;
                    cp = b;
                }
            }
        }
    }
    if (rates) std::copy(rate.begin(), rate.end(), rates);
    result->batch_width = widths[cw];
    result->cert_period = periods[cp];
    result->rate = rate[(size_t)cw * np + cp];
    result->trials = trials;
    result->sample_nodes = (int32_t)sample.size();
    result->tile_rows = 0;
    result->split_rows = 0;
    result->cached = 0;
    result->tile_trials = 0;

    // second stage: tile height and split depth at the chosen width and period
    if (o.tune_tiles) {
        kbnb_problem_desc d = *desc;
        d.batch_width = widths[cw];
        d.cert_period = periods[cp];
        d.tile_rows = 0;
        d.split_rows = 0;
        // the rule's resolution, from a problem of the chosen configuration
        kbnb_problem *P = nullptr;
        int rc = create_problem(&d, &P);
        if (rc) return rc;
        int64_t info[11];
        rc = problem_info(P, info, nullptr);
        destroy_problem(P);
        if (rc) return rc;
        const int tr_rule = (int)info[9], sr_rule = (int)info[10];
        const bool streaming = desc->x_dtype == KBNB_DTYPE_BF16 && info[8] != KBNB_ITER_F64;
        const int tiles[4] = {0, streaming ? 64 : 32, streaming ? 128 : 64, streaming ? 256 : 0};
        const int nt = streaming ? 4 : 3;
        const int splits[3] = {0, std::max(64, sr_rule / 2), 2 * sr_rule};
        double best_r = result->rate;  // the rule's rate from the first stage
        int bt = 0, bs = 0, t2 = 0;
        for (int a = 0; a < nt; ++a) {
            for (int b = 0; b < 3; ++b) {
                if (a == 0 && b == 0) continue;  // the first stage measured the rule
                if (a > 0 && tiles[a] == tr_rule) continue;  // the rule under another name
                if (now_s() - t_start > tlim) break;
                d.tile_rows = tiles[a];
                d.split_rows = splits[b];
                P = nullptr;
                rc = create_problem(&d, &P);
                if (rc == KBNB_E_BUDGET_EXCEEDED) continue;
                if (rc) return rc;
                std::vector<kbnb_node_desc> warm(sample.begin(), sample.begin() + std::min<size_t>(8, sample.size()));
                run_sample(P, warm, d.batch_width, rc);
                double dt = rc ? -1.0 : run_sample(P, sample, d.batch_width, rc);
                destroy_problem(P);
                if (rc) return rc;
                const double r = (double)sample.size() / dt;
                ++t2;
                // a candidate must beat the incumbent by more than the tie margin
                if (r > best_r * (1.0 + tie)) {
                    best_r = r;
                    bt = tiles[a];
                    bs = splits[b];
                }
            }
        }
        result->tile_rows = bt;
        result->split_rows = bs;
        result->tile_trials = t2;
        if (bt || bs) result->rate = best_r;
    }
    result->seconds = now_s() - t_start;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = *result;
    }
    return KBNB_OK;
}
