// kbnb_pool.cpp -- compact storage of a support-level Rashomon set (paper
// App. "compact Rashomon pool storage", Fig. of the support trie).
//
// A pool holds N records.  Record m stores a support as the path from the
// root of a prefix trie to its end node: trie node v (v >= 1) has a parent
// p(v) and an edge label a(v) (a feature index); the root is node 0.  Two
// records whose insertion sequences share a prefix share that prefix's
// nodes.  The record itself is (end node, value Phi_m); its |S_m|
// coefficients, ordered like the labels of its path from the root, sit in
// one flat vector c at offset o_{m}: o_0 = 0, o_m = o_{m-1} + |S_m|.
// Host-only code: no call here touches the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/kbnb.h"

namespace kbnb {
int set_error(int code, const char *fmt, ...);
}

struct kbnb_pool {
    std::vector<int32_t> parent{-1};  // p(v); the root's is -1
    std::vector<int32_t> label{-1};   // a(v); the root's is -1
    std::vector<int32_t> child{-1};   // first child (search links, not exported)
    std::vector<int32_t> sibling{-1};
    std::vector<int32_t> end_node;    // record m -> its trie node
    std::vector<double> value;        // Phi_m
    std::vector<int64_t> offset{0};   // o_0 .. o_N
    std::vector<double> coef;         // c

    int32_t walk(const int32_t *seq, int32_t len)
    {
        int32_t cur = 0;
        for (int32_t r = 0; r < len; ++r) {
            int32_t c = child[(size_t)cur];
            while (c >= 0 && label[(size_t)c] != seq[r]) c = sibling[(size_t)c];
            if (c < 0) {
                c = (int32_t)label.size();
                parent.push_back(cur);
                label.push_back(seq[r]);
                child.push_back(-1);
                sibling.push_back(child[(size_t)cur]);
                child[(size_t)cur] = c;
            }
            cur = c;
        }
        return cur;
    }
    // labels of record m's path, root first
    std::vector<int32_t> path(int64_t m) const
    {
        std::vector<int32_t> s;
        for (int32_t v = end_node[(size_t)m]; v > 0; v = parent[(size_t)v]) s.push_back(label[(size_t)v]);
        std::reverse(s.begin(), s.end());
        return s;
    }
};

namespace {
std::mutex g_mu;
std::map<const kbnb_problem *, std::unique_ptr<kbnb_pool>> g_sets;  // last collected set per problem
}  // namespace

namespace kbnb {
// pool helpers for branch_and_bound
kbnb_pool *pool_new() { return new kbnb_pool(); }
void pool_append(kbnb_pool *pl, const std::vector<int32_t> &seq, const double *coef, double v)
{
    pl->end_node.push_back(pl->walk(seq.data(), (int32_t)seq.size()));
    pl->value.push_back(v);
    for (size_t r = 0; r < seq.size(); ++r) pl->coef.push_back(coef ? coef[r] : 0.0);
    pl->offset.push_back((int64_t)pl->coef.size());
}
void store_rashomon(const kbnb_problem *P, kbnb_pool *pl)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_sets[P].reset(pl);
}
void drop_rashomon(const kbnb_problem *P)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_sets.erase(P);
}
}  // namespace kbnb

extern "C" int pool_create(kbnb_pool **out)
{
    if (!out) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "out is required");
    *out = new kbnb_pool();
    return KBNB_OK;
}

extern "C" int pool_destroy(kbnb_pool *pool)
{
    delete pool;
    return KBNB_OK;
}

extern "C" int pool_add(kbnb_pool *pool, const int32_t *seq, int32_t len, const double *coef, double value)
{
    if (!pool) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL pool");
    if (len < 0 || (len > 0 && !seq)) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "bad sequence");
    for (int32_t r = 0; r < len; ++r) {
        if (seq[r] < 0) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "negative feature index %d", seq[r]);
        for (int32_t q = 0; q < r; ++q)
            if (seq[q] == seq[r])
                return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "feature %d repeated in one support", seq[r]);
    }
    kbnb::pool_append(pool, std::vector<int32_t>(seq, seq + len), coef, value);
    return KBNB_OK;
}

extern "C" int pool_info(const kbnb_pool *pool, int64_t *records, int64_t *trie_nodes, int64_t *coefs)
{
    if (!pool) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL pool");
    if (records) *records = (int64_t)pool->value.size();
    if (trie_nodes) *trie_nodes = (int64_t)pool->label.size();
    if (coefs) *coefs = (int64_t)pool->coef.size();
    return KBNB_OK;
}

extern "C" int pool_export(const kbnb_pool *pool, int32_t *parent, int32_t *label, int32_t *end_node,
                           double *values, int64_t *offsets, double *coef)
{
    if (!pool) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL pool");
    const size_t T = pool->label.size(), N = pool->value.size();
    if (parent) memcpy(parent, pool->parent.data(), T * sizeof(int32_t));
    if (label) memcpy(label, pool->label.data(), T * sizeof(int32_t));
    if (end_node) memcpy(end_node, pool->end_node.data(), N * sizeof(int32_t));
    if (values) memcpy(values, pool->value.data(), N * sizeof(double));
    if (offsets) memcpy(offsets, pool->offset.data(), (N + 1) * sizeof(int64_t));
    if (coef) memcpy(coef, pool->coef.data(), pool->coef.size() * sizeof(double));
    return KBNB_OK;
}

extern "C" int pool_record(const kbnb_pool *pool, int64_t m, int32_t *seq, int32_t *len, double *coef,
                           double *value)
{
    if (!pool) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL pool");
    if (m < 0 || m >= (int64_t)pool->value.size())
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "no record %lld", (long long)m);
    const std::vector<int32_t> s = pool->path(m);
    if (len) *len = (int32_t)s.size();
    if (seq) std::copy(s.begin(), s.end(), seq);
    if (coef)
        std::copy(pool->coef.begin() + pool->offset[(size_t)m], pool->coef.begin() + pool->offset[(size_t)m + 1],
                  coef);
    if (value) *value = pool->value[(size_t)m];
    return KBNB_OK;
}

extern "C" int pool_summary(const kbnb_pool *pool, int32_t p, const double *reliance, double *out)
{
    if (!pool) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL pool");
    if (p <= 0 || !out) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "p > 0 and out are required");
    const size_t N = pool->value.size(), P = (size_t)p;
    for (size_t v = 1; v < pool->label.size(); ++v)
        if (pool->label[v] >= p)
            return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "feature %d outside [0, %d)", pool->label[v], p);
    double *freq = out, *mean = out + P, *amean = out + 2 * P, *pos = out + 3 * P, *cmin = out + 4 * P,
           *cmax = out + 5 * P, *rmin = out + 6 * P, *rmax = out + 7 * P, *rmean = out + 8 * P;
    std::fill(out, out + 9 * P, 0.0);
    if (N == 0) return KBNB_OK;
    // a feature absent from a record has coefficient 0 and reliance 0 there
    std::vector<int64_t> cnt(P, 0);
    for (size_t m = 0; m < N; ++m) {
        const std::vector<int32_t> s = pool->path((int64_t)m);
        const int64_t o = pool->offset[m];
        for (size_t r = 0; r < s.size(); ++r) {
            const size_t j = (size_t)s[r];
            const double c = pool->coef[(size_t)o + r];
            const double rv = reliance ? reliance[(size_t)o + r] : 0.0;
            if (cnt[j] == 0) {
                cmin[j] = cmax[j] = c;
                rmin[j] = rmax[j] = rv;
            } else {
                cmin[j] = std::min(cmin[j], c);
                cmax[j] = std::max(cmax[j], c);
                rmin[j] = std::min(rmin[j], rv);
                rmax[j] = std::max(rmax[j], rv);
            }
            ++cnt[j];
            mean[j] += c;
            amean[j] += std::fabs(c);
            pos[j] += c > 0 ? 1.0 : 0.0;
            rmean[j] += rv;
        }
    }
    for (size_t j = 0; j < P; ++j) {
        if (cnt[j] < (int64_t)N) {  // some records leave j out: their 0 joins the ranges
            cmin[j] = std::min(cmin[j], 0.0);
            cmax[j] = std::max(cmax[j], 0.0);
            rmin[j] = std::min(rmin[j], 0.0);
            rmax[j] = std::max(rmax[j], 0.0);
        }
        freq[j] = (double)cnt[j] / (double)N;
        mean[j] /= (double)N;
        amean[j] /= (double)N;
        pos[j] /= (double)N;
        rmean[j] /= (double)N;
    }
    if (!reliance)
        for (size_t j = 0; j < P; ++j) rmin[j] = rmax[j] = rmean[j] = 0.0;
    return KBNB_OK;
}

extern "C" int rashomon_pool(kbnb_problem *P, kbnb_pool **out)
{
    if (!P) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL problem");
    if (!out) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "out is required");
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_sets.find(P);
    if (it == g_sets.end()) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "no Rashomon set collected");
    *out = new kbnb_pool(*it->second);
    return KBNB_OK;
}

extern "C" int problem_info(kbnb_problem *prob, int64_t *i_out, double *d_out);

extern "C" int rashomon_entry(kbnb_problem *P, int64_t i, int32_t *support, int32_t *support_len,
                              double *beta, double *value)
{
    if (!P) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL problem");
    if (!support || !support_len || !value)
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "support, support_len and value are required");
    int64_t info[11];
    double dinfo[4];
    int rc = problem_info(P, info, dinfo);
    if (rc) return rc;
    const int p = (int)info[1], k = (int)info[2];
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_sets.find(P);
    if (it == g_sets.end() || i < 0 || i >= (int64_t)it->second->value.size())
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "no Rashomon entry %lld", (long long)i);
    const kbnb_pool &pl = *it->second;
    const std::vector<int32_t> s = pl.path(i);
    const double *c = pl.coef.data() + pl.offset[(size_t)i];
    std::vector<int32_t> sorted(s);
    std::sort(sorted.begin(), sorted.end());
    for (int r = 0; r < k; ++r) support[r] = r < (int)sorted.size() ? sorted[r] : -1;
    *support_len = (int32_t)s.size();
    *value = pl.value[(size_t)i];
    if (beta) {
        std::fill(beta, beta + p, 0.0);
        for (size_t r = 0; r < s.size(); ++r) beta[s[r]] = c[r];
    }
    return KBNB_OK;
}
