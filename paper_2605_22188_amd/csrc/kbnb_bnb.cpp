// kbnb_bnb.cpp -- best-bound branch and bound on top of submit_nodes /
// poll_bounds (paper Sec. 4.1, Fig. 1; Sec. 4.3).
//
// The host owns the tree: the open-node queue ordered by parent bound (deeper
// first on ties, then first-in), the incumbent and the global bound.  The
// device bounds whole batches: the driver keeps up to two batch widths of
// nodes in flight so finished slots are refilled at once.  For every node
// that survives its bound:
//   - its rounding support (J1 plus the kbar largest free |beta_j|) is
//     re-optimised on the device as the node J1 = support, J0 = complement
//     (that relaxation is exact, its primal value is an attained objective),
//     unless the same support was already evaluated;
//   - a node whose budget cannot bind (kbar = 0 or #free <= kbar) is closed:
//     its relaxation equals the value of its rounding support;
//   - otherwise it branches on the returned index into z_j = 0 and z_j = 1
//     children, both warm-started from the parent iterate (z_j = 0 zeroes
//     beta_j).
// Pruning: bound >= UB - 1e-6 |UB|.  Termination: no open or in-flight node,
// or (UB - global bound) <= rel_gap_tol * |UB|.  The reported lower bound is
// the least bound over every leaf of the explored tree (pruned nodes, closed
// nodes) and every node left open, so it is certified even when pruning used
// the relative slack.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <queue>
#include <set>
#include <string>
#include <vector>

#include "../../include/kbnb.h"

namespace {

struct Open {
    double lb;
    int depth;
    uint64_t seq;
    std::vector<int32_t> in, out;
    std::vector<int32_t> wi;  // warm start, sparse
    std::vector<double> wv;
};

struct OpenCmp {
    bool operator()(const Open *a, const Open *b) const
    {
        if (a->lb != b->lb) return a->lb > b->lb;
        if (a->depth != b->depth) return a->depth < b->depth;
        return a->seq > b->seq;
    }
};

struct Flight {
    bool reopt = false;
    Open *node = nullptr;           // bound node
    std::vector<int32_t> support;   // re-optimisation support
};

}  // namespace

extern "C" int problem_info(kbnb_problem *prob, int64_t *i_out, double *d_out);
namespace kbnb {
int set_error(int code, const char *fmt, ...);
}

extern "C" int branch_and_bound(kbnb_problem *P, const kbnb_bnb_options *opt, kbnb_bnb_result *res)
{
    if (!P) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL problem");
    if (!opt || !res || !res->support)
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "options, result and result->support are required");
    int64_t info[9];
    double dinfo[4];
    int rc = problem_info(P, info, dinfo);
    if (rc) return rc;
    const int p = (int)info[1], k = (int)info[2], m = (int)info[3];
    const double gap_tol = opt->rel_gap_tol > 0 ? opt->rel_gap_tol : 1e-6;
    const double node_tol = opt->node_rel_tol > 0 ? opt->node_rel_tol : 1e-6;
    const double prune_rel = 1e-6;
    const int max_it = opt->max_fista_iters > 0 ? opt->max_fista_iters : 20000;
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };

    std::priority_queue<Open *, std::vector<Open *>, OpenCmp> open;
    std::map<uint64_t, Flight> flight;
    std::multiset<double> flight_lb;
    std::set<std::vector<int32_t>> evaluated;
    uint64_t seq = 0, next_tag = 1;
    double UB = INFINITY;
    std::vector<int32_t> best_support;
    std::vector<double> best_beta(p, 0.0);
    int64_t nodes = 0, updates = 0;
    int status = 0;

    Open *root = new Open();
    root->lb = -INFINITY;
    root->depth = 0;
    root->seq = seq++;
    open.push(root);

    const int cap_flight = 2 * m;
    std::vector<kbnb_node_desc> batch;
    std::vector<std::vector<double>> warm_store;
    std::vector<kbnb_bound_result> out(m);
    std::vector<int32_t> sup((size_t)m * k);
    std::vector<double> betas((size_t)m * p);
    std::vector<int32_t> full_out;
    std::vector<std::vector<int32_t>> outs_store;
    double global_lb = -INFINITY;
    double leaf_lb = INFINITY;  // least bound of the discarded subtrees
    double last_log = 0.0;

    auto prunable = [&](double lb) { return lb >= UB - prune_rel * std::fabs(UB); };

    for (;;) {
        // drop open nodes that the incumbent prunes (the queue is ordered by bound)
        while (!open.empty() && prunable(open.top()->lb)) {
            Open *o = open.top();
            open.pop();
            leaf_lb = std::min(leaf_lb, o->lb);
            delete o;
            // every remaining node has a bound at least as large
            while (!open.empty()) {
                delete open.top();
                open.pop();
            }
        }
        double lb_open = open.empty() ? INFINITY : open.top()->lb;
        double lb_fl = flight_lb.empty() ? INFINITY : *flight_lb.begin();
        global_lb = std::min(lb_open, lb_fl);
        bool reopt_pending = false;
        for (auto &f : flight)
            if (f.second.reopt) { reopt_pending = true; break; }
        if (open.empty() && flight.empty()) break;
        if (std::isfinite(UB) && !reopt_pending && global_lb >= UB - gap_tol * std::fabs(UB)) break;
        if (opt->time_limit_s > 0 && elapsed() > opt->time_limit_s) { status = 1; break; }
        if (opt->max_nodes > 0 && nodes >= opt->max_nodes) { status = 2; break; }
        if (opt->log_every_s > 0 && elapsed() - last_log >= opt->log_every_s) {
            last_log = elapsed();
            fprintf(stderr, "[bnb] %.1fs nodes %lld open %zu in flight %zu UB %.10g LB %.10g\n",
                    last_log, (long long)nodes, open.size(), flight.size(), UB,
                    std::min(global_lb, leaf_lb));
            fflush(stderr);
        }

        // fill the device
        batch.clear();
        warm_store.clear();
        outs_store.clear();
        int room = cap_flight - (int)flight.size();
        while (room > 0 && !open.empty()) {
            Open *o = open.top();
            open.pop();
            kbnb_node_desc d{};
            const uint64_t tag = next_tag++;
            d.tag = tag;
            d.n_in = (int32_t)o->in.size();
            d.fixed_in = o->in.data();
            d.n_out = (int32_t)o->out.size();
            d.fixed_out = o->out.data();
            if (!o->wi.empty()) {
                warm_store.emplace_back(p, 0.0);
                for (size_t r = 0; r < o->wi.size(); ++r) warm_store.back()[o->wi[r]] = o->wv[r];
            }
            d.upper_bound = UB;
            d.rel_tol = node_tol;
            d.max_iters = max_it;
            batch.push_back(d);
            Flight f;
            f.node = o;
            flight[tag] = f;
            flight_lb.insert(o->lb);
            --room;
        }
        // warm-start pointers are set once the storage no longer moves
        {
            size_t wsi = 0;
            for (auto &d : batch) {
                Open *o = flight[d.tag].node;
                if (!o->wi.empty()) d.warm_start = warm_store[wsi++].data();
            }
        }
        if (!batch.empty()) {
            rc = submit_nodes(P, batch.data(), (int32_t)batch.size());
            if (rc) return rc;
        }
        // collect results
        int32_t got = 0;
        rc = poll_bounds(P, out.data(), m, &got, sup.data(), betas.data(), 200000);
        if (rc < 0) return rc;
        std::vector<kbnb_node_desc> reopts;
        std::vector<std::vector<int32_t>> reopt_in, reopt_out;
        for (int r = 0; r < got; ++r) {
            const kbnb_bound_result &br = out[r];
            auto it = flight.find(br.tag);
            if (it == flight.end()) continue;
            Flight f = std::move(it->second);
            flight.erase(it);
            const double *beta = betas.data() + (size_t)r * p;
            if (f.reopt) {
                const double v = br.primal_value;
                if (std::isfinite(v) && v < UB) {
                    UB = v;
                    best_support = f.support;
                    best_beta.assign(beta, beta + p);
                    ++updates;
                }
                continue;
            }
            Open *o = f.node;
            flight_lb.erase(flight_lb.find(o->lb));
            ++nodes;
            const double lb = std::max(br.lower_bound, o->lb);
            if (prunable(lb)) {
                leaf_lb = std::min(leaf_lb, lb);
                delete o;
                continue;
            }
            // rounding support -> re-optimisation
            std::vector<int32_t> S(sup.begin() + (size_t)r * k, sup.begin() + (size_t)r * k + br.support_len);
            if (!S.empty() && evaluated.insert(S).second) {
                reopt_in.push_back(S);
                std::vector<char> ins(p, 0);
                for (int j : S) ins[j] = 1;
                std::vector<int32_t> comp;
                for (int j = 0; j < p; ++j)
                    if (!ins[j]) comp.push_back(j);
                reopt_out.push_back(comp);
            }
            const int kbar = k - (int)o->in.size();
            const int pf = p - (int)o->in.size() - (int)o->out.size();
            const int j = br.branch_index;
            if (kbar <= 0 || pf <= kbar || j < 0) {
                leaf_lb = std::min(leaf_lb, lb);
                delete o;
                continue;
            }
            for (int side = 0; side < 2; ++side) {
                Open *c = new Open();
                c->lb = lb;
                c->depth = o->depth + 1;
                c->seq = seq++;
                c->in = o->in;
                c->out = o->out;
                if (side == 0) c->out.push_back(j);
                else c->in.push_back(j);
                std::sort(c->in.begin(), c->in.end());
                std::sort(c->out.begin(), c->out.end());
                for (int q = 0; q < p; ++q) {
                    if (beta[q] != 0.0 && !(side == 0 && q == j)) {
                        c->wi.push_back(q);
                        c->wv.push_back(beta[q]);
                    }
                }
                open.push(c);
            }
            delete o;
        }
        if (!reopt_in.empty()) {
            for (size_t r = 0; r < reopt_in.size(); ++r) {
                kbnb_node_desc d{};
                const uint64_t tag = next_tag++;
                d.tag = tag;
                d.n_in = (int32_t)reopt_in[r].size();
                d.fixed_in = reopt_in[r].data();
                d.n_out = (int32_t)reopt_out[r].size();
                d.fixed_out = reopt_out[r].data();
                d.upper_bound = INFINITY;
                d.rel_tol = std::min(1e-7, 0.1 * node_tol);
                d.max_iters = max_it;
                reopts.push_back(d);
                Flight f;
                f.reopt = true;
                f.support = reopt_in[r];
                flight[tag] = f;
            }
            rc = submit_nodes(P, reopts.data(), (int32_t)reopts.size());
            if (rc) return rc;
        }
    }
    // drain in-flight work so the handle is reusable
    while (!flight.empty()) {
        int32_t got = 0;
        rc = poll_bounds(P, out.data(), m, &got, sup.data(), betas.data(), 200000);
        if (rc < 0) return rc;
        for (int r = 0; r < got; ++r) {
            auto it = flight.find(out[r].tag);
            if (it == flight.end()) continue;
            if (it->second.reopt) {
                const double v = out[r].primal_value;
                if (std::isfinite(v) && v < UB) {
                    UB = v;
                    best_support = it->second.support;
                    best_beta.assign(betas.data() + (size_t)r * p, betas.data() + (size_t)(r + 1) * p);
                    ++updates;
                }
            } else {
                // unexplored: its parent's bound still holds for its subtree
                global_lb = std::min(global_lb, it->second.node->lb);
                delete it->second.node;
            }
            flight.erase(it);
        }
        if (got == 0 && rc == KBNB_TIMEOUT) {
            // nothing is progressing: should not happen; avoid spinning forever
            break;
        }
    }
    while (!open.empty()) {
        global_lb = std::min(global_lb, open.top()->lb);
        delete open.top();
        open.pop();
    }
    res->objective = UB;
    res->lower_bound = std::min(std::min(global_lb, leaf_lb), UB);
    res->rel_gap = std::isfinite(UB) ? (UB - res->lower_bound) / std::max(std::fabs(UB), 1e-12) : INFINITY;
    res->nodes = nodes;
    res->status = status;
    res->support_len = (int32_t)best_support.size();
    for (int r = 0; r < k; ++r) res->support[r] = r < (int)best_support.size() ? best_support[r] : -1;
    if (res->beta) memcpy(res->beta, best_beta.data(), sizeof(double) * p);
    res->incumbent_updates = updates;
    res->seconds = elapsed();
    return KBNB_OK;
}
