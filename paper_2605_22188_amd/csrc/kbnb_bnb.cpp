// kbnb_bnb.cpp -- best-bound branch and bound on top of submit_nodes /
// poll_bounds (paper Sec. 4.1, Fig. 1; Sec. 4.3), and the support-level
// Rashomon-set collection on the same tree (Sec. 4.5).
//
// The host owns the tree: the open-node queue (by parent bound, deeper first
// on ties, then first-in; or depth first on request), the incumbent and the
// global bound.  The
// device bounds whole batches: the driver keeps up to two batch widths of
// nodes in flight so finished slots are refilled at once.  For every node
// that survives its bound:
//   - its rounding support (J1 plus the kbar largest free |beta_j|) is
//     re-optimised on the device as the node J1 = support, J0 = complement
//     (that relaxation is exact, its primal value is an attained objective),
//     unless the same support was already evaluated;
//   - optimal-support mode: a node whose budget cannot bind (kbar = 0 or
//     #free <= kbar) is closed: its relaxation equals the value of its
//     rounding support;
//   - Rashomon mode: a node is a leaf only when no indicator is undecided
//     (kbar = 0 or nothing free); its support J1 is evaluated like a
//     rounding support.  Every support evaluated within the threshold is
//     recorded;
//   - otherwise it branches on the returned index (the first free index if
//     every free coordinate is zero) into z_j = 0 and z_j = 1 children, both
//     warm-started from the parent iterate (z_j = 0 zeroes beta_j).
// Pruning: optimal-support mode, bound >= UB - 1e-6 |UB|; Rashomon mode,
// bound > tau = min((1 + eps) UB, v_(N)), v_(N) the N-th best recorded value.
// Termination: no open or in-flight node, or (optimal-support mode) (UB -
// global bound) <= rel_gap_tol * |UB|.  The reported lower bound is the
// least bound over every leaf of the explored tree (pruned nodes, closed
// nodes) and every node left open, so it is certified even when pruning used
// the relative slack.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <queue>
#include <set>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/kbnb.h"

namespace {

// Certificate of a bound (audit mode): the node (J1 = in, J0 = out) whose
// dual function was evaluated, and the iterate beta whose dual point
// zeta = -l'(X beta) gave the value `bound`.  A node's bound may be its own
// certificate or one inherited from an ancestor (whose node contains it).
struct Cert {
    std::vector<int32_t> in, out;
    std::vector<double> beta;
    double bound;
};
typedef std::shared_ptr<const Cert> CertPtr;

struct WarmStart {
    std::vector<int32_t> idx;
    std::vector<double> val;
};

struct Open {
    double lb;
    int depth;
    uint64_t seq;
    std::vector<int32_t> in, out;
    // warm start: the parent's iterate (sparse, shared by both children; the
    // engine ignores its entries on J0, so the z_j = 0 child starts from it
    // with beta_j = 0)
    std::shared_ptr<const WarmStart> warm;
    CertPtr cert;             // audit mode: the certificate of lb (null at the root)
};

// Queue entry: the ordering key kept beside the node, so heap operations
// compare entries without touching the nodes.  Order: best bound (smaller
// bound, then deeper, then first in), or depth first (deeper, then smaller
// bound, then first in).
struct OpenRef {
    double lb;
    int depth;
    uint64_t seq;
    Open *node;
};
struct OpenCmp {
    bool dfs = false;
    bool operator()(const OpenRef &a, const OpenRef &b) const
    {
        if (dfs && a.depth != b.depth) return a.depth < b.depth;
        if (a.lb != b.lb) return a.lb > b.lb;
        if (a.depth != b.depth) return a.depth < b.depth;
        return a.seq > b.seq;
    }
};

enum FlightKind { FL_NODE, FL_SUPPORT };

struct Flight {
    FlightKind kind = FL_NODE;
    Open *node = nullptr;           // bound node
    std::vector<int32_t> support;   // evaluated support (ascending)
};

struct Candidate {
    double value;
    std::vector<double> beta;
};

// hash of an index sequence (supports as keys of the host's lookup tables)
struct SeqHash {
    size_t operator()(const std::vector<int32_t> &v) const
    {
        uint64_t h = 0x9E3779B97F4A7C15ull ^ v.size();
        for (int32_t x : v) {
            h ^= (uint64_t)(uint32_t)x + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
            h *= 0xBF58476D1CE4E5B9ull;
        }
        return (size_t)(h ^ (h >> 31));
    }
};
template <typename V> using SeqMap = std::unordered_map<std::vector<int32_t>, V, SeqHash>;
using SeqSet = std::unordered_set<std::vector<int32_t>, SeqHash>;

}  // namespace

namespace kbnb {
// Leaves of the last audited search per problem (audit mode).  A leaf is a
// subtree the search discarded, with the bound it used for it and that
// bound's certificate.
struct AuditLeaf {
    int32_t kind;  // 0 pruned, 1 closed, 2 Rashomon leaf (its support's bound), 3 left unexplored
    std::vector<int32_t> in, out;
    double bound;
    CertPtr cert;
};
static std::mutex g_audit_mu;
static std::map<const kbnb_problem *, std::shared_ptr<std::vector<AuditLeaf>>> g_audit;
void drop_audit(const kbnb_problem *P)
{
    std::lock_guard<std::mutex> g(g_audit_mu);
    g_audit.erase(P);
}
}  // namespace kbnb

extern "C" int problem_info(kbnb_problem *prob, int64_t *i_out, double *d_out);
namespace kbnb {
bool outstanding(kbnb_problem *P);
int poll_with_lb_beta(kbnb_problem *P, kbnb_bound_result *out, int cap, int *n_out, int32_t *supports,
                      double *betas, double *betas_lb, int timeout_us);
void keep_lb_beta(kbnb_problem *P, bool on);
int set_error(int code, const char *fmt, ...);
// the collected set's storage (kbnb_pool.cpp)
kbnb_pool *pool_new();
void pool_append(kbnb_pool *pl, const std::vector<int32_t> &seq, const double *coef, double v);
void store_rashomon(const kbnb_problem *P, kbnb_pool *pl);
// batched support re-optimisation on the device (kbnb_engine.hip)
int eval_supports_launch(kbnb_problem *P, const int32_t *lab, const int64_t *off, int count, int maxlen,
                         const double *warm, double tol, int max_iter);
int eval_supports_collect(kbnb_problem *P, double *values, double *lower, double *coefs, int32_t *status,
                          int32_t *iters, double *coefs_lb);
bool eval_supports_ready(kbnb_problem *P);
int support_groups(kbnb_problem *P, int count, int maxlen);
}  // namespace kbnb

extern "C" int branch_and_bound(kbnb_problem *P, const kbnb_bnb_options *opt, kbnb_bnb_result *res)
{
    if (!P) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL problem");
    if (!opt || !res || !res->support)
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "options, result and result->support are required");
    const bool rs = opt->rashomon != 0;
    if (rs && !(opt->rashomon_eps >= 0 && std::isfinite(opt->rashomon_eps)))
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "rashomon_eps must be finite and >= 0");
    if (rs && opt->rashomon_n < 0) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "rashomon_n must be >= 0");
    int64_t info[11];
    double dinfo[4];
    int rc = problem_info(P, info, dinfo);
    if (rc) return rc;
    // every result the loop polls must be one of its own nodes
    if (kbnb::outstanding(P))
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT,
                               "the problem has nodes queued, running or unpolled; poll or cancel them first");
    const int p = (int)info[1], k = (int)info[2], m = (int)info[3];
    const double gap_tol = opt->rel_gap_tol > 0 ? opt->rel_gap_tol : 1e-6;
    const double node_tol = opt->node_rel_tol > 0 ? opt->node_rel_tol : 1e-6;
    const double support_tol = std::min(1e-7, 0.1 * node_tol);
    const double prune_rel = 1e-6;
    const int max_it = opt->max_fista_iters > 0 ? opt->max_fista_iters : 20000;
    const double eps = rs ? opt->rashomon_eps : 0.0;
    const int64_t capN = rs ? opt->rashomon_n : 0;
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };

    if (opt->node_order != 0 && opt->node_order != 1)
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "node_order must be 0 or 1");
    if (opt->support_path < 0 || opt->support_path > 2)
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "support_path must be 0, 1 or 2");
    const bool dfs = opt->node_order == 1;
    const bool audit = opt->audit != 0;
    auto leaves = std::make_shared<std::vector<kbnb::AuditLeaf>>();
    SeqMap<CertPtr> support_cert;  // audit: certificate of each support's bound
    auto complement = [&](const std::vector<int32_t> &S) {
        std::vector<char> ins((size_t)p, 0);
        for (int32_t j : S) ins[(size_t)j] = 1;
        std::vector<int32_t> c;
        for (int j = 0; j < p; ++j)
            if (!ins[(size_t)j]) c.push_back(j);
        return c;
    };
    auto add_leaf = [&](int kind, const std::vector<int32_t> &in, const std::vector<int32_t> &out, double bound,
                        const CertPtr &cert) {
        if (audit) leaves->push_back(kbnb::AuditLeaf{kind, in, out, bound, cert});
    };
    std::priority_queue<OpenRef, std::vector<OpenRef>, OpenCmp> open(OpenCmp{dfs});
    // bounds of the open nodes, kept in depth-first order only: in best-bound
    // order the least bound is the queue's top
    std::multiset<double> open_lbs;
    auto push_open = [&](Open *o) {
        if (dfs) open_lbs.insert(o->lb);
        open.push(OpenRef{o->lb, o->depth, o->seq, o});
    };
    auto pop_open = [&]() {
        Open *o = open.top().node;
        open.pop();
        if (dfs) open_lbs.erase(open_lbs.find(o->lb));
        return o;
    };
    auto least_open = [&]() {
        if (open.empty()) return (double)INFINITY;
        return dfs ? *open_lbs.begin() : open.top().lb;
    };
    std::unordered_map<uint64_t, Flight> flight;
    flight.reserve((size_t)4 * m);
    std::multiset<double> flight_lb;
    SeqSet evaluated;             // supports submitted or known
    SeqMap<Candidate> recorded;   // Rashomon mode: within the threshold when found
    // the capN smallest recorded values (a max-heap: its top is the N-th best
    // once it holds capN of them)
    std::priority_queue<double> best_vals;
    // Rashomon leaves: a leaf's certified bound is its support's evaluated
    // bound; leaves whose support is still being evaluated wait for it
    // (with their parent's bound, which holds meanwhile)
    SeqMap<double> support_lb;
    SeqMap<std::pair<double, CertPtr>> leaf_waiting;
    uint64_t seq = 0, next_tag = 1;
    double UB = INFINITY;
    std::vector<int32_t> best_support;
    std::vector<double> best_beta(p, 0.0);
    int64_t nodes = 0, updates = 0;
    int status = 0;

    // Rashomon threshold: (1 + eps) UB, capped by the N-th best recorded value
    auto tau = [&]() {
        const double t = (1.0 + eps) * UB;
        if (capN > 0 && (int64_t)best_vals.size() >= capN) return std::min(t, best_vals.top());
        return t;
    };
    auto prunable = [&](double lb) { return rs ? lb > tau() : lb >= UB - prune_rel * std::fabs(UB); };
    auto is_leaf = [&](const Open *o) {
        const int kbar = k - (int)o->in.size();
        const int pf = p - (int)o->in.size() - (int)o->out.size();
        return kbar <= 0 || pf == 0;
    };
    double leaf_lb = INFINITY;  // least bound of the discarded subtrees
    // evaluated support S: value v (attained at beta) and certified bound lb
    // beta_lb (audit mode, nullable): the coefficients whose dual point gave lb
    auto take_support = [&](const std::vector<int32_t> &S, double v, double lb, const double *beta,
                            const double *beta_lb) {
        support_lb[S] = lb;
        CertPtr sc;
        if (audit && beta_lb) {
            sc = std::make_shared<const Cert>(Cert{S, complement(S), std::vector<double>(beta_lb, beta_lb + p), lb});
            support_cert[S] = sc;
        }
        auto w = leaf_waiting.find(S);
        if (w != leaf_waiting.end()) {
            leaf_lb = std::min(leaf_lb, lb);
            add_leaf(2, S, complement(S), lb, sc);
            leaf_waiting.erase(w);
        }
        if (std::isfinite(v) && v < UB) {
            UB = v;
            best_support = S;
            best_beta.assign(beta, beta + p);
            ++updates;
        }
        if (rs && std::isfinite(v) && v <= tau() && !recorded.count(S)) {
            recorded[S] = Candidate{v, std::vector<double>(beta, beta + p)};
            if (capN > 0) {
                if ((int64_t)best_vals.size() < capN) {
                    best_vals.push(v);
                } else if (v < best_vals.top()) {
                    best_vals.pop();
                    best_vals.push(v);
                }
            }
        }
    };

    Open *root = new Open();
    root->lb = -INFINITY;
    root->depth = 0;
    root->seq = seq++;
    push_open(root);

    const int cap_flight = 2 * m;
    std::vector<kbnb_node_desc> batch;
    std::vector<std::vector<int32_t>> set_store;  // index lists of support evaluations
    std::vector<kbnb_bound_result> out(m);
    std::vector<int32_t> sup((size_t)m * k);
    std::vector<double> betas((size_t)m * p);
    std::vector<double> betas_lb(audit ? (size_t)m * p : 0);
    if (audit) kbnb::keep_lb_beta(P, true);
    auto poll = [&](int32_t *got, int timeout_us) {
        return audit ? kbnb::poll_with_lb_beta(P, out.data(), m, got, sup.data(), betas.data(), betas_lb.data(),
                                               timeout_us)
                     : poll_bounds(P, out.data(), m, got, sup.data(), betas.data(), timeout_us);
    };
    double global_lb = -INFINITY;
    double last_log = 0.0;
    double t_poll = 0, t_flush = 0, t_fill = 0, t_res = 0;  // host time split (progress lines)

    // Support evaluations: with k <= 64 they are batched into the dedicated
    // re-optimisation kernel (one batch on the device at a time, beside the
    // node rounds); otherwise each is the node J1 = S, J0 = complement.  On
    // tall instances the kernel needs a support's rows split over several
    // workgroups to keep up with the batched node contractions: without
    // that split (a device that cannot hold two workgroups per support of a
    // batch of 16) the automatic choice is the node path there.
    bool dev_reopt = k <= 64 && opt->support_path != 2;
    if (dev_reopt && opt->support_path == 0 && info[0] > 32768) dev_reopt = kbnb::support_groups(P, 16, k) >= 2;
    // One batch of support evaluations is on the device at a time: each pass
    // of the loop collects the batch launched in the previous pass (it ran
    // while the host filled and processed nodes) and launches the pending
    // supports.
    std::vector<std::vector<int32_t>> pending, inflight;
    std::vector<int32_t> in_lab;   // inputs of the batch in flight, alive until collected
    std::vector<int64_t> in_off;
    auto collect_supports = [&]() -> int {
        if (inflight.empty()) return 0;
        const size_t cnt = inflight.size();
        std::vector<double> val(cnt), low(cnt), coef(std::max<size_t>(in_lab.size(), 1));
        std::vector<double> coef_lb(audit ? coef.size() : 0);
        int erc = kbnb::eval_supports_collect(P, val.data(), low.data(), coef.data(), nullptr, nullptr,
                                              audit ? coef_lb.data() : nullptr);
        if (erc) return erc;
        std::vector<double> dense, dense_lb;
        for (size_t i = 0; i < cnt; ++i) {
            const std::vector<int32_t> &S = inflight[i];
            const double v = val[i];
            // a dense beta only for a support that is kept
            const bool keep = std::isfinite(v) && (v < UB || (rs && v <= tau() && !recorded.count(S)));
            if (keep) {
                dense.assign(p, 0.0);
                for (size_t r = 0; r < S.size(); ++r) dense[(size_t)S[r]] = coef[(size_t)in_off[i] + r];
            }
            if (audit) {
                dense_lb.assign(p, 0.0);
                for (size_t r = 0; r < S.size(); ++r) dense_lb[(size_t)S[r]] = coef_lb[(size_t)in_off[i] + r];
            }
            take_support(S, v, low[i], keep ? dense.data() : nullptr, audit ? dense_lb.data() : nullptr);
        }
        inflight.clear();
        return 0;
    };
    auto launch_supports = [&]() -> int {
        if (pending.empty() || !inflight.empty()) return 0;
        in_lab.clear();
        in_off.assign(1, 0);
        int maxlen = 0;
        for (const auto &S : pending) {
            in_lab.insert(in_lab.end(), S.begin(), S.end());
            in_off.push_back((int64_t)in_lab.size());
            maxlen = std::max(maxlen, (int)S.size());
        }
        int erc = kbnb::eval_supports_launch(P, in_lab.data(), in_off.data(), (int)pending.size(), maxlen, nullptr,
                                             support_tol, max_it);
        if (erc) return erc;
        inflight.swap(pending);
        pending.clear();
        return 0;
    };
    // collect the batch in flight and launch the pending one
    auto cycle_supports = [&]() -> int {
        // the batch in flight is collected once it has finished: the loop
        // keeps bounding nodes meanwhile instead of waiting for it
        if (!inflight.empty() && !kbnb::eval_supports_ready(P)) return 0;
        int erc = collect_supports();
        return erc ? erc : launch_supports();
    };
    // everything evaluated (blocking)
    auto flush_supports = [&]() -> int {
        int erc = collect_supports();  // waits for the batch in flight
        if (!erc) erc = launch_supports();
        return erc ? erc : collect_supports();
    };
    // a support evaluation: the node J1 = S, J0 = complement
    auto support_desc = [&](const std::vector<int32_t> &S, std::vector<kbnb_node_desc> &dst) {
        if (dev_reopt) {
            pending.push_back(S);
            evaluated.insert(S);
            return;
        }
        std::vector<char> ins(p, 0);
        for (int j : S) ins[j] = 1;
        std::vector<int32_t> comp;
        for (int j = 0; j < p; ++j)
            if (!ins[j]) comp.push_back(j);
        set_store.push_back(S);
        set_store.push_back(std::move(comp));
        kbnb_node_desc d{};
        const uint64_t tag = next_tag++;
        d.tag = tag;
        d.upper_bound = INFINITY;
        d.rel_tol = support_tol;
        d.max_iters = max_it;
        dst.push_back(d);
        Flight f;
        f.kind = FL_SUPPORT;
        f.support = S;
        flight[tag] = f;
        evaluated.insert(S);
    };
    // the index pointers of support evaluations, once set_store no longer moves
    auto bind_sets = [&](std::vector<kbnb_node_desc> &v) {
        size_t si = 0;
        for (auto &d : v) {
            if (flight[d.tag].kind != FL_SUPPORT) continue;
            const std::vector<int32_t> &in = set_store[si++];
            const std::vector<int32_t> &ou = set_store[si++];
            d.n_in = (int32_t)in.size();
            d.fixed_in = in.data();
            d.n_out = (int32_t)ou.size();
            d.fixed_out = ou.data();
        }
    };

    for (;;) {
        // drop open nodes that the incumbent prunes: when the least open
        // bound is prunable, every open node is
        if (!open.empty() && prunable(least_open())) {
            leaf_lb = std::min(leaf_lb, least_open());
            while (!open.empty()) {
                Open *o = pop_open();
                add_leaf(0, o->in, o->out, o->lb, o->cert);
                delete o;
            }
        }
        double lb_open = least_open();
        double lb_fl = flight_lb.empty() ? INFINITY : *flight_lb.begin();
        global_lb = std::min(lb_open, lb_fl);
        const bool batch_pending = !pending.empty() || !inflight.empty();
        bool support_pending = batch_pending;
        for (auto &f : flight)
            if (f.second.kind == FL_SUPPORT) { support_pending = true; break; }
        const bool bound_met = !rs && std::isfinite(UB) && global_lb >= UB - gap_tol * std::fabs(UB);
        if ((open.empty() && flight.empty()) || (bound_met && batch_pending)) {
            // nothing else to wait for: settle the support evaluations first
            if (!batch_pending) break;
            double tm0 = elapsed();
            rc = flush_supports();
            t_flush += elapsed() - tm0;
            if (rc) break;
            continue;
        }
        if (bound_met && !support_pending) break;
        if (opt->time_limit_s > 0 && elapsed() > opt->time_limit_s) { status = 1; break; }
        if (opt->max_nodes > 0 && nodes >= opt->max_nodes) { status = 2; break; }
        if (opt->log_every_s > 0 && elapsed() - last_log >= opt->log_every_s) {
            last_log = elapsed();
            fprintf(stderr,
                    "[bnb] %.1fs nodes %lld open %zu in flight %zu UB %.10g LB %.10g%s "
                    "(host s: poll %.2f supports %.2f fill %.2f results %.2f)\n",
                    last_log, (long long)nodes, open.size(), flight.size(), UB, std::min(global_lb, leaf_lb),
                    rs ? " (collecting)" : "", t_poll, t_flush, t_fill, t_res);
            fflush(stderr);
        }

        // fill the device
        double tm = elapsed();
        batch.clear();
        set_store.clear();
        int room = cap_flight - (int)flight.size();
        while (room > 0 && !open.empty()) {
            Open *o = pop_open();
            if (prunable(o->lb)) {  // depth first: pruned at the pop
                leaf_lb = std::min(leaf_lb, o->lb);
                add_leaf(0, o->in, o->out, o->lb, o->cert);
                delete o;
                continue;
            }
            if (rs && is_leaf(o)) {
                // Rashomon leaf: its support J1 is evaluated (once)
                auto known = support_lb.find(o->in);
                if (known != support_lb.end()) {
                    leaf_lb = std::min(leaf_lb, known->second);
                    if (audit) {
                        auto sc = support_cert.find(o->in);
                        add_leaf(2, o->in, complement(o->in), known->second,
                                 sc == support_cert.end() ? nullptr : sc->second);
                    }
                } else {
                    auto w = leaf_waiting.find(o->in);
                    if (w == leaf_waiting.end()) leaf_waiting[o->in] = {o->lb, o->cert};
                    else if (o->lb < w->second.first) w->second = {o->lb, o->cert};
                    if (!evaluated.count(o->in)) {
                        support_desc(o->in, batch);
                        --room;
                    }
                }
                delete o;
                continue;
            }
            kbnb_node_desc d{};
            const uint64_t tag = next_tag++;
            d.tag = tag;
            d.n_in = (int32_t)o->in.size();
            d.fixed_in = o->in.data();
            d.n_out = (int32_t)o->out.size();
            d.fixed_out = o->out.data();
            // the engine stops a node at bound >= ub - 1e-6 |ub|; in Rashomon
            // mode that must imply bound > tau
            d.upper_bound = rs ? tau() * (1.0 + 4e-6) : UB;
            d.rel_tol = node_tol;
            d.max_iters = max_it;
            // a node that will be branched stops as soon as it cannot be
            // pruned; one the driver closes (integral: kbar <= 0 or every free
            // coordinate fits the budget) keeps its tight bound
            {
                const int kb = k - (int)o->in.size();
                const int pf = p - (int)o->in.size() - (int)o->out.size();
                d.stop_unprunable = (rs || (kb > 0 && pf > kb)) ? 1 : 0;
            }
            batch.push_back(d);
            Flight f;
            f.node = o;
            flight[tag] = f;
            flight_lb.insert(o->lb);
            --room;
        }
        t_fill += elapsed() - tm;
        tm = elapsed();
        // sparse warm starts, and the index pointers of support evaluations
        // once set_store no longer moves
        {
            for (auto &d : batch) {
                Flight &f = flight[d.tag];
                if (f.kind == FL_NODE && f.node->warm) {
                    const WarmStart &ws = *f.node->warm;
                    d.warm_nnz = (int32_t)ws.idx.size();
                    d.warm_idx = ws.idx.data();
                    d.warm_val = ws.val.data();
                }
            }
            bind_sets(batch);
        }
        if (!batch.empty()) {
            rc = submit_nodes(P, batch.data(), (int32_t)batch.size());
            if (rc) break;
        }
        t_fill += elapsed() - tm;
        // collect results
        tm = elapsed();
        int32_t got = 0;
        rc = poll(&got, 200000);
        t_poll += elapsed() - tm;
        if (rc < 0) break;
        rc = 0;
        tm = elapsed();
        std::vector<kbnb_node_desc> evals;
        set_store.clear();
        for (int r = 0; r < got; ++r) {
            const kbnb_bound_result &br = out[r];
            auto it = flight.find(br.tag);
            if (it == flight.end()) continue;
            Flight f = std::move(it->second);
            flight.erase(it);
            const double *beta = betas.data() + (size_t)r * p;
            const double *beta_lb = audit ? betas_lb.data() + (size_t)r * p : nullptr;
            if (f.kind == FL_SUPPORT) {
                take_support(f.support, br.primal_value, br.lower_bound, beta, beta_lb);
                continue;
            }
            Open *o = f.node;
            flight_lb.erase(flight_lb.find(o->lb));
            ++nodes;
            if (br.status == KBNB_ERROR) {
                // a non-finite iterate: neither closing nor pruning the node
                // would be justified by its bound
                global_lb = std::min(global_lb, o->lb);
                delete o;
                rc = kbnb::set_error(KBNB_E_DEVICE, "node %llu: non-finite iterate (status ERROR)",
                                     (unsigned long long)br.tag);
                break;
            }
            const double lb = std::max(br.lower_bound, o->lb);
            CertPtr cert = o->cert;
            if (audit && br.lower_bound >= o->lb)
                cert = std::make_shared<const Cert>(
                    Cert{o->in, o->out, std::vector<double>(beta_lb, beta_lb + p), br.lower_bound});
            if (prunable(lb)) {
                leaf_lb = std::min(leaf_lb, lb);
                add_leaf(0, o->in, o->out, lb, cert);
                delete o;
                continue;
            }
            // rounding support -> re-optimisation
            std::vector<int32_t> S(sup.begin() + (size_t)r * k, sup.begin() + (size_t)r * k + br.support_len);
            if (!S.empty() && !evaluated.count(S)) support_desc(S, evals);
            const int kbar = k - (int)o->in.size();
            const int pf = p - (int)o->in.size() - (int)o->out.size();
            int j = br.branch_index;
            // closed: integral, or every free coordinate is zero at a tight
            // bound (a node stopped early as unprunable is branched instead)
            if (!rs && (kbar <= 0 || pf <= kbar || (j < 0 && br.status != KBNB_UNPRUNABLE))) {
                leaf_lb = std::min(leaf_lb, lb);
                add_leaf(1, o->in, o->out, lb, cert);
                delete o;
                continue;
            }
            if (j < 0) {  // every free coordinate is zero: the first free index
                // (the smallest index in neither sorted list)
                size_t a = 0, b = 0;
                for (int q = 0; q < p; ++q) {
                    if (a < o->in.size() && o->in[a] == q) { ++a; continue; }
                    if (b < o->out.size() && o->out[b] == q) { ++b; continue; }
                    j = q;
                    break;
                }
            }
            // the parent's iterate, sparse, shared by both children
            std::shared_ptr<WarmStart> ws;
            {
                size_t nnz = 0;
                for (int q = 0; q < p; ++q) nnz += (beta[q] != 0.0);
                if (nnz) {
                    ws = std::make_shared<WarmStart>();
                    ws->idx.reserve(nnz);
                    ws->val.reserve(nnz);
                    for (int q = 0; q < p; ++q)
                        if (beta[q] != 0.0) {
                            ws->idx.push_back(q);
                            ws->val.push_back(beta[q]);
                        }
                }
            }
            // children z_j = 1 (a copy of the parent's sets) and z_j = 0 (the
            // parent's sets moved); both index lists stay sorted.  The z_j = 0
            // child comes first in queue order among equals (the smaller seq).
            const uint64_t seq0 = seq;
            seq += 2;
            for (int side = 1; side >= 0; --side) {
                Open *c = new Open();
                c->lb = lb;
                c->cert = cert;
                c->depth = o->depth + 1;
                c->seq = seq0 + (uint64_t)side;
                c->warm = ws;
                if (side == 1) {
                    c->in = o->in;
                    c->out = o->out;
                } else {
                    c->in = std::move(o->in);
                    c->out = std::move(o->out);
                }
                std::vector<int32_t> &grow = (side == 0) ? c->out : c->in;
                grow.insert(std::upper_bound(grow.begin(), grow.end(), j), j);
                push_open(c);
            }
            delete o;
        }
        t_res += elapsed() - tm;
        if (rc) break;
        tm = elapsed();
        rc = cycle_supports();
        t_flush += elapsed() - tm;
        if (rc) break;
        if (!evals.empty()) {
            bind_sets(evals);
            rc = submit_nodes(P, evals.data(), (int32_t)evals.size());
            if (rc) break;
        }
    }
    if (!rc) rc = flush_supports();
    else if (!inflight.empty()) (void)collect_supports();  // leave no batch on the device
    // Nodes still in flight: take what has already completed, then cancel
    // the rest (the engine drops their results), so the handle is idle and
    // reusable.  An unexplored node's parent bound holds for its subtree.
    while (!flight.empty()) {
        int32_t got = 0;
        int prc = poll(&got, 0);
        if (prc < 0) {
            if (!rc) rc = prc;
            break;
        }
        if (got == 0) break;
        for (int r = 0; r < got; ++r) {
            auto it = flight.find(out[r].tag);
            if (it == flight.end()) continue;
            if (it->second.kind == FL_SUPPORT) {
                if (!rc && out[r].status != KBNB_ERROR)
                    take_support(it->second.support, out[r].primal_value, out[r].lower_bound,
                                 betas.data() + (size_t)r * p, audit ? betas_lb.data() + (size_t)r * p : nullptr);
            } else {
                // bounded but not expanded: its parent's bound (certified by
                // the parent's certificate) holds for its subtree
                Open *o = it->second.node;
                global_lb = std::min(global_lb, o->lb);
                add_leaf(3, o->in, o->out, o->lb, o->cert);
                delete o;
            }
            flight.erase(it);
        }
    }
    for (auto &f : flight)
        if (f.second.kind == FL_NODE) {
            global_lb = std::min(global_lb, f.second.node->lb);
            add_leaf(3, f.second.node->in, f.second.node->out, f.second.node->lb, f.second.node->cert);
            delete f.second.node;
        }
    if (!flight.empty()) {
        flight.clear();
        const int crc = cancel_nodes(P);
        if (!rc) rc = crc;
    }
    while (!open.empty()) {
        Open *o = pop_open();
        global_lb = std::min(global_lb, o->lb);
        add_leaf(3, o->in, o->out, o->lb, o->cert);
        delete o;
    }
    for (auto &w : leaf_waiting) {
        global_lb = std::min(global_lb, w.second.first);
        add_leaf(2, w.first, complement(w.first), w.second.first, w.second.second);
    }
    if (audit) {
        kbnb::keep_lb_beta(P, false);
        std::lock_guard<std::mutex> g(kbnb::g_audit_mu);
        kbnb::g_audit[P] = leaves;
    }
    if (rc) return rc;
    res->objective = UB;
    res->lower_bound = std::min(std::min(global_lb, leaf_lb), UB);
    res->rel_gap = std::isfinite(UB) ? (UB - res->lower_bound) / std::max(std::fabs(UB), 1e-12) : INFINITY;
    res->nodes = nodes;
    // a tree exhausted with a gap above the tolerance (nodes that hit their
    // iteration cap keep loose bounds) is not reported optimal
    if (status == 0 && !(res->rel_gap <= gap_tol)) status = 3;
    res->status = status;
    res->support_len = (int32_t)best_support.size();
    for (int r = 0; r < k; ++r) res->support[r] = r < (int)best_support.size() ? best_support[r] : -1;
    if (res->beta) memcpy(res->beta, best_beta.data(), sizeof(double) * p);
    res->incumbent_updates = updates;
    res->audit_leaves = audit ? (int64_t)leaves->size() : 0;
    res->rashomon_size = 0;
    if (rs) {
        // the set: recorded supports within the final threshold, by value,
        // ties by the support sequence; the best N when capped
        const double t = tau();
        std::vector<std::pair<double, const std::vector<int32_t> *>> sel;
        for (auto &kv : recorded)
            if (kv.second.value <= t) sel.push_back({kv.second.value, &kv.first});
        std::sort(sel.begin(), sel.end(), [](const auto &a, const auto &b) {
            return a.first != b.first ? a.first < b.first : *a.second < *b.second;
        });
        if (capN > 0 && (int64_t)sel.size() > capN) sel.resize((size_t)capN);
        kbnb_pool *pool = kbnb::pool_new();
        std::vector<double> c;
        for (auto &e : sel) {
            const std::vector<double> &beta = recorded[*e.second].beta;
            c.clear();
            for (int32_t j : *e.second) c.push_back(beta[(size_t)j]);
            kbnb::pool_append(pool, *e.second, c.data(), e.first);
        }
        res->rashomon_size = (int64_t)sel.size();
        kbnb::store_rashomon(P, pool);
    }
    res->seconds = elapsed();
    return KBNB_OK;
}

extern "C" int bnb_audit_leaf(kbnb_problem *P, int64_t i, int32_t *kind, double *bound, int8_t *leaf_state,
                              int8_t *cert_state, double *cert_beta, double *cert_bound)
{
    if (!P) return kbnb::set_error(KBNB_E_BAD_HANDLE, "NULL problem");
    int64_t info[11];
    int rc = problem_info(P, info, nullptr);
    if (rc) return rc;
    const int p = (int)info[1];
    std::shared_ptr<std::vector<kbnb::AuditLeaf>> lv;
    {
        std::lock_guard<std::mutex> g(kbnb::g_audit_mu);
        auto it = kbnb::g_audit.find(P);
        if (it != kbnb::g_audit.end()) lv = it->second;
    }
    if (!lv) return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "no audited search on this problem");
    if (i < 0 || i >= (int64_t)lv->size())
        return kbnb::set_error(KBNB_E_INVALID_ARGUMENT, "leaf %lld outside [0, %zu)", (long long)i, lv->size());
    const kbnb::AuditLeaf &L = (*lv)[(size_t)i];
    auto fill = [p](int8_t *st, const std::vector<int32_t> &in, const std::vector<int32_t> &out) {
        for (int j = 0; j < p; ++j) st[j] = 0;
        for (int32_t j : in) st[j] = 1;
        for (int32_t j : out) st[j] = -1;
    };
    if (kind) *kind = L.kind;
    if (bound) *bound = L.bound;
    if (leaf_state) fill(leaf_state, L.in, L.out);
    if (L.cert) {
        if (cert_state) fill(cert_state, L.cert->in, L.cert->out);
        if (cert_beta) memcpy(cert_beta, L.cert->beta.data(), sizeof(double) * (size_t)p);
        if (cert_bound) *cert_bound = L.cert->bound;
    } else {
        if (cert_state) memset(cert_state, 0, (size_t)p);
        if (cert_beta) memset(cert_beta, 0, sizeof(double) * (size_t)p);
        if (cert_bound) *cert_bound = -INFINITY;
    }
    return KBNB_OK;
}
