// kbnb_engine.hip -- host side of libkbnb: problem setup, the node-slot engine
// (continuous batching over a fixed set of device slots), the C ABI of
// include/kbnb.h and the branch-and-bound driver.
//
// Engine round (one worker thread per problem, one HIP stream):
//   1. admit queued nodes into free slots (one H2D copy of packed records and
//      one scatter kernel);
//   2. replay the captured graph: `cert_period` FISTA steps (fwd, bwd, prox)
//      followed by the float64 certificate (cfwd, cbwd, cfin);
//   3. copy the per-slot status arrays back, retire the slots whose status is
//      final (their iterates are gathered into one buffer and copied back),
//      and hand the results to poll_bounds.
// Slots that finish are refilled at the next round while the others keep
// iterating, so the batch stays full while work is queued (Sec. 4.1 batch
// assembly; App. E.4 sizing replaced by a device-memory budget).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <queue>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/kbnb.h"
#include "kbnb_internal.h"

using namespace kbnb;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(KBNB_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

extern "C" const char *last_error(void) { return g_last_error.c_str(); }

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

namespace kbnb {
// error reporting for the host-side drivers built on the C ABI
int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
}  // namespace kbnb

// ---------------------------------------------------------------------------
// problem object
// ---------------------------------------------------------------------------
struct PendingNode {
    uint64_t tag;
    double t_submit = 0;      // steady-clock seconds at submit_nodes
    std::vector<int8_t> st;  // ldp entries
    std::vector<double> warm; // empty or p entries
    std::vector<int32_t> widx; // or a sparse warm start (warm empty)
    std::vector<double> wval;
    int kbar, n0;
    double ub, tol;
    int max_iter;
    int early;
};

struct DoneNode {
    kbnb_bound_result r;
    std::vector<int32_t> sup;
    std::vector<double> beta;
    std::vector<double> beta_lb;  // filled when the problem keeps them (audits)
};

// One launch configuration of a round: the launches cover the first `mact`
// slot columns, with split-K counts chosen for that many column tiles.  Each
// has its own captured graph, built on first use.
struct Variant {
    int mact = 0;
    int gsplit = 1, gchunk = 0;
    int qsplit = 1, qchunk = 0;
    hipGraphExec_t graph = nullptr;
    bool captured = false;
};

// Host view of one copy of the slot-state block.
struct HostSlots {
    int32_t *status = nullptr, *iter = nullptr, *jstar = nullptr, *slen = nullptr, *sup = nullptr;
    double *lb = nullptr, *phi = nullptr, *gap = nullptr;
};

struct kbnb_problem {
    int device = 0;                  // the device current at create_problem
    uint64_t charged = 0;            // bytes charged to the process-wide device budget
    bool own_stream = true;          // false: the stream belongs to the shared pool
    unsigned char *scratch = nullptr; // that device's copy of the allocation-free scratch array
    // instance
    int n = 0, p = 0, k = 0, loss = 0, xtype = 0;
    double lambda2 = 0, M = 0, L = 0, eta = 0;
    bool iter_f64 = false;
    int ti_bytes = 4;
    // plane mode (bfloat16 X, float32 or anchored iteration): tiled copies of
    // X and X^T, and the point and R as nb bfloat16 planes
    bool planes = false;
    int nb = 0, nkb_x = 0, nkb_xt = 0;
    int tile_rows = 0;   // tile height of the iteration's contractions (0: rule)
    int split_rows = 0;  // rows of X per split of X^T R (0: rule)
    int reopt_groups = 0; // workgroups per support in the re-optimisation (0: automatic)
    uint16_t *xtile = nullptr, *xttile = nullptr, *yp = nullptr, *rp = nullptr;
    // sizes
    int ldp = 0, npad = 0, pm = 0, m = 0, mpad = 0, pp = 256;
    int tiles_n = 0;
    // split-K buffers are allocated for the largest split count of any launch
    // width (the narrowest width has the most splits)
    int gsplit_alloc = 1, qsplit_alloc = 1;
    int cert_period = 8;
    uint64_t budget = 0, bytes = 0;
    // device memory
    void *arena = nullptr;
    bool own_x = true;
    void *X = nullptr, *XT = nullptr, *Yi = nullptr, *R = nullptr, *Gp = nullptr;
    double *y = nullptr, *B = nullptr, *Bprev = nullptr, *Z = nullptr, *Qp = nullptr;
    double *lsum = nullptr, *csum = nullptr, *gbuf = nullptr;
    double *gbuf_lb = nullptr;  // gathered Blb columns (only when results carry them)
    double *h_gbuf_lb = nullptr;
    bool want_lb_beta = false;  // results also carry the iterate of the certified bound
    double *Bbest = nullptr;   // iterate of the best certified primal value [mpad][ldp]
    bool anchored = false;     // anchored float32 iteration
    Anchor an{};               // its buffers (all NULL when off)
    int8_t *st = nullptr;
    uint8_t *stage_d = nullptr;
    int32_t *gslots_d = nullptr;
    SlotState ss{};
    // pinned host mirrors, double-buffered: the engine enqueues round r + 1
    // before it reads round r's slot states
    uint8_t *stage_h = nullptr;     // two halves of mpad admission records
    int rec_bytes = 0;
    HostSlots hs[2];
    int32_t *h_gslots = nullptr;
    double *h_gbuf = nullptr;
    char *slot_dev = nullptr;   // contiguous device block of the slot arrays
    char *slot_host = nullptr;  // two pinned mirrors of that block
    size_t slot_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t sstream = nullptr;  // support re-optimisation (created on first use)
    void *sbuf = nullptr;           // its device buffers, grown on demand
    char *spin = nullptr;           // pinned host mirror of sbuf's input and output regions
    size_t spin_bytes = 0;
    size_t s_in_bytes = 0, s_out_off = 0, s_out_bytes = 0;  // those regions of the batch in flight
    size_t sbuf_bytes = 0;
    hipEvent_t sev = nullptr;       // end of the support batch in flight
    int s_count = 0;                // that batch: supports and stored coefficients
    int64_t s_coefs = 0;
    double *s_val = nullptr, *s_low = nullptr, *s_coef = nullptr, *s_coef_lb = nullptr;
    int32_t *s_st = nullptr, *s_it = nullptr;
    SupportLaunch s_launch;         // that batch's launch (split rows: steps launched so far)
    int s_steps = 0;
    int s_steps_hint = 128;         // step launches the last split batch needed
    hipStream_t gstream = nullptr;  // gathers beside a round enqueued ahead (created on first use:
                                    // streams share the process's few hardware queues)
    hipEvent_t ev_round[2] = {nullptr, nullptr};
    int64_t round_id[2] = {0, 0};
    std::vector<int> round_kinds[2];  // timed launches of the round (instrumentation)
    double round_useful[2] = {0, 0}, round_slots[2] = {0, 0};
    std::vector<int64_t> slot_round;  // round at which each slot's node was admitted
    int64_t next_round = 0;
    bool use_graphs = true;
    Consts c{};
    // engine
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<PendingNode> pending;
    std::deque<DoneNode> done;
    std::vector<uint64_t> slot_tag;
    std::set<int> free_slots;        // lowest index first, so running slots stay packed
    std::vector<char> occupied;      // slot holds an admitted, unretired node
    std::vector<char> cancelled;     // slot's node was cancelled: its result is dropped
    std::vector<double> slot_t_submit, slot_t_admit;  // per slot: its node's submit / admission time
    bool cancel_dev = false;         // cancelled slots still to be stopped on the device
    std::vector<Variant> var;        // launch widths 64, 128, ..., mpad
    int active = 0;
    bool shutdown = false;
    int engine_error = 0;
    std::string engine_msg;
    std::mutex api_mu;  // serialises calls on this handle
    // stats
    std::atomic<long> rounds{0};
    // kernel timing (instrumentation): per kernel type total ms and launches
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double kt_ms[8] = {0};
    int64_t kt_n[8] = {0};
    double useful_cols = 0;   // sum over timed iteration launches of sum_b (p - |J0_b|)
    double running_cols = 0;  // sum over timed iteration launches of running slots
    std::vector<int> slot_n0; // |J0| of the node in each slot
};

static int round_pow2_down(int64_t v)
{
    int r = 1;
    while ((int64_t)r * 2 <= v) r *= 2;
    return r;
}

// ---------------------------------------------------------------------------
// per-slot bytes and arena layout
// ---------------------------------------------------------------------------
struct Layout {
    size_t off[32];
    size_t total;
};

static size_t per_slot_bytes(const kbnb_problem *P)
{
    // the point and R: float / double, or nb bfloat16 planes
    const size_t ti = P->planes ? 2 * (size_t)P->nb : (size_t)P->ti_bytes;
    size_t b = 0;
    b += (size_t)P->ldp * (ti + 8 + 8 + 8 + 8 + 1);    // Yi, B, Bprev, Bbest, Blb, st
    b += (size_t)P->npad * (ti + 8);                   // R, Z
    b += (size_t)P->gsplit_alloc * P->ldp * P->ti_bytes; // Gp
    b += (size_t)P->qsplit_alloc * P->ldp * 8;         // Qp
    b += (size_t)P->tiles_n * 16;                      // lsum, csum
    b += (size_t)P->ldp * 16 + 128 + P->k * 4;         // gather buffers, scalars, support
    b += (size_t)P->pp * 4;                            // sort permutation
    if (P->anchored) b += (size_t)P->npad * 8 + (size_t)P->ldp * 16;  // S_c, beta_c, grad F(beta_c)
    return b;
}

// Split-K for a launch covering `mact` columns: enough workgroups to cover
// the 256 CUs a few times and no split deeper than 4096 rows (a workgroup
// walks its split serially), at most 32 splits (the per-node kernels add the
// partials, exactly the splits the same round's launch wrote).
static void splits_for(const kbnb_problem *P, int mact, Variant &v)
{
    if (P->planes) {
        // the streaming X^T R: 256-row tiles; at least 2048 workgroups (eight
        // per CU) where 32 splits allow, in a multiple of 8 splits so that no
        // split slot of the launch grid (8 per tile group) stays empty, and
        // splits of a multiple of 128 rows (the tiled layout's k block)
        const int st = ((P->pm + 255) / 256) * (mact / GEMM_BN);
        int ws = std::min(32, (int)round_up(std::max(1, (2048 + st - 1) / st), 8));
        int ch = (int)round_up((P->npad + ws - 1) / ws, 128);
        if (P->split_rows > 0) ch = (int)round_up(std::max(P->split_rows, (P->npad + 31) / 32), 128);
        v.gchunk = ch;
        v.gsplit = (P->npad + ch - 1) / ch;
    }
    const int tiles = (P->pm / GEMM_BM) * (mact / GEMM_BN);
    const int kt = P->npad / GEMM_BK;  // 16-wide k chunks
    int want = std::max(1, (256 + tiles - 1) / tiles);
    want = std::max(want, (P->npad + 4095) / 4096);
    want = std::min(want, std::max(1, kt / 4));
    want = std::min(want, 32);
    // split s runs on XCD s % 8: a count off a multiple of 8 leaves some XCDs
    // a split more than the rest (25 splits: XCD 0 takes 4, the others 3),
    // and fewer than 8 leaves XCDs idle; round to a multiple of 8 within the caps
    if (want > 1 && want % 8) {
        const int cap = std::min(32, std::max(1, kt / 4));
        const int up = (want + 7) / 8 * 8, down = want / 8 * 8;
        if (up <= cap) want = up;
        else if (down >= 8) want = down;
    }
    const int chunk = (int)round_up((P->npad + want - 1) / want, GEMM_BK);
    v.mact = mact;
    if (!P->planes) {
        // a given split depth, kept to at most 32 splits
        const int gch = (P->split_rows > 0)
                            ? (int)round_up(std::max(P->split_rows, (P->npad + 31) / 32), GEMM_BK)
                            : chunk;
        v.gchunk = gch;
        v.gsplit = (P->npad + gch - 1) / gch;
    }
    v.qchunk = chunk;
    v.qsplit = (P->npad + chunk - 1) / chunk;
}

static void choose_splits(kbnb_problem *P)
{
    P->var.clear();
    for (int w = GEMM_BN; ; w *= 2) {
        Variant v;
        splits_for(P, std::min(w, P->mpad), v);
        P->var.push_back(v);
        if (w >= P->mpad) break;
    }
    P->gsplit_alloc = P->qsplit_alloc = 1;
    for (const Variant &v : P->var) {
        P->gsplit_alloc = std::max(P->gsplit_alloc, v.gsplit);
        P->qsplit_alloc = std::max(P->qsplit_alloc, v.qsplit);
    }
}

// total_out != NULL: only compute the arena's size into *total_out
static int alloc_arena(kbnb_problem *P, size_t xbytes, size_t xel, size_t *total_out = nullptr)
{
    const size_t ti = P->ti_bytes;
    const size_t mp = P->mpad;
    std::vector<std::pair<void **, size_t>> items;
    size_t sizes[] = {
        P->own_x ? xbytes : 0,                   // X
        (size_t)P->pm * P->npad * xel,           // XT
        (size_t)P->npad * 8,                     // y
        P->planes ? 0 : mp * P->ldp * ti,        // Yi
        P->planes ? 0 : mp * P->npad * ti,       // R
        (size_t)P->gsplit_alloc * mp * P->ldp * ti, // Gp
        mp * P->ldp * 8,                         // B
        mp * P->ldp * 8,                         // Bprev
        mp * P->npad * 8,                        // Z
        (size_t)P->qsplit_alloc * mp * P->ldp * 8, // Qp
        (size_t)P->tiles_n * mp * 8,             // lsum
        (size_t)P->tiles_n * mp * 8,             // csum
        mp * P->ldp,                             // st
        mp * P->rec_bytes,                       // stage
        mp * 4,                                  // gather slots
        mp * P->ldp * 8,                         // gather buffer
        mp * 8 * 7,                              // double slot arrays
        mp * 4 * 7,                              // int slot arrays
        mp * P->k * 4,                           // supports
        mp * P->ldp * 8,                         // Bbest
        mp * (size_t)P->pp * 4,                  // sort permutations
        P->anchored ? mp * P->npad * 8 : 0,      // anchor S_c
        P->anchored ? mp * P->ldp * 8 : 0,       // anchor beta_c
        P->anchored ? mp * P->ldp * 8 : 0,       // anchor grad F(beta_c)
        P->anchored ? (size_t)P->ldp * 8 : 0,    // grad F(0)
        mp * P->ldp * 8,                         // Blb
        mp * P->ldp * 8,                         // second gather buffer (Blb columns)
        P->planes ? (size_t)round_up(P->npad, 16) * P->nkb_x * 128 * 2 : 0,  // tiled X
        P->planes ? (size_t)P->pm * P->nkb_xt * 128 * 2 : 0,                 // tiled X^T
        P->planes ? (size_t)P->nb * mp * P->ldp * 2 : 0,                      // planes of Y
        P->planes ? (size_t)P->nb * mp * P->npad * 2 : 0,                     // planes of R
    };
    const int nitems = sizeof(sizes) / sizeof(sizes[0]);
    size_t off[32];
    size_t total = 0;
    for (int i = 0; i < nitems; ++i) {
        off[i] = total;
        total += round_up(sizes[i], 256);
    }
    if (total_out) {
        *total_out = total;
        return 0;
    }
    if (P->budget && total > P->budget)
        return fail(KBNB_E_BUDGET_EXCEEDED, "problem needs %zu bytes, budget %llu", total,
                    (unsigned long long)P->budget);
    void *a = nullptr;
    hipError_t e = hipMalloc(&a, total);
    if (e != hipSuccess) return fail(KBNB_E_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", total, hipGetErrorString(e));
    e = hipMemsetAsync(a, 0, total, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) {
        (void)hipFree(a);
        return fail(KBNB_E_DEVICE, "clearing device memory failed: %s", hipGetErrorString(e));
    }
    P->arena = a;
    P->bytes = total;
    char *base = (char *)a;
    if (P->own_x) P->X = base + off[0];
    P->XT = base + off[1];
    P->y = (double *)(base + off[2]);
    P->Yi = base + off[3];
    P->R = base + off[4];
    P->Gp = base + off[5];
    P->B = (double *)(base + off[6]);
    P->Bprev = (double *)(base + off[7]);
    P->Z = (double *)(base + off[8]);
    P->Qp = (double *)(base + off[9]);
    P->lsum = (double *)(base + off[10]);
    P->csum = (double *)(base + off[11]);
    P->st = (int8_t *)(base + off[12]);
    P->stage_d = (uint8_t *)(base + off[13]);
    P->gslots_d = (int32_t *)(base + off[14]);
    P->gbuf = (double *)(base + off[15]);
    double *dd = (double *)(base + off[16]);
    int32_t *ii = (int32_t *)(base + off[17]);
    P->ss.theta = dd + 0 * mp;
    P->ss.tmom = dd + 1 * mp;
    P->ss.lb = dd + 2 * mp;
    P->ss.phi = dd + 3 * mp;
    P->ss.gap = dd + 4 * mp;
    P->ss.ub = dd + 5 * mp;
    P->ss.tol = dd + 6 * mp;
    P->ss.status = ii + 0 * mp;
    P->ss.iter = ii + 1 * mp;
    P->ss.max_iter = ii + 2 * mp;
    P->ss.kbar = ii + 3 * mp;
    P->ss.jstar = ii + 4 * mp;
    P->ss.slen = ii + 5 * mp;
    P->ss.early = ii + 6 * mp;
    P->ss.sup = (int32_t *)(base + off[18]);
    P->Bbest = (double *)(base + off[19]);
    P->ss.perm = (int32_t *)(base + off[20]);
    if (P->anchored) {
        P->an.sc = (double *)(base + off[21]);
        P->an.bc = (double *)(base + off[22]);
        P->an.gc = (double *)(base + off[23]);
        P->an.g0 = (const double *)(base + off[24]);
    }
    P->ss.blb = (double *)(base + off[25]);
    P->gbuf_lb = (double *)(base + off[26]);
    if (P->planes) {
        P->xtile = (uint16_t *)(base + off[27]);
        P->xttile = (uint16_t *)(base + off[28]);
        P->yp = (uint16_t *)(base + off[29]);
        P->rp = (uint16_t *)(base + off[30]);
        P->Yi = nullptr;
        P->R = nullptr;
    }
    P->slot_dev = base + off[16];
    P->slot_bytes = off[18] + sizes[18] - off[16];
    return 0;
}

// ---------------------------------------------------------------------------
// graph of one engine round
// ---------------------------------------------------------------------------
static Consts consts_for(const kbnb_problem *P, const Variant &v)
{
    Consts c = P->c;
    c.mact = v.mact;
    return c;
}

static void enqueue_round(kbnb_problem *P, const Variant &v)
{
    hipStream_t s = P->stream;
    const Consts c = consts_for(P, v);
    for (int it = 0; it < P->cert_period; ++it) {
        launch_fwd_dloss(s, P->xtype, P->iter_f64, P->X, P->Yi, P->R, P->y, c, P->ss.status, P->an);
        launch_bwd(s, P->xtype, P->iter_f64, P->XT, P->R, P->Gp, v.gsplit, v.gchunk, c, P->ss.status);
        launch_prox_iter(s, P->iter_f64, P->Gp, v.gsplit, P->B, P->Bprev, P->Yi, P->st, P->ss, c, P->an);
    }
    launch_cert_fwd(s, P->xtype, P->X, P->B, P->Z, P->y, P->lsum, P->csum, c, P->ss.status, P->an.sc);
    launch_cert_bwd(s, P->xtype, P->XT, P->Z, P->Qp, v.qsplit, v.qchunk, c, P->ss.status);
    launch_cert_finish(s, P->Qp, v.qsplit, P->lsum, P->csum, P->tiles_n, P->B, P->Bbest, P->st, P->ss, c, 1,
                       P->an, P->Bprev, (float *)P->Yi);
}

// Kernel types for the timing instrumentation.
enum { KT_FWD = 0, KT_BWD = 1, KT_PROX = 2, KT_CFWD = 3, KT_CBWD = 4, KT_CFIN = 5, KT_ADMIT = 6, KT_RED = 7 };

// Same launches as enqueue_round, each bracketed by a hipEvent pair on the
// engine stream; the elapsed times are read after the round synchronises.
static int enqueue_round_timed(kbnb_problem *P, const Variant &v, std::vector<int> &kinds)
{
    hipStream_t s = P->stream;
    const Consts c = consts_for(P, v);
    const size_t need = 2 * (3 * (size_t)P->cert_period + 3);
    while (P->ev.size() < need) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        P->ev.push_back(e);
    }
    kinds.clear();
    size_t q = 0;
    // each launch carries its own start/stop events (kernel timestamps)
    auto timed = [&](int kind) {
        kinds.push_back(kind);
        g_ktime.start = P->ev[q];
        g_ktime.stop = P->ev[q + 1];
        q += 2;
    };
    for (int it = 0; it < P->cert_period; ++it) {
        timed(KT_FWD);
        launch_fwd_dloss(s, P->xtype, P->iter_f64, P->X, P->Yi, P->R, P->y, c, P->ss.status, P->an);
        timed(KT_BWD);
        launch_bwd(s, P->xtype, P->iter_f64, P->XT, P->R, P->Gp, v.gsplit, v.gchunk, c, P->ss.status);
        timed(KT_PROX);
        launch_prox_iter(s, P->iter_f64, P->Gp, v.gsplit, P->B, P->Bprev, P->Yi, P->st, P->ss, c, P->an);
    }
    timed(KT_CFWD);
    launch_cert_fwd(s, P->xtype, P->X, P->B, P->Z, P->y, P->lsum, P->csum, c, P->ss.status, P->an.sc);
    timed(KT_CBWD);
    launch_cert_bwd(s, P->xtype, P->XT, P->Z, P->Qp, v.qsplit, v.qchunk, c, P->ss.status);
    timed(KT_CFIN);
    launch_cert_finish(s, P->Qp, v.qsplit, P->lsum, P->csum, P->tiles_n, P->B, P->Bbest, P->st, P->ss, c, 1,
                       P->an, P->Bprev, (float *)P->Yi);
    g_ktime = KernelTiming{};
    HIP_TRY(hipGetLastError());
    return 0;
}

// capture one round of variant v into a graph (once); on failure the round
// is issued as direct launches
static void build_graph(kbnb_problem *P, Variant &v)
{
    v.captured = true;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    enqueue_round(P, v);
    if (hipStreamEndCapture(P->stream, &g) != hipSuccess || !g) {
        (void)hipGetLastError();
        return;
    }
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    v.graph = ge;
}

__global__ void k_gather_cols(const double *__restrict__ B, int ldp, int p,
                              const int32_t *__restrict__ slots, double *__restrict__ out)
{
    const int r = blockIdx.x;
    const int64_t src = (int64_t)slots[r] * ldp;
    for (int j = threadIdx.x; j < p; j += blockDim.x) out[(int64_t)r * p + j] = B[src + j];
}

// Stops cancelled slots: a running slot in the mask gets a final status
// (iteration cap), so the next rounds skip it and the host retires it.
struct SlotMask {
    uint32_t w[4096 / 32];
};
__global__ void k_cancel_slots(int32_t *__restrict__ status, int m, SlotMask mask)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < m && ((mask.w[b >> 5] >> (b & 31)) & 1u) && status[b] == SLOT_RUNNING) status[b] = KBNB_MAXITER;
}

// ---------------------------------------------------------------------------
// engine worker
// ---------------------------------------------------------------------------
#define HIP_BREAK(expr)                                                                  \
    {                                                                                    \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            rc = fail(KBNB_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
            break;                                                                       \
        }                                                                                \
    }

// Admit queued nodes into the lowest free slots and enqueue one round (its
// admissions, the captured graph of the narrowest covering width, and the
// copy of the slot states into host buffer `buf`).  Called and returns with
// the lock held; `enq` tells whether a round was enqueued.
static int enqueue_round_async(kbnb_problem *P, std::unique_lock<std::mutex> &lk, int buf, bool &enq)
{
    enq = false;
    const int64_t rid = P->next_round;
    int nadm = 0;
    // slots cancelled since the last round: stopped on the device before
    // this round's admissions (a cancelled slot stays occupied until retired,
    // so no admission can target it)
    bool stop_cancelled = false;
    SlotMask cmask{};
    if (P->cancel_dev) {
        P->cancel_dev = false;
        for (int b = 0; b < P->m; ++b)
            if (P->occupied[b] && P->cancelled[b]) {
                cmask.w[b >> 5] |= 1u << (b & 31);
                stop_cancelled = true;
            }
    }
    uint8_t *stage = P->stage_h + (size_t)buf * P->mpad * P->rec_bytes;
    while (!P->pending.empty() && !P->free_slots.empty()) {
        PendingNode nd = std::move(P->pending.front());
        P->pending.pop_front();
        const int slot = *P->free_slots.begin();
        P->free_slots.erase(P->free_slots.begin());
        P->occupied[slot] = 1;
        P->slot_round[slot] = rid;
        uint8_t *rec = stage + (size_t)nadm * P->rec_bytes;
        AdmitRec h{};
        h.slot = slot;
        h.kbar = nd.kbar;
        h.max_iter = nd.max_iter;
        h.has_warm = (nd.warm.empty() && nd.widx.empty()) ? 0 : 1;
        h.ub = nd.ub;
        h.tol = nd.tol;
        h.early = nd.early;
        memcpy(rec, &h, sizeof h);
        memcpy(rec + sizeof(AdmitRec), nd.st.data(), P->ldp);
        if (h.has_warm) {
            const size_t woff = round_up(sizeof(AdmitRec) + P->ldp, 8);
            double *w = reinterpret_cast<double *>(rec + woff);
            if (!nd.warm.empty()) {
                memcpy(w, nd.warm.data(), sizeof(double) * P->p);
            } else {
                memset(w, 0, sizeof(double) * P->p);
                for (size_t r = 0; r < nd.widx.size(); ++r) w[nd.widx[r]] = nd.wval[r];
            }
        }
        P->slot_tag[slot] = nd.tag;
        P->slot_n0[slot] = nd.n0;
        P->slot_t_submit[slot] = nd.t_submit;
        P->slot_t_admit[slot] = now_s();
        ++P->active;
        ++nadm;
    }
    if (P->active == 0) return 0;
    const bool timed = P->timing;
    P->round_useful[buf] = P->round_slots[buf] = 0;
    if (timed) {
        for (int b = 0; b < P->m; ++b)
            if (P->occupied[b]) {
                P->round_useful[buf] += P->p - P->slot_n0[b];
                P->round_slots[buf] += 1;
            }
    }
    // launch width: the narrowest variant covering every occupied slot
    int hi = 0;
    for (int b = P->m - 1; b >= 0; --b)
        if (P->occupied[b]) { hi = b + 1; break; }
    Variant *var = &P->var.back();
    for (Variant &v : P->var)
        if (v.mact >= hi) { var = &v; break; }
    lk.unlock();
    hipStream_t s = P->stream;
    int rc = 0;
    P->round_kinds[buf].clear();
    do {
        if (stop_cancelled) {
            hipLaunchKernelGGL(k_cancel_slots, dim3((P->m + 255) / 256), dim3(256), 0, s, P->ss.status, P->m, cmask);
            HIP_BREAK(hipGetLastError());
        }
        if (nadm) {
            HIP_BREAK(hipMemcpyAsync(P->stage_d, stage, (size_t)nadm * P->rec_bytes, hipMemcpyHostToDevice, s));
            launch_admit(s, P->iter_f64, P->stage_d, nadm, P->rec_bytes, P->B, P->Bprev, P->Bbest, P->Yi,
                         P->st, P->ss, P->c, P->an);
        }
        if (!timed && P->use_graphs && !var->captured) build_graph(P, *var);
        if (timed) {
            rc = enqueue_round_timed(P, *var, P->round_kinds[buf]);
            if (rc) break;
        } else if (var->graph) {
            HIP_BREAK(hipGraphLaunch(var->graph, s));
        } else {
            enqueue_round(P, *var);
        }
        HIP_BREAK(hipMemcpyAsync(P->slot_host + (size_t)buf * P->slot_bytes, P->slot_dev, P->slot_bytes,
                                 hipMemcpyDeviceToHost, s));
        HIP_BREAK(hipEventRecord(P->ev_round[buf], s));
    } while (0);
    lk.lock();
    if (rc) return rc;
    P->round_id[buf] = rid;
    P->next_round = rid + 1;
    enq = true;
    return 0;
}

// Wait for the round in host buffer `buf`, gather the best iterates of the
// nodes that finished in it and hand their results over.  A slot counts only
// if its node was admitted at or before that round.  With a round already
// enqueued behind it (`ahead`) the gather runs on the side stream, beside
// that round; otherwise on the problem's own stream, so it never waits
// behind other problems' work queued on a shared hardware queue.  Called and
// returns with the lock held.
static int process_round(kbnb_problem *P, std::unique_lock<std::mutex> &lk, int buf, bool ahead)
{
    lk.unlock();
    const HostSlots &h = P->hs[buf];
    const int64_t rid = P->round_id[buf];
    const bool want_lb = P->want_lb_beta;
    int rc = 0, nfin = 0;
    do {
        HIP_BREAK(hipEventSynchronize(P->ev_round[buf]));
        const std::vector<int> &kinds = P->round_kinds[buf];
        for (size_t e = 0; e < kinds.size(); ++e) {
            float ms = 0.f;
            HIP_BREAK(hipEventElapsedTime(&ms, P->ev[2 * e], P->ev[2 * e + 1]));
            P->kt_ms[kinds[e]] += ms;
            P->kt_n[kinds[e]] += 1;
        }
        if (rc) break;
        if (!kinds.empty()) {
            P->useful_cols += P->round_useful[buf] * P->cert_period;
            P->running_cols += P->round_slots[buf] * P->cert_period;
        }
        for (int b = 0; b < P->m; ++b)
            if (P->occupied[b] && P->slot_round[b] <= rid && h.status[b] >= 0) P->h_gslots[nfin++] = b;
        if (nfin) {
            if (ahead && !P->gstream) HIP_BREAK(hipStreamCreate(&P->gstream));
            hipStream_t g = ahead ? P->gstream : P->stream;
            HIP_BREAK(hipMemcpyAsync(P->gslots_d, P->h_gslots, (size_t)nfin * 4, hipMemcpyHostToDevice, g));
            hipLaunchKernelGGL(k_gather_cols, dim3(nfin), dim3(256), 0, g, P->Bbest, P->ldp, P->p, P->gslots_d, P->gbuf);
            HIP_BREAK(hipMemcpyAsync(P->h_gbuf, P->gbuf, (size_t)nfin * P->p * 8, hipMemcpyDeviceToHost, g));
            if (want_lb) {
                hipLaunchKernelGGL(k_gather_cols, dim3(nfin), dim3(256), 0, g, P->ss.blb, P->ldp, P->p, P->gslots_d,
                                   P->gbuf_lb);
                HIP_BREAK(hipMemcpyAsync(P->h_gbuf_lb, P->gbuf_lb, (size_t)nfin * P->p * 8, hipMemcpyDeviceToHost, g));
            }
            HIP_BREAK(hipStreamSynchronize(g));
        }
    } while (0);
    lk.lock();
    if (rc) return rc;
    const double t_done = now_s();
    for (int r = 0; r < nfin; ++r) {
        const int b = P->h_gslots[r];
        if (P->cancelled[b]) {  // a cancelled node: its result is never returned
            P->cancelled[b] = 0;
            P->free_slots.insert(b);
            P->occupied[b] = 0;
            --P->active;
            continue;
        }
        DoneNode d;
        d.r.tag = P->slot_tag[b];
        d.r.lower_bound = h.lb[b];
        d.r.primal_value = h.phi[b];
        d.r.rel_gap = h.gap[b];
        d.r.status = h.status[b];
        d.r.iterations = h.iter[b];
        d.r.branch_index = h.jstar[b];
        d.r.support_len = h.slen[b];
        d.r.queue_seconds = P->slot_t_admit[b] - P->slot_t_submit[b];
        d.r.solve_seconds = t_done - P->slot_t_admit[b];
        d.sup.assign(h.sup + (size_t)b * P->k, h.sup + (size_t)(b + 1) * P->k);
        d.beta.assign(P->h_gbuf + (size_t)r * P->p, P->h_gbuf + (size_t)(r + 1) * P->p);
        if (want_lb) d.beta_lb.assign(P->h_gbuf_lb + (size_t)r * P->p, P->h_gbuf_lb + (size_t)(r + 1) * P->p);
        P->done.push_back(std::move(d));
        // the slot's device status stays >= 0 (not running) until a node is
        // admitted into it again
        P->free_slots.insert(b);
        P->occupied[b] = 0;
        --P->active;
    }
    P->rounds++;
    P->cv_done.notify_all();
    return 0;
}

// Problems of this process with nodes in flight (admitted or queued).
static std::atomic<int> g_busy_engines{0};

// The worker can keep two rounds in flight: it enqueues round r + 1 and then
// processes round r, so the device runs a round while the host hands over
// the previous one's results and stages new admissions.  It does so only
// while its problem is the only one with work: otherwise other problems'
// rounds already fill those host gaps, and a second queued round would only
// add queueing delay to every node.  It also needs 8 occupied slots (a
// round enqueued ahead runs empty if every node finished, which is likely
// when few are in flight) and no kernel timing (instrumentation).
static void engine_main(kbnb_problem *P)
{
    std::unique_lock<std::mutex> lk(P->mu);
    int pend = -1, next = 0, rc = 0;
    bool busy = false;
    for (;;) {
        const bool has_work = P->active > 0 || !P->pending.empty();
        if (has_work != busy) {
            busy = has_work;
            g_busy_engines += busy ? 1 : -1;
        }
        if (pend < 0) {
            P->cv_work.wait(lk, [&] { return P->shutdown || P->active > 0 || !P->pending.empty(); });
            if (P->shutdown) break;
            if (!busy) {
                busy = true;
                ++g_busy_engines;
            }
        }
        bool enq = false;
        const bool ahead_ok = !P->timing && P->active >= 8 && g_busy_engines.load() <= 1;
        if (!P->shutdown && (pend < 0 || ahead_ok) && (P->active > 0 || !P->pending.empty())) {
            rc = enqueue_round_async(P, lk, next, enq);
            if (rc) break;
        }
        if (pend >= 0) {
            rc = process_round(P, lk, pend, enq);
            if (rc) break;
            pend = -1;
        }
        if (enq) {
            pend = next;
            next ^= 1;
        }
        if (P->shutdown && pend < 0) break;
    }
    if (rc) {
        P->engine_error = rc;
        P->engine_msg = g_last_error;
        // fail every queued node; running ones are abandoned
        P->pending.clear();
        P->cv_done.notify_all();
    }
    if (pend >= 0) {
        lk.unlock();
        (void)hipEventSynchronize(P->ev_round[pend]);
        lk.lock();
    }
    if (busy) --g_busy_engines;
}

// ---------------------------------------------------------------------------
// lambda_max(X^T X) by the Lanczos method with full reorthogonalisation: the
// products X^T (X v) run on the device in float64, the Krylov basis and the
// tridiagonal matrix T stay on the host.  The largest eigenvalue of T (by
// Sturm-sequence bisection) is a lower estimate of lambda_max that converges
// in tens of products where the power iteration needs thousands on
// correlated designs; the step uses 1.02 times it.
// ---------------------------------------------------------------------------
// largest eigenvalue of the symmetric tridiagonal matrix (a[0..k), b[0..k-1))
static double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b, int k)
{
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {  // Gershgorin interval
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    // count(x) = eigenvalues below x (the negative pivots of T - x I)
    auto below = [&](double x) {
        int c = 0;
        double d = 1.0;
        for (int i = 0; i < k; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), 1e-300); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) < k) lo = mid;  // some eigenvalue lies at or above mid
        else hi = mid;
    }
    return hi;
}

static int estimate_L(kbnb_problem *P)
{
    const int n = P->n, p = P->p;
    double *dv = nullptr, *ds = nullptr, *dw = nullptr;
    HIP_TRY(hipMalloc(&dv, sizeof(double) * p));
    HIP_TRY(hipMalloc(&ds, sizeof(double) * P->npad));
    HIP_TRY(hipMalloc(&dw, sizeof(double) * p));
    const int kmax = std::min(p, 300);
    std::vector<std::vector<double>> V;
    std::vector<double> alpha, beta, v(p), w(p);
    // deterministic start with no special direction: splitmix-style hashing
    double nrm = 0;
    for (int j = 0; j < p; ++j) {
        uint64_t z = 0x9E3779B97F4A7C15ull * (uint64_t)(j + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[j] = 0.5 + (double)(z >> 11) * (1.0 / 9007199254740992.0);
        nrm += v[j] * v[j];
    }
    nrm = std::sqrt(nrm);
    for (auto &x : v) x /= nrm;
    double lam = 0, prev = -1.0;
    int rc = 0, stable = 0;
    for (int it = 0; it < kmax; ++it) {
        V.push_back(v);
        if (hipMemcpyAsync(dv, v.data(), sizeof(double) * p, hipMemcpyHostToDevice, P->stream) != hipSuccess) { rc = -1; break; }
        launch_matvec_f64(P->stream, P->xtype, P->X, P->ldp, n, p, dv, ds);
        launch_matvec_f64(P->stream, P->xtype, P->XT, P->npad, p, n, ds, dw);
        if (hipMemcpyAsync(w.data(), dw, sizeof(double) * p, hipMemcpyDeviceToHost, P->stream) != hipSuccess) { rc = -1; break; }
        if (hipStreamSynchronize(P->stream) != hipSuccess) { rc = -1; break; }
        double a = 0;
        for (int j = 0; j < p; ++j) a += v[j] * w[j];
        alpha.push_back(a);
        // w -= V (V^T w), twice (full reorthogonalisation)
        for (int pass = 0; pass < 2; ++pass)
            for (const auto &q : V) {
                double c = 0;
                for (int j = 0; j < p; ++j) c += q[j] * w[j];
                for (int j = 0; j < p; ++j) w[j] -= c * q[j];
            }
        double bn = 0;
        for (int j = 0; j < p; ++j) bn += w[j] * w[j];
        bn = std::sqrt(bn);
        lam = tridiag_max_eig(alpha, beta, (int)alpha.size());
        // converged: the estimate has not moved for three steps, or the
        // Krylov space is invariant (its Ritz values are eigenvalues)
        stable = (prev > 0 && std::fabs(lam - prev) <= 1e-13 * lam) ? stable + 1 : 0;
        prev = lam;
        if (stable >= 3 || !(bn > 1e-12 * std::max(lam, 1e-300))) break;
        beta.push_back(bn);
        for (int j = 0; j < p; ++j) v[j] = w[j] / bn;
    }
    (void)hipFree(dv);
    (void)hipFree(ds);
    (void)hipFree(dw);
    if (rc) return fail(KBNB_E_DEVICE, "Lanczos iteration failed");
    const double cl = (P->loss == KBNB_LOSS_SQUARED) ? 2.0 : 0.25;
    P->L = 1.02 * cl * std::max(lam, 1e-300);
    P->eta = 1.0 / P->L;
    return 0;
}

// grad F(0) = X^T l'(0, y) in float64: the anchor gradient of every newly
// admitted node of an anchored problem (l'(0, y) = -2 y squared, -y / 2 logistic)
static int anchor_grad0(kbnb_problem *P)
{
    std::vector<double> yh(P->n), v(P->npad, 0.0);
    HIP_TRY(hipMemcpy(yh.data(), P->y, sizeof(double) * P->n, hipMemcpyDeviceToHost));
    for (int i = 0; i < P->n; ++i) v[i] = (P->loss == KBNB_LOSS_SQUARED) ? -2.0 * yh[i] : -0.5 * yh[i];
    double *dv = nullptr;
    HIP_TRY(hipMalloc(&dv, sizeof(double) * P->npad));
    hipError_t e = hipMemcpy(dv, v.data(), sizeof(double) * P->npad, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        launch_matvec_f64(P->stream, P->xtype, P->XT, P->npad, P->p, P->n, dv, const_cast<double *>(P->an.g0));
        e = hipStreamSynchronize(P->stream);
    }
    (void)hipFree(dv);
    if (e != hipSuccess) return fail(KBNB_E_DEVICE, "anchor gradient failed: %s", hipGetErrorString(e));
    return 0;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point: a file-scope device array of
// fixed size, one copy per device, its address looked up once per device.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char *> g_scratch_ptr;  // device -> address of its copy

// Called with `dev` current (create_problem).
static int scratch_for_device(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(KBNB_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, (unsigned char *)ptr).first;
    }
    *out = it->second;
    return 0;
}

// ---------------------------------------------------------------------------
// Process-wide device budget and shared stream pool (per device).  Every
// problem's arena is charged against its device's budget at create_problem
// and released at destroy_problem; a problem that does not fit shrinks its
// automatic batch width, waits for releases (admit_timeout_ms) or is refused.
// ---------------------------------------------------------------------------
struct DeviceShare {
    uint64_t budget = 0;  // 0: unlimited
    uint64_t used = 0;
    int pool_size = 0;    // 0: one stream per problem
    std::vector<hipStream_t> pool;
    int pool_next = 0;
};
static std::mutex g_dev_mu;
static std::condition_variable g_dev_cv;
static std::map<int, DeviceShare> g_dev;

extern "C" int device_budget(int64_t bytes, int64_t *used)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(KBNB_E_NO_DEVICE, "no HIP device is visible");
    std::lock_guard<std::mutex> g(g_dev_mu);
    DeviceShare &D = g_dev[dev];
    if (bytes >= 0) D.budget = (uint64_t)bytes;
    if (used) *used = (int64_t)D.used;
    g_dev_cv.notify_all();  // a larger budget may admit waiting problems
    return KBNB_OK;
}

extern "C" int engine_streams(int32_t count)
{
    if (count < 0 || count > 64) return fail(KBNB_E_INVALID_ARGUMENT, "stream count %d outside [0, 64]", count);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(KBNB_E_NO_DEVICE, "no HIP device is visible");
    std::lock_guard<std::mutex> g(g_dev_mu);
    g_dev[dev].pool_size = count;
    return KBNB_OK;
}

// The problem's stream: its own, or the next of the device's shared pool.
static int take_stream(kbnb_problem *P)
{
    std::lock_guard<std::mutex> g(g_dev_mu);
    DeviceShare &D = g_dev[P->device];
    if (D.pool_size <= 0) {
        P->own_stream = true;
        return hipStreamCreate(&P->stream) == hipSuccess ? 0 : -1;
    }
    while ((int)D.pool.size() < D.pool_size) {
        hipStream_t st = nullptr;
        if (hipStreamCreate(&st) != hipSuccess) return -1;
        D.pool.push_back(st);  // pool streams live until the process ends
    }
    P->stream = D.pool[(size_t)(D.pool_next++ % D.pool_size)];
    P->own_stream = false;
    return 0;
}

static void release_charge(kbnb_problem *P)
{
    if (!P->charged) return;
    std::lock_guard<std::mutex> g(g_dev_mu);
    DeviceShare &D = g_dev[P->device];
    D.used -= std::min<uint64_t>(D.used, P->charged);
    P->charged = 0;
    g_dev_cv.notify_all();
}

// ---------------------------------------------------------------------------
// create / destroy
// ---------------------------------------------------------------------------
static int device_ok()
{
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0)
        return fail(KBNB_E_NO_DEVICE, "no HIP device is visible");
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(KBNB_E_NO_DEVICE, "hipGetDeviceProperties failed");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(KBNB_E_NO_DEVICE, "device %s is not gfx950", prop.gcnArchName);
    return 0;
}

static void free_problem(kbnb_problem *P)
{
    if (!P) return;
    if (P->worker.joinable()) {
        {
            std::lock_guard<std::mutex> g(P->mu);
            P->shutdown = true;
        }
        P->cv_work.notify_all();
        P->worker.join();
    }
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    for (Variant &v : P->var)
        if (v.graph) (void)hipGraphExecDestroy(v.graph);
    if (P->gstream) (void)hipStreamSynchronize(P->gstream);
    for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : P->ev_round)
        if (e) (void)hipEventDestroy(e);
    if (P->arena) (void)hipFree(P->arena);
    void *pins[] = {P->stage_h, P->slot_host, P->h_gslots, P->h_gbuf, P->h_gbuf_lb};
    for (void *q : pins)
        if (q) (void)hipHostFree(q);
    if (P->sstream) (void)hipStreamSynchronize(P->sstream);
    if (P->sev) (void)hipEventDestroy(P->sev);
    if (P->sbuf) (void)hipFree(P->sbuf);
    if (P->spin) (void)hipHostFree(P->spin);
    if (P->sstream) (void)hipStreamDestroy(P->sstream);
    if (P->gstream) (void)hipStreamDestroy(P->gstream);
    if (P->stream && P->own_stream) (void)hipStreamDestroy(P->stream);
    release_charge(P);
    delete P;
}

extern "C" int create_problem(const kbnb_problem_desc *d, kbnb_problem **out)
{
    if (!d || !out) return fail(KBNB_E_INVALID_ARGUMENT, "NULL argument");
    *out = nullptr;
    if (d->n <= 0 || d->p <= 0 || d->k <= 0 || d->k > d->p)
        return fail(KBNB_E_INVALID_ARGUMENT, "need n > 0, 0 < k <= p (n=%d p=%d k=%d)", d->n, d->p, d->k);
    if (d->p > 8192) return fail(KBNB_E_INVALID_ARGUMENT, "p=%d exceeds the supported maximum 8192", d->p);
    if (d->k > 128) return fail(KBNB_E_INVALID_ARGUMENT, "k=%d exceeds the supported maximum 128", d->k);
    if (d->loss != KBNB_LOSS_SQUARED && d->loss != KBNB_LOSS_LOGISTIC)
        return fail(KBNB_E_INVALID_ARGUMENT, "unknown loss %d", d->loss);
    if (!(d->lambda2 > 0) || !std::isfinite(d->lambda2) || !(d->M > 0) || !std::isfinite(d->M))
        return fail(KBNB_E_INVALID_ARGUMENT, "lambda2 and M must be finite and positive");
    if (d->x_dtype < 0 || d->x_dtype > 2) return fail(KBNB_E_INVALID_ARGUMENT, "unknown x_dtype %d", d->x_dtype);
    if (d->mem_flags < 0 || d->mem_flags > 2) return fail(KBNB_E_INVALID_ARGUMENT, "unknown mem_flags %d", d->mem_flags);
    if (!d->X || !d->y) return fail(KBNB_E_INVALID_ARGUMENT, "X and y must be given");
    if (d->ldx < d->p) return fail(KBNB_E_INVALID_ARGUMENT, "ldx=%lld < p", (long long)d->ldx);
    if (d->batch_width < 0 || d->batch_width > 4096) return fail(KBNB_E_INVALID_ARGUMENT, "batch_width out of range");
    if (d->cert_period < 0 || d->cert_period > 1000) return fail(KBNB_E_INVALID_ARGUMENT, "cert_period out of range");
    if (d->iter_dtype < KBNB_ITER_AUTO || d->iter_dtype > KBNB_ITER_ANCHORED)
        return fail(KBNB_E_INVALID_ARGUMENT, "unknown iter_dtype %d", d->iter_dtype);
    if ((d->iter_dtype == KBNB_ITER_F32 || d->iter_dtype == KBNB_ITER_ANCHORED) &&
        d->x_dtype == KBNB_DTYPE_F64)
        return fail(KBNB_E_INVALID_ARGUMENT, "a float32 iteration needs float32 or bfloat16 X");
    if (d->tile_rows != 0 && d->tile_rows != 32 && d->tile_rows != 64 && d->tile_rows != 128 && d->tile_rows != 256)
        return fail(KBNB_E_INVALID_ARGUMENT, "tile_rows %d is not 0, 32, 64, 128 or 256", d->tile_rows);
    if (d->split_rows < 0) return fail(KBNB_E_INVALID_ARGUMENT, "negative split_rows");
    if (d->reopt_groups < 0 || d->reopt_groups > 1024)
        return fail(KBNB_E_INVALID_ARGUMENT, "reopt_groups %d is not in [0, 1024]", d->reopt_groups);
    int rc = device_ok();
    if (rc) return rc;
    // device inputs were produced on the caller's stream: wait for that work
    // before any copy or kernel of this library reads them
    if (d->mem_flags != KBNB_MEM_HOST_COPY && d->hip_stream) {
        hipError_t e = hipStreamSynchronize((hipStream_t)d->hip_stream);
        if (e != hipSuccess) return fail(KBNB_E_DEVICE, "synchronising the caller's stream failed: %s", hipGetErrorString(e));
    }
    if (d->mem_flags == KBNB_MEM_HOST_COPY) {
        for (int i = 0; i < d->n; ++i) {
            const double yi = d->y[i];
            if (!std::isfinite(yi)) return fail(KBNB_E_INVALID_ARGUMENT, "y[%d] is not finite", i);
            if (d->loss == KBNB_LOSS_LOGISTIC && yi != 1.0 && yi != -1.0)
                return fail(KBNB_E_INVALID_ARGUMENT, "logistic y[%d]=%g is not +-1", i, yi);
        }
    }

    kbnb_problem *P = new kbnb_problem();
    (void)hipGetDevice(&P->device);
    rc = scratch_for_device(P->device, &P->scratch);
    if (rc) { delete P; return rc; }
    P->n = d->n; P->p = d->p; P->k = d->k; P->loss = d->loss;
    P->lambda2 = d->lambda2; P->M = d->M;
    P->xtype = d->x_dtype;
    // AUTO: float64 products for float64 X; otherwise anchored for the
    // squared loss (plain float32 stalls near a 1e-6 gap there) and for tall
    // instances, plain float32 for the rest
    P->iter_f64 = (d->x_dtype == KBNB_DTYPE_F64) || (d->iter_dtype == KBNB_ITER_F64);
    P->anchored = !P->iter_f64 && (d->iter_dtype == KBNB_ITER_ANCHORED ||
                                   (d->iter_dtype == KBNB_ITER_AUTO &&
                                    (d->loss == KBNB_LOSS_SQUARED || d->n > 10000)));
    P->ti_bytes = P->iter_f64 ? 8 : 4;
    P->ldp = (int)round_up(P->p, 16);
    while (P->pp < P->p) P->pp *= 2;
    P->npad = (int)round_up(P->n, 64);
    P->pm = (int)round_up(P->ldp, 64);
    P->planes = (d->x_dtype == KBNB_DTYPE_BF16) && !P->iter_f64;
    if (d->tile_rows && (P->planes ? d->tile_rows < 64 : d->tile_rows > 64)) {
        const int tr = d->tile_rows;
        delete P;
        return fail(KBNB_E_INVALID_ARGUMENT,
                    "tile_rows %d does not apply: 32 or 64 for the per-tile contractions, 64, 128 or 256 "
                    "for the streaming ones (bfloat16 X with a float32 or anchored iteration)", tr);
    }
    P->tile_rows = d->tile_rows;
    P->split_rows = d->split_rows;
    P->reopt_groups = d->reopt_groups;
    if (P->planes) {
        P->nb = P->anchored ? 2 : 3;
        P->nkb_x = (P->ldp + 127) / 128;
        P->nkb_xt = (P->npad + 127) / 128;
    }
    // per-row-tile loss sums of the certificate: sized for 32-row tiles (the
    // arena is zeroed, so rows a 64-row launch does not write stay zero)
    P->tiles_n = P->npad / 32;
    P->cert_period = d->cert_period ? d->cert_period : 8;
    P->budget = d->hbm_budget_bytes ? d->hbm_budget_bytes : (8ull << 30);
    P->own_x = (d->mem_flags != KBNB_MEM_DEVICE_BORROW);
    const size_t xel = (d->x_dtype == KBNB_DTYPE_F64) ? 8 : (d->x_dtype == KBNB_DTYPE_F32 ? 4 : 2);
    const size_t xbytes = (size_t)P->npad * P->ldp * xel;
    P->rec_bytes = (int)round_up(round_up(sizeof(AdmitRec) + P->ldp, 8) + 8 * (size_t)P->ldp, 256);

    if (take_stream(P) != 0 ||
        hipEventCreateWithFlags(&P->ev_round[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_round[1], hipEventDisableTiming) != hipSuccess) {
        free_problem(P);
        return fail(KBNB_E_DEVICE, "stream or event creation failed");
    }
    // batch width from the budget
    int m = d->batch_width;
    if (m == 0) {
        P->mpad = 64; P->m = 64;
        choose_splits(P);
        const size_t fixed = (P->planes ? 4 : 2) * xbytes + (size_t)P->npad * 8 + (1 << 20);
        const size_t per = per_slot_bytes(P) + P->rec_bytes;
        int64_t cap = (P->budget > fixed) ? (int64_t)((P->budget - fixed) / per) : 0;
        if (cap < 1) {
            free_problem(P);
            return fail(KBNB_E_BUDGET_EXCEEDED, "the budget cannot hold X and one node slot");
        }
        m = std::min<int64_t>(1024, round_pow2_down(cap));
    }
    // charge the arena to the device's process-wide budget: an automatic
    // width shrinks (powers of two) to what is left; otherwise wait for
    // releases up to admit_timeout_ms, then refuse
    {
        const bool auto_width = d->batch_width == 0;
        auto set_width = [&](int mm) {
            P->m = mm;
            P->mpad = (int)round_up(mm, GEMM_BN);
            choose_splits(P);
        };
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(d->admit_timeout_ms);
        std::unique_lock<std::mutex> lk(g_dev_mu);
        size_t total = 0;
        // the widest width that fits (only the given one for a fixed width)
        auto try_admit = [&]() {
            DeviceShare &D = g_dev[P->device];
            for (int mm = m;; mm = round_pow2_down(mm - 1)) {
                set_width(mm);
                alloc_arena(P, xbytes, xel, &total);
                if (D.budget == 0 || D.used + total <= D.budget) {
                    D.used += total;
                    P->charged = total;
                    return true;
                }
                if (!auto_width || mm <= 1) return false;
            }
        };
        bool admitted = try_admit();
        while (!admitted) {
            const bool timed_out = g_dev_cv.wait_until(lk, deadline) == std::cv_status::timeout;
            admitted = try_admit();
            if (!admitted && timed_out) {
                set_width(m);
                alloc_arena(P, xbytes, xel, &total);
                const unsigned long long used = g_dev[P->device].used, bud = g_dev[P->device].budget;
                lk.unlock();
                free_problem(P);
                return fail(KBNB_E_BUDGET_EXCEEDED,
                            "the device budget has %llu of %llu bytes in use; the problem needs %zu "
                            "(waited %d ms)", used, bud, total, d->admit_timeout_ms);
            }
        }
    }
    P->slot_tag.assign(P->m, 0);
    P->slot_n0.assign(P->m, 0);
    for (int b = 0; b < P->m; ++b) P->free_slots.insert(b);
    P->occupied.assign(P->m, 0);
    P->cancelled.assign(P->m, 0);
    P->slot_t_submit.assign(P->m, 0.0);
    P->slot_t_admit.assign(P->m, 0.0);
    P->slot_round.assign(P->m, 0);

    rc = alloc_arena(P, xbytes, xel);
    if (rc) { free_problem(P); return rc; }
    if (P->own_x) {
        if (d->mem_flags == KBNB_MEM_HOST_COPY) {
            hipError_t e = hipMemcpy2D(P->X, (size_t)P->ldp * xel, d->X, (size_t)d->ldx * xel,
                                       (size_t)P->p * xel, P->n, hipMemcpyHostToDevice);
            if (e != hipSuccess) { free_problem(P); return fail(KBNB_E_DEVICE, "copying X failed: %s", hipGetErrorString(e)); }
        } else {
            hipError_t e = hipMemcpy2D(P->X, (size_t)P->ldp * xel, d->X, (size_t)d->ldx * xel,
                                       (size_t)P->p * xel, P->n, hipMemcpyDeviceToDevice);
            if (e != hipSuccess) { free_problem(P); return fail(KBNB_E_DEVICE, "copying X failed: %s", hipGetErrorString(e)); }
        }
    } else {
        if (d->ldx != P->ldp) { free_problem(P); return fail(KBNB_E_INVALID_ARGUMENT, "DEVICE_BORROW needs ldx == %d", P->ldp); }
        P->X = const_cast<void *>(d->X);
    }
    {
        hipError_t e = hipMemcpy(P->y, d->y, sizeof(double) * P->n,
                                 d->mem_flags == KBNB_MEM_HOST_COPY ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice);
        if (e != hipSuccess) { free_problem(P); return fail(KBNB_E_DEVICE, "copying y failed: %s", hipGetErrorString(e)); }
    }
    launch_transpose(P->stream, P->xtype, P->X, P->XT, P->n, P->p, P->ldp, P->npad, P->pm);
    if (P->planes) {
        // rows of X past n are zero in the (cleared) arena; a borrowed X may
        // hold only n rows
        launch_tile_bf16(P->stream, (const uint16_t *)P->X, P->ldp, P->n, P->ldp, P->xtile);
        launch_tile_bf16(P->stream, (const uint16_t *)P->XT, P->npad, P->pm, P->npad, P->xttile);
    }
    if (hipStreamSynchronize(P->stream) != hipSuccess) { free_problem(P); return fail(KBNB_E_DEVICE, "transpose failed"); }
    // pinned host mirrors
    {
        const size_t mb = P->mpad;
        bool okp = hipHostMalloc((void **)&P->stage_h, 2 * mb * P->rec_bytes, 0) == hipSuccess &&
                   hipHostMalloc((void **)&P->slot_host, 2 * P->slot_bytes, 0) == hipSuccess &&
                   hipHostMalloc((void **)&P->h_gslots, mb * 4, 0) == hipSuccess &&
                   hipHostMalloc((void **)&P->h_gbuf, mb * P->p * 8, 0) == hipSuccess &&
                   hipHostMalloc((void **)&P->h_gbuf_lb, mb * P->p * 8, 0) == hipSuccess;
        if (okp) {
            for (int q = 0; q < 2; ++q) {
                char *hb = P->slot_host + (size_t)q * P->slot_bytes;
                auto view = [&](const void *dev) { return hb + ((const char *)dev - P->slot_dev); };
                HostSlots &h = P->hs[q];
                h.status = (int32_t *)view(P->ss.status);
                h.iter = (int32_t *)view(P->ss.iter);
                h.jstar = (int32_t *)view(P->ss.jstar);
                h.slen = (int32_t *)view(P->ss.slen);
                h.sup = (int32_t *)view(P->ss.sup);
                h.lb = (double *)view(P->ss.lb);
                h.phi = (double *)view(P->ss.phi);
                h.gap = (double *)view(P->ss.gap);
            }
        }
        if (!okp) { free_problem(P); return fail(KBNB_E_OUT_OF_MEMORY, "pinned host allocation failed"); }
    }
    // all slots start empty
    {
        std::vector<int32_t> empty(P->mpad, SLOT_EMPTY);
        if (hipMemcpy(P->ss.status, empty.data(), 4 * P->mpad, hipMemcpyHostToDevice) != hipSuccess) {
            free_problem(P);
            return fail(KBNB_E_DEVICE, "slot init failed");
        }
    }
    rc = estimate_L(P);
    if (rc) { free_problem(P); return rc; }
    if (P->anchored) {
        rc = anchor_grad0(P);
        if (rc) { free_problem(P); return rc; }
    }
    P->c.n = P->n; P->c.p = P->p; P->c.k = P->k; P->c.loss = P->loss;
    P->c.ldp = P->ldp; P->c.npad = P->npad; P->c.pm = P->pm; P->c.mpad = P->mpad; P->c.m = P->m;
    P->c.pp = P->pp;
    P->c.lambda2 = P->lambda2; P->c.M = P->M; P->c.eta = P->eta;
    P->c.mact = P->mpad;
    P->c.xtile = P->xtile; P->c.xttile = P->xttile;
    P->c.nkb_x = P->nkb_x; P->c.nkb_xt = P->nkb_xt;
    P->c.yp = P->yp; P->c.rp = P->rp; P->c.nb = P->nb;
    P->c.tile_rows = P->tile_rows;
    for (Variant &v : P->var) build_graph(P, v);
    if (hipStreamSynchronize(P->stream) != hipSuccess) { free_problem(P); return fail(KBNB_E_DEVICE, "setup failed"); }
    P->worker = std::thread(engine_main, P);
    *out = P;
    return KBNB_OK;
}

namespace kbnb {
void drop_rashomon(const kbnb_problem *P);
void drop_audit(const kbnb_problem *P);
}

extern "C" int destroy_problem(kbnb_problem *P)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    kbnb::drop_rashomon(P);
    kbnb::drop_audit(P);
    free_problem(P);
    return KBNB_OK;
}

// ---------------------------------------------------------------------------
// submit / poll
// ---------------------------------------------------------------------------
static int build_state(const kbnb_problem *P, const kbnb_node_desc &nd, std::vector<int8_t> &st, int &kbar)
{
    st.assign(P->ldp, -1);
    for (int j = 0; j < P->p; ++j) st[j] = 0;
    if (nd.n_in < 0 || nd.n_out < 0) return fail(KBNB_E_INVALID_ARGUMENT, "negative set size");
    if (nd.n_in > P->k) return fail(KBNB_E_INVALID_ARGUMENT, "|J1|=%d exceeds k=%d", nd.n_in, P->k);
    if ((nd.n_in && !nd.fixed_in) || (nd.n_out && !nd.fixed_out)) return fail(KBNB_E_INVALID_ARGUMENT, "NULL index list");
    for (int r = 0; r < nd.n_in; ++r) {
        const int j = nd.fixed_in[r];
        if (j < 0 || j >= P->p) return fail(KBNB_E_INVALID_ARGUMENT, "fixed_in index %d out of range", j);
        if (st[j] != 0) return fail(KBNB_E_INVALID_ARGUMENT, "duplicate index %d", j);
        st[j] = 1;
    }
    for (int r = 0; r < nd.n_out; ++r) {
        const int j = nd.fixed_out[r];
        if (j < 0 || j >= P->p) return fail(KBNB_E_INVALID_ARGUMENT, "fixed_out index %d out of range", j);
        if (st[j] != 0) return fail(KBNB_E_INVALID_ARGUMENT, "index %d is fixed twice", j);
        st[j] = -1;
    }
    kbar = P->k - nd.n_in;
    return 0;
}

static int submit_locked(kbnb_problem *P, const kbnb_node_desc *nodes, int count)
{
    std::vector<PendingNode> staged;
    staged.reserve(count);
    for (int i = 0; i < count; ++i) {
        const kbnb_node_desc &nd = nodes[i];
        PendingNode pn;
        int rc = build_state(P, nd, pn.st, pn.kbar);
        if (rc) return fail(rc, "node %d: %s", i, g_last_error.c_str());
        if (nd.warm_start) {
            pn.warm.assign(nd.warm_start, nd.warm_start + P->p);
            for (int j = 0; j < P->p; ++j)
                if (!std::isfinite(pn.warm[j])) return fail(KBNB_E_INVALID_ARGUMENT, "node %d: warm start not finite", i);
        } else if (nd.warm_nnz > 0) {
            if (!nd.warm_idx || !nd.warm_val || nd.warm_nnz > P->p)
                return fail(KBNB_E_INVALID_ARGUMENT, "node %d: bad sparse warm start", i);
            pn.widx.assign(nd.warm_idx, nd.warm_idx + nd.warm_nnz);
            pn.wval.assign(nd.warm_val, nd.warm_val + nd.warm_nnz);
            for (int r = 0; r < nd.warm_nnz; ++r)
                if (pn.widx[r] < 0 || pn.widx[r] >= P->p || !std::isfinite(pn.wval[r]))
                    return fail(KBNB_E_INVALID_ARGUMENT, "node %d: sparse warm start entry %d out of range or not finite",
                                i, r);
        } else if (nd.warm_nnz < 0) {
            return fail(KBNB_E_INVALID_ARGUMENT, "node %d: negative warm_nnz", i);
        }
        if (std::isnan(nd.upper_bound)) return fail(KBNB_E_INVALID_ARGUMENT, "node %d: upper bound is NaN", i);
        if (nd.rel_tol < 0 || std::isnan(nd.rel_tol)) return fail(KBNB_E_INVALID_ARGUMENT, "node %d: bad rel_tol", i);
        if (nd.max_iters < 0) return fail(KBNB_E_INVALID_ARGUMENT, "node %d: negative max_iters", i);
        pn.tag = nd.tag;
        pn.t_submit = now_s();
        pn.n0 = nd.n_out;
        pn.ub = nd.upper_bound;
        pn.tol = nd.rel_tol > 0 ? nd.rel_tol : 1e-6;
        pn.max_iter = nd.max_iters > 0 ? nd.max_iters : 20000;
        pn.early = nd.stop_unprunable != 0;
        staged.push_back(std::move(pn));
    }
    {
        std::lock_guard<std::mutex> g(P->mu);
        if (P->engine_error) return fail(P->engine_error, "engine stopped: %s", P->engine_msg.c_str());
        for (auto &pn : staged) P->pending.push_back(std::move(pn));
    }
    P->cv_work.notify_all();
    return KBNB_OK;
}

extern "C" int submit_nodes(kbnb_problem *P, const kbnb_node_desc *nodes, int32_t count)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (count < 0 || (count > 0 && !nodes)) return fail(KBNB_E_INVALID_ARGUMENT, "bad node array");
    return submit_locked(P, nodes, count);
}

static int poll_impl(kbnb_problem *P, kbnb_bound_result *out, int cap, int *n_out, int32_t *supports,
                     double *betas, int timeout_us, double *betas_lb = nullptr)
{
    std::unique_lock<std::mutex> lk(P->mu);
    auto ready = [&] {
        return !P->done.empty() || P->engine_error ||
               (P->pending.empty() && P->active == 0);
    };
    if (timeout_us < 0) P->cv_done.wait(lk, ready);
    else if (timeout_us > 0) P->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    int cnt = 0;
    while (cnt < cap && !P->done.empty()) {
        DoneNode &d = P->done.front();
        out[cnt] = d.r;
        if (supports)
            for (int r = 0; r < P->k; ++r) supports[(size_t)cnt * P->k + r] = d.sup[r];
        if (betas) memcpy(betas + (size_t)cnt * P->p, d.beta.data(), sizeof(double) * P->p);
        if (betas_lb) {
            if (d.beta_lb.size() == (size_t)P->p) memcpy(betas_lb + (size_t)cnt * P->p, d.beta_lb.data(), sizeof(double) * P->p);
            else for (int j = 0; j < P->p; ++j) betas_lb[(size_t)cnt * P->p + j] = NAN;
        }
        P->done.pop_front();
        ++cnt;
    }
    *n_out = cnt;
    if (cnt == 0 && P->engine_error) return fail(P->engine_error, "engine stopped: %s", P->engine_msg.c_str());
    return cnt ? KBNB_OK : KBNB_TIMEOUT;
}

extern "C" int cancel_nodes(kbnb_problem *P)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    std::unique_lock<std::mutex> lk(P->mu);
    P->pending.clear();
    P->done.clear();
    bool any = false;
    for (int b = 0; b < P->m; ++b)
        if (P->occupied[b]) {
            P->cancelled[b] = 1;
            any = true;
        }
    if (any) P->cancel_dev = true;
    P->cv_work.notify_all();
    // the cancelled slots are stopped at the next round and retired after it
    P->cv_done.wait(lk, [&] {
        if (P->engine_error) return true;
        for (int b = 0; b < P->m; ++b)
            if (P->occupied[b] && P->cancelled[b]) return false;
        return true;
    });
    if (P->engine_error) return fail(P->engine_error, "engine stopped: %s", P->engine_msg.c_str());
    return KBNB_OK;
}

namespace kbnb {
// poll_bounds that also returns, per result, the iterate whose dual point
// gave its certified bound (NaN rows for nodes finished before keep_lb_beta)
int poll_with_lb_beta(kbnb_problem *P, kbnb_bound_result *out, int cap, int *n_out, int32_t *supports,
                      double *betas, double *betas_lb, int timeout_us)
{
    return poll_impl(P, out, cap, n_out, supports, betas, timeout_us, betas_lb);
}
// results retired from now on carry the iterate of their certified bound
void keep_lb_beta(kbnb_problem *P, bool on)
{
    std::lock_guard<std::mutex> g(P->mu);
    P->want_lb_beta = on;
}
// nodes queued, running or completed but not yet polled
bool outstanding(kbnb_problem *P)
{
    std::lock_guard<std::mutex> g(P->mu);
    return !P->pending.empty() || P->active > 0 || !P->done.empty();
}
}  // namespace kbnb

extern "C" int poll_bounds(kbnb_problem *P, kbnb_bound_result *out, int32_t cap, int32_t *n_out,
                           int32_t *supports, double *betas, int32_t timeout_us)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (!out || !n_out || cap < 0) return fail(KBNB_E_INVALID_ARGUMENT, "bad output arguments");
    return poll_impl(P, out, cap, n_out, supports, betas, timeout_us);
}

extern "C" int problem_info(kbnb_problem *P, int64_t *i_out, double *d_out)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (i_out) {
        i_out[0] = P->n; i_out[1] = P->p; i_out[2] = P->k; i_out[3] = P->m;
        i_out[4] = P->cert_period; i_out[5] = P->loss;
        i_out[6] = P->var.back().gsplit; i_out[7] = P->rounds.load();
        i_out[8] = P->iter_f64 ? KBNB_ITER_F64 : (P->anchored ? KBNB_ITER_ANCHORED : KBNB_ITER_F32);
        // resolved tile height and split depth of the full-width launches
        const Variant &v = P->var.back();
        int tr = P->tile_rows;
        if (!tr) {  // the forward launch's rule
            if (P->planes) tr = 4 * stream_wave_rows(0, P->npad, v.mact / GEMM_BN, 1);
            else tr = ((int64_t)(P->npad / 64) * (v.mact / GEMM_BN) < 512) ? 32 : 64;
        }
        i_out[9] = tr;
        i_out[10] = v.gchunk;
    }
    if (d_out) {
        d_out[0] = P->L; d_out[1] = P->lambda2; d_out[2] = P->M; d_out[3] = (double)P->bytes;
    }
    return KBNB_OK;
}

// ---------------------------------------------------------------------------
// step-level entry points (synchronous, own stream and buffers)
// ---------------------------------------------------------------------------
struct TmpStream {
    hipStream_t s = nullptr;
    std::vector<void *> bufs;
    ~TmpStream()
    {
        if (s) (void)hipStreamSynchronize(s);
        for (void *b : bufs) (void)hipFree(b);
        if (s) (void)hipStreamDestroy(s);
    }
    template <typename T> int alloc(T **p, size_t count)
    {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
            return fail(KBNB_E_OUT_OF_MEMORY, "hipMalloc failed");
        bufs.push_back(q);
        *p = (T *)q;
        return 0;
    }
};

static int check_states(const kbnb_problem *P, int m, const int8_t *states, std::vector<int8_t> &st,
                        std::vector<int32_t> &kbar)
{
    st.assign((size_t)m * P->ldp, -1);
    kbar.assign(m, 0);
    for (int b = 0; b < m; ++b) {
        int nin = 0;
        for (int j = 0; j < P->p; ++j) {
            const int8_t s = states[(size_t)b * P->p + j];
            if (s < -1 || s > 1) return fail(KBNB_E_INVALID_ARGUMENT, "state value %d", (int)s);
            st[(size_t)b * P->ldp + j] = s;
            nin += (s == 1);
        }
        if (nin > P->k) return fail(KBNB_E_INVALID_ARGUMENT, "node %d fixes %d > k indices in", b, nin);
        kbar[b] = P->k - nin;
    }
    return 0;
}

extern "C" int prox_batch(kbnb_problem *P, int32_t m, const int8_t *states, const double *u, double eta,
                          double *beta_out)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (m <= 0 || !states || !u || !beta_out || !(eta > 0))
        return fail(KBNB_E_INVALID_ARGUMENT, "bad prox_batch arguments");
    std::lock_guard<std::mutex> g(P->api_mu);
    std::vector<int8_t> st;
    std::vector<int32_t> kbar;
    int rc = check_states(P, m, states, st, kbar);
    if (rc) return rc;
    std::vector<double> uh((size_t)m * P->ldp, 0.0);
    for (int b = 0; b < m; ++b)
        for (int j = 0; j < P->p; ++j) uh[(size_t)b * P->ldp + j] = u[(size_t)b * P->p + j];
    TmpStream T;
    HIP_TRY(hipStreamCreate(&T.s));
    double *dU, *dB;
    int8_t *dst;
    int32_t *dk;
    if ((rc = T.alloc(&dU, uh.size())) || (rc = T.alloc(&dB, uh.size())) || (rc = T.alloc(&dst, st.size())) ||
        (rc = T.alloc(&dk, (size_t)m)))
        return rc;
    HIP_TRY(hipMemcpyAsync(dU, uh.data(), uh.size() * 8, hipMemcpyHostToDevice, T.s));
    HIP_TRY(hipMemcpyAsync(dst, st.data(), st.size(), hipMemcpyHostToDevice, T.s));
    HIP_TRY(hipMemcpyAsync(dk, kbar.data(), (size_t)m * 4, hipMemcpyHostToDevice, T.s));
    Consts c = P->c;
    launch_prox_batch(T.s, dU, dst, dk, dB, m, eta, c);
    HIP_TRY(hipGetLastError());
    std::vector<double> bh(uh.size());
    HIP_TRY(hipMemcpyAsync(bh.data(), dB, bh.size() * 8, hipMemcpyDeviceToHost, T.s));
    HIP_TRY(hipStreamSynchronize(T.s));
    for (int b = 0; b < m; ++b)
        for (int j = 0; j < P->p; ++j) beta_out[(size_t)b * P->p + j] = bh[(size_t)b * P->ldp + j];
    return KBNB_OK;
}

extern "C" int certify_batch(kbnb_problem *P, int32_t m, const int8_t *states, const double *betas,
                             double *phi, double *psi, int32_t *supports, int32_t *branch)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (m <= 0 || !states || !betas || !phi || !psi) return fail(KBNB_E_INVALID_ARGUMENT, "bad certify_batch arguments");
    std::lock_guard<std::mutex> g(P->api_mu);
    std::vector<int8_t> st;
    std::vector<int32_t> kbar;
    int rc = check_states(P, m, states, st, kbar);
    if (rc) return rc;
    const int mpad = (int)round_up(m, GEMM_BN);
    std::vector<double> bh((size_t)mpad * P->ldp, 0.0);
    for (int b = 0; b < m; ++b)
        for (int j = 0; j < P->p; ++j) bh[(size_t)b * P->ldp + j] = betas[(size_t)b * P->p + j];
    st.resize((size_t)mpad * P->ldp, -1);
    kbar.resize(mpad, 0);
    TmpStream T;
    HIP_TRY(hipStreamCreate(&T.s));
    Consts c = P->c;
    c.mpad = mpad;
    c.m = m;
    c.mact = mpad;
    Variant v;
    splits_for(P, mpad, v);
    double *dB, *dZ, *dQ, *dQs, *dl, *dc, *dlb, *dphi;
    int8_t *dst;
    int32_t *dk, *dsup, *djs, *dslen;
    const int qsplit = v.qsplit;
    if ((rc = T.alloc(&dB, bh.size())) || (rc = T.alloc(&dZ, (size_t)mpad * P->npad)) ||
        (rc = T.alloc(&dQ, (size_t)qsplit * mpad * P->ldp)) || (rc = T.alloc(&dQs, (size_t)mpad * P->ldp)) ||
        (rc = T.alloc(&dl, (size_t)P->tiles_n * mpad)) ||
        (rc = T.alloc(&dc, (size_t)P->tiles_n * mpad)) || (rc = T.alloc(&dlb, (size_t)mpad)) ||
        (rc = T.alloc(&dphi, (size_t)mpad)) || (rc = T.alloc(&dst, st.size())) || (rc = T.alloc(&dk, (size_t)mpad)) ||
        (rc = T.alloc(&dsup, (size_t)mpad * P->k)) || (rc = T.alloc(&djs, (size_t)mpad)) ||
        (rc = T.alloc(&dslen, (size_t)mpad)))
        return rc;
    HIP_TRY(hipMemcpyAsync(dB, bh.data(), bh.size() * 8, hipMemcpyHostToDevice, T.s));
    HIP_TRY(hipMemcpyAsync(dst, st.data(), st.size(), hipMemcpyHostToDevice, T.s));
    HIP_TRY(hipMemcpyAsync(dk, kbar.data(), (size_t)mpad * 4, hipMemcpyHostToDevice, T.s));
    HIP_TRY(hipMemsetAsync(dQ, 0, (size_t)qsplit * mpad * P->ldp * 8, T.s));
    HIP_TRY(hipMemsetAsync(dl, 0, (size_t)P->tiles_n * mpad * 8, T.s));
    HIP_TRY(hipMemsetAsync(dc, 0, (size_t)P->tiles_n * mpad * 8, T.s));
    SlotState ss{};
    ss.lb = dlb; ss.phi = dphi; ss.kbar = dk; ss.sup = dsup; ss.jstar = djs; ss.slen = dslen;
    launch_cert_fwd(T.s, P->xtype, P->X, dB, dZ, P->y, dl, dc, c, nullptr, nullptr);
    launch_cert_bwd(T.s, P->xtype, P->XT, dZ, dQ, qsplit, v.qchunk, c, nullptr);
    launch_cert_finish(T.s, dQ, qsplit, dl, dc, P->tiles_n, dB, nullptr, dst, ss, c, 0, Anchor{}, nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(psi, dlb, (size_t)m * 8, hipMemcpyDeviceToHost, T.s));
    HIP_TRY(hipMemcpyAsync(phi, dphi, (size_t)m * 8, hipMemcpyDeviceToHost, T.s));
    if (supports) HIP_TRY(hipMemcpyAsync(supports, dsup, (size_t)m * P->k * 4, hipMemcpyDeviceToHost, T.s));
    if (branch) HIP_TRY(hipMemcpyAsync(branch, djs, (size_t)m * 4, hipMemcpyDeviceToHost, T.s));
    HIP_TRY(hipStreamSynchronize(T.s));
    return KBNB_OK;
}

// ---------------------------------------------------------------------------
// certify_batch_noalloc: the certificate of certify_batch on device arrays,
// with every intermediate buffer in the problem device's scratch array.
// ---------------------------------------------------------------------------
// node b < mpad: pad the caller's [m][p] states and iterates into the
// [mpad][ldp] layout of the certificate kernels, count J1 and flag invalid
// states (a value outside {-1, 0, 1} or |J1| > k); clear the loss sums
__global__ __launch_bounds__(256) void k_na_pack(const int8_t *__restrict__ states, const double *__restrict__ betas,
                                                 int m, int p, int ldp, int k, int8_t *__restrict__ st,
                                                 double *__restrict__ B, int32_t *__restrict__ kbar,
                                                 int32_t *__restrict__ bad, double *__restrict__ lsum,
                                                 double *__restrict__ csum, int tiles_n, int mpad)
{
    __shared__ int s_nin;
    const int b = blockIdx.x;
    if (threadIdx.x == 0) s_nin = 0;
    __syncthreads();
    int nin = 0, inval = 0;
    for (int j = threadIdx.x; j < ldp; j += blockDim.x) {
        const bool real = b < m && j < p;
        const int s = real ? (int)states[(int64_t)b * p + j] : -1;
        const bool ok = s >= -1 && s <= 1;
        inval |= ok ? 0 : 1;
        nin += (ok && s == 1) ? 1 : 0;
        st[(int64_t)b * ldp + j] = (int8_t)(ok ? s : -1);
        B[(int64_t)b * ldp + j] = real ? betas[(int64_t)b * p + j] : 0.0;
    }
    for (int q = threadIdx.x; q < tiles_n; q += blockDim.x) {
        lsum[(int64_t)q * mpad + b] = 0.0;
        csum[(int64_t)q * mpad + b] = 0.0;
    }
    if (nin) atomicAdd(&s_nin, nin);
    inval = __syncthreads_or(inval);  // also orders the additions before the read below
    nin = s_nin;
    if (threadIdx.x == 0) {
        const bool bd = inval || nin > k;
        bad[b] = bd ? 1 : 0;
        kbar[b] = bd ? 0 : k - nin;
    }
}

// node b < m: results into the caller's arrays (NaN / -1 for an invalid node)
__global__ void k_na_unpack(int m, int k, const int32_t *__restrict__ bad, const double *__restrict__ lb,
                            const double *__restrict__ ph, const int32_t *__restrict__ sup,
                            const int32_t *__restrict__ js, double *__restrict__ phi, double *__restrict__ psi,
                            int32_t *__restrict__ sup_out, int32_t *__restrict__ br_out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m) return;
    const bool bd = bad[b] != 0;
    phi[b] = bd ? NAN : ph[b];
    psi[b] = bd ? NAN : lb[b];
    if (sup_out)
        for (int r = 0; r < k; ++r) sup_out[(int64_t)b * k + r] = bd ? -1 : sup[(int64_t)b * k + r];
    if (br_out) br_out[b] = bd ? -1 : js[b];
}

// scratch bytes certify_batch_noalloc needs for m nodes (and the pieces' offsets)
struct NaLayout {
    size_t B, Z, Q, ls, cs, st, kb, lb, ph, sup, js, sl, bad, total;
};
static NaLayout na_layout(const kbnb_problem *P, int mpad, int qsplit)
{
    NaLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += round_up(bytes, 256);
        return at;
    };
    L.B = take((size_t)mpad * P->ldp * 8);
    L.Z = take((size_t)mpad * P->npad * 8);
    L.Q = take((size_t)qsplit * mpad * P->ldp * 8);
    L.ls = take((size_t)P->tiles_n * mpad * 8);
    L.cs = take((size_t)P->tiles_n * mpad * 8);
    L.st = take((size_t)mpad * P->ldp);
    L.kb = take((size_t)mpad * 4);
    L.lb = take((size_t)mpad * 8);
    L.ph = take((size_t)mpad * 8);
    L.sup = take((size_t)mpad * P->k * 4);
    L.js = take((size_t)mpad * 4);
    L.sl = take((size_t)mpad * 4);
    L.bad = take((size_t)mpad * 4);
    L.total = o;
    return L;
}

extern "C" int certify_batch_noalloc(kbnb_problem *P, int32_t m, const int8_t *states, const double *betas,
                                     double *phi, double *psi, int32_t *supports, int32_t *branch,
                                     void *hip_stream)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (m <= 0 || !states || !betas || !phi || !psi)
        return fail(KBNB_E_INVALID_ARGUMENT, "bad certify_batch_noalloc arguments");
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : P->stream;
    {
        hipDevice_t sd = 0;
        HIP_TRY(hipStreamGetDevice(s, &sd));
        if ((int)sd != P->device)
            return fail(KBNB_E_INVALID_ARGUMENT, "the stream belongs to device %d, the problem to device %d", (int)sd,
                        P->device);
    }
    const int mpad = (int)round_up(m, GEMM_BN);
    Variant v;
    splits_for(P, mpad, v);
    const NaLayout L = na_layout(P, mpad, v.qsplit);
    if (L.total > NOALLOC_SCRATCH_BYTES)
        return fail(KBNB_E_INVALID_ARGUMENT,
                    "m=%d needs %zu bytes of scratch at n=%d, p=%d; the maximum is %zu bytes (use fewer nodes per call)",
                    m, L.total, P->n, P->p, NOALLOC_SCRATCH_BYTES);
    std::lock_guard<std::mutex> g(P->api_mu);
    unsigned char *base = P->scratch;
    double *dB = (double *)(base + L.B), *dZ = (double *)(base + L.Z), *dQ = (double *)(base + L.Q);
    double *dl = (double *)(base + L.ls), *dc = (double *)(base + L.cs);
    int8_t *dst = (int8_t *)(base + L.st);
    int32_t *dk = (int32_t *)(base + L.kb), *dsup = (int32_t *)(base + L.sup), *djs = (int32_t *)(base + L.js);
    int32_t *dsl = (int32_t *)(base + L.sl), *dbad = (int32_t *)(base + L.bad);
    double *dlb = (double *)(base + L.lb), *dph = (double *)(base + L.ph);
    Consts c = P->c;
    c.mpad = mpad;
    c.m = m;
    c.mact = mpad;
    hipLaunchKernelGGL(k_na_pack, dim3(mpad), dim3(256), 0, s, states, betas, m, P->p, P->ldp, P->k, dst, dB, dk,
                       dbad, dl, dc, P->tiles_n, mpad);
    SlotState ss{};
    ss.lb = dlb; ss.phi = dph; ss.kbar = dk; ss.sup = dsup; ss.jstar = djs; ss.slen = dsl;
    launch_cert_fwd(s, P->xtype, P->X, dB, dZ, P->y, dl, dc, c, nullptr, nullptr);
    launch_cert_bwd(s, P->xtype, P->XT, dZ, dQ, v.qsplit, v.qchunk, c, nullptr);
    launch_cert_finish(s, dQ, v.qsplit, dl, dc, P->tiles_n, dB, nullptr, dst, ss, c, 0, Anchor{}, nullptr, nullptr);
    hipLaunchKernelGGL(k_na_unpack, dim3((m + 255) / 256), dim3(256), 0, s, m, P->k, dbad, dlb, dph, dsup, djs, phi,
                       psi, supports, branch);
    HIP_TRY(hipGetLastError());
    return KBNB_OK;
}

namespace kbnb {
// Batched support re-optimisation on the problem's side stream (the engine's
// rounds continue meanwhile).  Supports: lab[off[i] .. off[i + 1]), at most
// SUPPORT_EVAL_MAX labels each, validated by the caller.  eval_supports_launch
// enqueues one batch (inputs are copied before it returns); the matching
// eval_supports_collect waits for it and copies the results out (coefs in
// the layout of lab).  One batch at a time per problem.
int eval_supports_launch(kbnb_problem *P, const int32_t *lab, const int64_t *off, int count, int maxlen,
                         const double *warm, double tol, int max_iter)
{
    if (maxlen > SUPPORT_EVAL_MAX)
        return fail(KBNB_E_INVALID_ARGUMENT, "support of %d features (at most %d)", maxlen, SUPPORT_EVAL_MAX);
    std::lock_guard<std::mutex> g(P->api_mu);
    if (P->s_count > 0) return fail(KBNB_E_INVALID_ARGUMENT, "a support batch is already in flight");
    if (count <= 0) return KBNB_OK;
    if (!P->sstream) HIP_TRY(hipStreamCreate(&P->sstream));
    if (!P->sev) HIP_TRY(hipEventCreateWithFlags(&P->sev, hipEventDisableTiming));
    const size_t C = (size_t)off[count], Cn = std::max<size_t>(C, 1), N = (size_t)count;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_lab = al(Cn * 4), b_off = al((N + 1) * 8), b_warm = al(Cn * 8), b_coef = al(Cn * 8),
                 b_val = al(N * 8), b_low = al(N * 8), b_st = al(N * 4), b_it = al(N * 4), b_clb = al(Cn * 8);
    // work area of the split-row re-optimisation (0 bytes for one workgroup per support)
    size_t b_work = 0;
    const int groups = support_eval_plan(P->xtype, P->n, count, maxlen, P->reopt_groups, &b_work);
    b_work = al(b_work);
    const size_t need = b_lab + b_off + b_warm + b_coef + b_val + b_low + b_st + b_it + b_clb + b_work;
    if (need > P->sbuf_bytes) {
        HIP_TRY(hipStreamSynchronize(P->sstream));
        if (P->sbuf) (void)hipFree(P->sbuf);
        P->sbuf = nullptr;
        P->sbuf_bytes = 0;
        const size_t want = std::max(need, (size_t)1 << 20);
        if (hipMalloc(&P->sbuf, want) != hipSuccess) return fail(KBNB_E_OUT_OF_MEMORY, "hipMalloc failed");
        P->sbuf_bytes = want;
    }
    char *b = (char *)P->sbuf;
    int32_t *dlab = (int32_t *)b; b += b_lab;
    int64_t *doff = (int64_t *)b; b += b_off;
    double *dwarm = (double *)b; b += b_warm;
    P->s_coef = (double *)b; b += b_coef;
    P->s_val = (double *)b; b += b_val;
    P->s_low = (double *)b; b += b_low;
    P->s_st = (int32_t *)b; b += b_st;
    P->s_it = (int32_t *)b; b += b_it;
    P->s_coef_lb = (double *)b; b += b_clb;
    void *dwork = b_work ? (void *)b : nullptr;
    hipStream_t s = P->sstream;
    // inputs and outputs pass through a pinned mirror of the device buffer's
    // layout: one copy each way
    const size_t in_bytes = b_lab + b_off + b_warm, out_off = in_bytes,
                 out_bytes = b_coef + b_val + b_low + b_st + b_it + b_clb;
    if (in_bytes + out_bytes > P->spin_bytes) {
        if (P->spin) (void)hipHostFree(P->spin);
        P->spin = nullptr;
        P->spin_bytes = 0;
        const size_t want = std::max(in_bytes + out_bytes, (size_t)1 << 20);
        if (hipHostMalloc((void **)&P->spin, want) != hipSuccess)
            return fail(KBNB_E_OUT_OF_MEMORY, "hipHostMalloc failed");
        P->spin_bytes = want;
    }
    memcpy(P->spin, lab, 4 * C);
    memcpy(P->spin + b_lab, off, 8 * (N + 1));
    if (warm) memcpy(P->spin + b_lab + b_off, warm, 8 * C);
    HIP_TRY(hipMemcpyAsync(dlab, P->spin, warm ? in_bytes : b_lab + b_off, hipMemcpyHostToDevice, s));
    P->s_in_bytes = in_bytes;
    P->s_out_off = out_off;
    P->s_out_bytes = out_bytes;
    SupportLaunch &SL = P->s_launch;
    SL = SupportLaunch{};
    SL.xtype = P->xtype; SL.XT = P->XT; SL.npad = P->npad; SL.n = P->n; SL.loss = P->loss; SL.y = P->y;
    SL.lab = dlab; SL.off = doff; SL.count = count; SL.maxlen = maxlen; SL.warm = warm ? dwarm : nullptr;
    SL.lambda2 = P->lambda2; SL.M = P->M; SL.tol = tol; SL.max_iter = max_iter; SL.cert_every = 10;
    SL.beta_out = P->s_coef; SL.value = P->s_val; SL.lower = P->s_low; SL.status = P->s_st; SL.iters = P->s_it;
    SL.beta_lb_out = P->s_coef_lb;
    SL.groups = groups; SL.work = dwork; SL.work_bytes = b_work;
    // split rows: as many step launches as the last batch needed to start
    // with; collect adds more until every support has finished
    P->s_steps = b_work ? std::min(max_iter + 1, P->s_steps_hint) : 0;
    const int lrc = launch_support_start(s, SL, P->s_steps);
    if (lrc == -1) return fail(KBNB_E_INVALID_ARGUMENT, "support too long");
    if (lrc != 0) return fail(KBNB_E_DEVICE, "support re-optimisation launch failed");
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(P->sev, s));
    P->s_count = count;
    P->s_coefs = (int64_t)C;
    return KBNB_OK;
}

// True when no support batch is in flight or the one in flight has reached
// its last enqueued step (eval_supports_collect then returns without waiting,
// unless split-row supports need more steps).
bool eval_supports_ready(kbnb_problem *P)
{
    std::lock_guard<std::mutex> g(P->api_mu);
    if (P->s_count == 0 || !P->sev) return true;
    return hipEventQuery(P->sev) == hipSuccess;
}

// Workgroups per support that eval_supports_launch would use for a batch of
// `count` supports of at most maxlen features.
int support_groups(kbnb_problem *P, int count, int maxlen)
{
    size_t wb = 0;
    return support_eval_plan(P->xtype, P->n, count, maxlen, P->reopt_groups, &wb);
}

int eval_supports_collect(kbnb_problem *P, double *values, double *lower, double *coefs, int32_t *status,
                          int32_t *iters, double *coefs_lb)
{
    std::lock_guard<std::mutex> g(P->api_mu);
    const size_t N = (size_t)P->s_count, C = (size_t)P->s_coefs;
    if (N == 0) return KBNB_OK;
    P->s_count = 0;
    hipStream_t s = P->sstream;
    HIP_TRY(hipEventSynchronize(P->sev));
    const SupportLaunch &SL = P->s_launch;
    if (SL.work) {
        // more step launches until every support has finished (max_iter + 1
        // of them finish all), doubling each time
        for (;;) {
            int32_t nd = 0;
            HIP_TRY(hipMemcpyAsync(&nd, support_done_counter(SL), 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (nd >= SL.count) break;
            if (P->s_steps >= SL.max_iter + 1)
                return fail(KBNB_E_DEVICE, "%d of %d supports unfinished after %d steps", SL.count - nd, SL.count,
                            P->s_steps);
            const int more = std::min(SL.max_iter + 1 - P->s_steps, std::max(32, P->s_steps));
            if (launch_support_steps(s, SL, more) != 0) return fail(KBNB_E_DEVICE, "step launch failed");
            HIP_TRY(hipGetLastError());
            P->s_steps += more;
        }
        std::vector<int32_t> it(N);
        HIP_TRY(hipMemcpyAsync(it.data(), P->s_it, 4 * N, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        P->s_steps_hint = std::max(16, 1 + *std::max_element(it.begin(), it.end()));
    }
    // every output in one copy into the pinned mirror, then to the caller
    char *pm = P->spin + P->s_out_off;
    HIP_TRY(hipMemcpyAsync(pm, P->s_coef, P->s_out_bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    auto host = [&](const void *dev) { return pm + ((const char *)dev - (const char *)P->s_coef); };
    memcpy(values, host(P->s_val), 8 * N);
    memcpy(lower, host(P->s_low), 8 * N);
    if (coefs && C) memcpy(coefs, host(P->s_coef), 8 * C);
    if (status) memcpy(status, host(P->s_st), 4 * N);
    if (iters) memcpy(iters, host(P->s_it), 4 * N);
    if (coefs_lb && C) memcpy(coefs_lb, host(P->s_coef_lb), 8 * C);
    return KBNB_OK;
}

// Blocking: one batch, launched and collected.
int eval_supports(kbnb_problem *P, const int32_t *lab, const int64_t *off, int count, int maxlen,
                  const double *warm, double tol, int max_iter, double *values, double *lower, double *coefs,
                  int32_t *status, int32_t *iters)
{
    if (count <= 0) return KBNB_OK;
    int rc = eval_supports_launch(P, lab, off, count, maxlen, warm, tol, max_iter);
    if (rc) return rc;
    return eval_supports_collect(P, values, lower, coefs, status, iters, nullptr);
}
}  // namespace kbnb

extern "C" int evaluate_supports(kbnb_problem *P, int32_t count, const int32_t *supports, double rel_tol,
                                 int32_t max_iters, double *values, double *lower_bounds, double *betas,
                                 int32_t *status, int32_t *iterations)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (count < 0 || (count > 0 && (!supports || !values || !lower_bounds)))
        return fail(KBNB_E_INVALID_ARGUMENT, "supports, values and lower_bounds are required");
    if (count == 0) return KBNB_OK;
    if (!(rel_tol >= 0.0) || max_iters < 0) return fail(KBNB_E_INVALID_ARGUMENT, "bad rel_tol or max_iters");
    const double tol = rel_tol > 0.0 ? rel_tol : 1e-9;
    const int mi = max_iters > 0 ? max_iters : 20000;
    const int k = P->k, p = P->p;
    std::vector<int32_t> lab;
    std::vector<int64_t> off(1, 0);
    std::vector<char> seen(p, 0);
    int maxlen = 0;
    for (int i = 0; i < count; ++i) {
        const int32_t *S = supports + (size_t)i * k;
        int len = 0;
        while (len < k && S[len] >= 0) ++len;
        for (int r = 0; r < len; ++r) {
            if (S[r] >= p) return fail(KBNB_E_INVALID_ARGUMENT, "support %d: index %d outside [0, %d)", i, S[r], p);
            if (seen[S[r]]) return fail(KBNB_E_INVALID_ARGUMENT, "support %d: index %d repeated", i, S[r]);
            seen[S[r]] = 1;
            lab.push_back(S[r]);
        }
        for (int r = 0; r < len; ++r) seen[S[r]] = 0;
        maxlen = std::max(maxlen, len);
        off.push_back((int64_t)lab.size());
    }
    if (maxlen > SUPPORT_EVAL_MAX)
        return fail(KBNB_E_INVALID_ARGUMENT, "supports of more than %d features", SUPPORT_EVAL_MAX);
    std::vector<double> coefs(std::max<size_t>(lab.size(), 1));
    int rc = kbnb::eval_supports(P, lab.data(), off.data(), count, maxlen, nullptr, tol, mi, values, lower_bounds,
                                 coefs.data(), status, iterations);
    if (rc) return rc;
    if (betas) {
        std::fill(betas, betas + (size_t)count * p, 0.0);
        for (int i = 0; i < count; ++i)
            for (int64_t q = off[i]; q < off[i + 1]; ++q) betas[(size_t)i * p + lab[(size_t)q]] = coefs[(size_t)q];
    }
    return KBNB_OK;
}

// Fixed-model reliance of every stored coefficient of a pool (read through
// the pool's public calls), computed on the device from the instance.
extern "C" int rashomon_reliance(kbnb_problem *P, const kbnb_pool *pool, double *reliance)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    if (!pool || !reliance) return fail(KBNB_E_INVALID_ARGUMENT, "pool and reliance are required");
    int64_t N = 0, T = 0, C = 0;
    int rc = pool_info(pool, &N, &T, &C);
    if (rc) return rc;
    if (N == 0) return KBNB_OK;
    if (N > (int64_t)INT32_MAX) return fail(KBNB_E_INVALID_ARGUMENT, "too many records");
    std::vector<int32_t> parent((size_t)T), label((size_t)T), end((size_t)N);
    std::vector<int64_t> off((size_t)N + 1);
    std::vector<double> coef((size_t)std::max<int64_t>(C, 1));
    rc = pool_export(pool, parent.data(), label.data(), end.data(), nullptr, off.data(), coef.data());
    if (rc) return rc;
    // labels of every record in path order (root first), the order of its coefficients
    std::vector<int32_t> lab((size_t)std::max<int64_t>(C, 1));
    for (int64_t m = 0; m < N; ++m) {
        int64_t r = off[(size_t)m + 1];
        for (int32_t v = end[(size_t)m]; v > 0; v = parent[(size_t)v]) {
            const int32_t j = label[(size_t)v];
            if (j < 0 || j >= P->p)
                return fail(KBNB_E_INVALID_ARGUMENT, "record %lld holds feature %d outside [0, %d)", (long long)m, j,
                            P->p);
            lab[(size_t)--r] = j;
        }
    }
    std::lock_guard<std::mutex> g(P->api_mu);
    TmpStream Ts;
    HIP_TRY(hipStreamCreate(&Ts.s));
    int32_t *dlab;
    int64_t *doff;
    double *dcoef, *dout;
    if ((rc = Ts.alloc(&dlab, (size_t)std::max<int64_t>(C, 1))) || (rc = Ts.alloc(&doff, (size_t)N + 1)) ||
        (rc = Ts.alloc(&dcoef, (size_t)std::max<int64_t>(C, 1))) || (rc = Ts.alloc(&dout, (size_t)std::max<int64_t>(C, 1))))
        return rc;
    HIP_TRY(hipMemcpyAsync(dlab, lab.data(), sizeof(int32_t) * (size_t)C, hipMemcpyHostToDevice, Ts.s));
    HIP_TRY(hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * ((size_t)N + 1), hipMemcpyHostToDevice, Ts.s));
    HIP_TRY(hipMemcpyAsync(dcoef, coef.data(), sizeof(double) * (size_t)C, hipMemcpyHostToDevice, Ts.s));
    launch_reliance(Ts.s, P->xtype, P->XT, P->npad, P->n, P->loss, P->y, dlab, doff, dcoef, (int)N, dout);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(reliance, dout, sizeof(double) * (size_t)C, hipMemcpyDeviceToHost, Ts.s));
    HIP_TRY(hipStreamSynchronize(Ts.s));
    return KBNB_OK;
}

extern "C" int kernel_stats(kbnb_problem *P, int32_t mode, double *out)
{
    if (!P) return fail(KBNB_E_BAD_HANDLE, "NULL problem");
    std::lock_guard<std::mutex> g(P->mu);
    if (out) {
        for (int i = 0; i < 8; ++i) {
            out[i] = P->kt_ms[i];
            out[8 + i] = (double)P->kt_n[i];
        }
        out[16] = P->useful_cols;
        out[17] = P->running_cols;
    }
    if (mode == 1) {
        for (int i = 0; i < 8; ++i) { P->kt_ms[i] = 0; P->kt_n[i] = 0; }
        P->useful_cols = P->running_cols = 0;
        P->timing = true;
    } else if (mode == 0) {
        P->timing = false;
    }
    return KBNB_OK;
}
