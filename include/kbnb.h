/*
 * kbnb.h -- C ABI of the batched node-bound library for cardinality-
 * constrained GLMs on AMD Instinct MI355X (gfx950).
 *
 * Problem (paper, Sec. 1, eqs. intro_sparse_glm / intro_sparse_glm_mip):
 *     min_beta  sum_i l(x_i^T beta, y_i) + lambda2 ||beta||_2^2
 *     s.t.      ||beta||_0 <= k,  ||beta||_inf <= M,
 * with the squared loss l = (y - s)^2 or the logistic loss
 * l = log(1 + exp(-y s)), y in {-1, +1}.
 *
 * A branch-and-bound node fixes some support indicators: a fixed-in set J1
 * (z_j = 1) and a fixed-out set J0 (z_j = 0); the rest are free (Sec. 3).  For
 * each node the library computes the perspective-relaxation lower bound of
 * Sec. 3 (eq. node_composite) by accelerated proximal gradient over a whole
 * batch of nodes at once (Sec. 4.2, eq. pgd_step_matrix_form), certified in
 * float64 by the Fenchel dual (eqs. prelim_fenchel_dual,
 * batched_dual_value_component): every reported lower bound is a value of
 * the dual function at some dual point, so it never exceeds the node's
 * optimum.  Rounding and branching outputs follow Sec. 4.3 (after Thm. 4.1).
 *
 * Conventions
 *  - Every call returns 0 (KBNB_OK) on success or a negative KBNB_E* code;
 *    last_error() then describes the failure.  poll_bounds may return
 *    KBNB_TIMEOUT (positive, not an error).
 *  - Indices are 0-based int32.  Matrices are row-major.
 *  - The caller owns every array it passes and may free it when the call
 *    returns, except device arrays given with KBNB_MEM_DEVICE_BORROW, which
 *    must outlive the problem.  Results are written into caller buffers.
 *  - A problem handle is owned by the library until destroy_problem.  Calls
 *    on one handle are serialised internally; different handles are
 *    independent and may be used from different threads.
 *  - Errors are atomic: a call that fails admits or changes nothing.
 */
#ifndef KBNB_H
#define KBNB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define KBNB_OK 0
#define KBNB_TIMEOUT 1             /* poll_bounds: nothing completed in time */
#define KBNB_E_INVALID_ARGUMENT (-1)
#define KBNB_E_OUT_OF_MEMORY (-2)
#define KBNB_E_BUDGET_EXCEEDED (-3) /* the problem can never fit its HBM budget */
#define KBNB_E_DEVICE (-4)          /* a HIP runtime call failed */
#define KBNB_E_BAD_HANDLE (-5)
#define KBNB_E_NO_DEVICE (-6)       /* no gfx950 device is visible */

/* losses */
#define KBNB_LOSS_SQUARED 0
#define KBNB_LOSS_LOGISTIC 1

/* storage type of X: the stored values define the instance exactly */
#define KBNB_DTYPE_F64 0
#define KBNB_DTYPE_F32 1
#define KBNB_DTYPE_BF16 2 /* uint16 bfloat16 bit patterns */

/* precision of the iteration's products (certificates are float64 always) */
#define KBNB_ITER_AUTO 0 /* F64 for float64 X; else ANCHORED for the squared loss or
                            n > 10000, F32 otherwise.  Plain float32 iterations can stall
                            near a 1e-6 relative gap: with the squared loss the natural
                            dual point zeta = -l'(X beta) is first-order sensitive to
                            rounding in the iterate, and float32 gradient sums over many
                            rows lose the accuracy the gap needs; the anchored iteration
                            does not have that floor. */
#define KBNB_ITER_F32 1  /* float32 (bfloat16 MFMA for bfloat16 X); needs F32 or BF16 X */
#define KBNB_ITER_F64 2  /* float64 products on any X */
#define KBNB_ITER_ANCHORED 3 /* float32 (bfloat16 MFMA for bfloat16 X) products of the change
                                since the node's last certificate, added to that certificate's
                                float64 gradient: rounding shrinks as the iterate settles, so
                                the iteration reaches float64-level gaps; needs F32 or BF16 X */

/* where X and y live */
#define KBNB_MEM_HOST_COPY 0      /* host arrays, copied at create_problem */
#define KBNB_MEM_DEVICE_COPY 1    /* device arrays, copied at create_problem */
#define KBNB_MEM_DEVICE_BORROW 2  /* device arrays; X must be row-major with ldx ==
                                     p rounded up to 16 and zero padding; kept */

/* node status */
#define KBNB_CONVERGED 0 /* (primal - lower_bound) <= rel_tol * |primal| */
#define KBNB_PRUNED 1    /* lower_bound >= upper_bound - 1e-6 * |upper_bound| */
#define KBNB_MAXITER 2   /* iteration cap reached; the bound is still valid */
#define KBNB_ERROR 3     /* non-finite iterate; the bound is the last valid one */
#define KBNB_UNPRUNABLE 4 /* stopped early (stop_unprunable): primal_value < upper_bound -
                             1e-6 |upper_bound|, so the node value is below the pruning
                             threshold and no bound can prune it; lower_bound is
                             certified but not tight */

typedef struct kbnb_problem kbnb_problem;

typedef struct {
    int32_t n, p, k;   /* rows, features, sparsity budget (1 <= k <= p) */
    int32_t loss;      /* KBNB_LOSS_* */
    double lambda2;    /* ridge weight, > 0 */
    double M;          /* box bound, > 0 */
    int32_t x_dtype;   /* KBNB_DTYPE_* */
    int32_t mem_flags; /* KBNB_MEM_* */
    const void *X;     /* n x p, row-major, leading dimension ldx (elements) */
    int64_t ldx;
    const double *y;   /* length n (logistic: entries -1 or +1) */
    void *hip_stream;  /* NULL, or the caller's hipStream_t that produced X and y
                          (DEVICE_COPY / DEVICE_BORROW): create_problem waits for
                          the work queued on it before reading them.  The library
                          then runs on its own streams. */
    uint64_t hbm_budget_bytes; /* device-memory budget of this problem; 0 = 8 GiB */
    int32_t batch_width;       /* node slots; 0 = chosen from the budget (max 1024) */
    int32_t cert_period;       /* iterations between float64 certificates; 0 = 8.  A node
                                  finishes only at a certificate, so a longer period adds
                                  steps past convergence and saves certificates: it pays
                                  where the FP64 contractions are costly next to a step
                                  (tall bfloat16 X); autotune measures periods */
    int32_t iter_dtype;        /* KBNB_ITER_*: precision of the iteration's products */
    int32_t admit_timeout_ms;  /* when the process-wide device budget (device_budget) cannot
                                  hold the problem: how long create_problem waits for other
                                  problems to release memory before KBNB_E_BUDGET_EXCEEDED
                                  (0: refuse at once) */
    int32_t tile_rows;         /* row height of the iteration's contraction tiles: 0 = chosen
                                  by launch size; 32 or 64 for the per-tile MFMA kernels, 64,
                                  128 or 256 for the streaming kernel of bfloat16 X with a
                                  float32 or anchored iteration (autotune chooses it) */
    int32_t split_rows;        /* rows of X per split-K part of X^T R: 0 = chosen by launch
                                  size; raised where it would give more than 32 parts */
    int32_t reopt_groups;      /* workgroups per support in the support re-optimisation
                                  (evaluate_supports, branch_and_bound), at most 1024: 0 =
                                  chosen from n and the batch size; 1 = one workgroup per
                                  support; g >= 2 = g workgroups (at most n) sharing the
                                  support's rows, one launch per step */
} kbnb_problem_desc;

typedef struct {
    uint64_t tag;               /* returned unchanged in the result */
    int32_t n_in;               /* |J1| <= k */
    const int32_t *fixed_in;    /* J1, distinct indices in [0, p) */
    int32_t n_out;              /* |J0| */
    const int32_t *fixed_out;   /* J0, disjoint from J1 */
    const double *warm_start;   /* NULL or length p (J0 entries are ignored) */
    double upper_bound;         /* incumbent for pruning; +inf = solve to rel_tol */
    double rel_tol;             /* 0 -> 1e-6 */
    int32_t max_iters;          /* 0 -> 20000 */
    int32_t stop_unprunable;    /* nonzero: stop with KBNB_UNPRUNABLE as soon as a
                                   certificate shows that the node cannot be pruned
                                   by a finite upper_bound (branch and bound only
                                   needs to branch it) */
    int32_t warm_nnz;           /* sparse warm start, used when warm_start is NULL: */
    const int32_t *warm_idx;    /*   warm_nnz distinct indices in [0, p) and their */
    const double *warm_val;     /*   finite values (J0 entries are ignored) */
} kbnb_node_desc;

typedef struct {
    uint64_t tag;
    double lower_bound;   /* certified float64 dual value, <= the node optimum */
    double primal_value;  /* float64 primal value of the returned iterate */
    double rel_gap;       /* (primal_value - lower_bound) / max(|primal_value|, 1e-12) */
    int32_t status;       /* KBNB_CONVERGED / PRUNED / MAXITER / ERROR / UNPRUNABLE */
    int32_t iterations;
    int32_t branch_index; /* argmax of |beta_j| over free j (lowest index on ties); -1 if none */
    int32_t support_len;  /* |J1| + min(kbar, #free): length of the rounding support */
    double queue_seconds; /* submit_nodes to admission into a slot (waiting for a free slot) */
    double solve_seconds; /* admission to the end of the round that finished the node */
} kbnb_bound_result;

/*
 * device_budget -- the process-wide budget of device memory for the arenas of
 * all problems on the current device (App. E.4's memory model applied across
 * problems): bytes >= 0 sets it (0 = unlimited, the default), bytes < 0 only
 * reads.  *used (nullable) receives the bytes currently charged.  Each
 * create_problem charges its arena; destroy_problem releases it.  A problem
 * with an automatic batch width takes the widest power-of-two width that
 * fits what is left (its own hbm_budget_bytes still caps it); one that cannot
 * fit even then, or a fixed width that does not fit, waits up to its
 * admit_timeout_ms for releases and is then refused with
 * KBNB_E_BUDGET_EXCEEDED.  Lowering the budget does not evict problems.
 *
 * engine_streams -- problems created afterwards on the current device share
 * `count` streams (assigned round-robin) instead of one stream each (count
 * 0, the default): their rounds queue on fewer hardware queues.  At most 64.
 */
int device_budget(int64_t bytes, int64_t *used);
int engine_streams(int32_t count);

/*
 * create_problem -- validate the instance, copy X and y to the device in the
 * instance's storage type (plus a transposed copy for the X^T R products),
 * estimate the smoothness constant (Lanczos on X^T X, on the device), size
 * the node-slot batch from the HBM budget, and start the problem's engine.
 * Passage: Sec. 1 (problem) and App. E.4 (batch sizing from a memory budget).
 * Returns KBNB_E_INVALID_ARGUMENT for bad sizes/values, KBNB_E_BUDGET_EXCEEDED
 * if X alone does not fit the budget, KBNB_E_NO_DEVICE / KBNB_E_DEVICE for
 * runtime failures.  On success *out holds a new handle.
 */
int create_problem(const kbnb_problem_desc *desc, kbnb_problem **out);

/* destroy_problem -- cancel queued and running nodes, stop the engine, free
 * every device and host allocation of the handle.  KBNB_E_BAD_HANDLE on NULL. */
int destroy_problem(kbnb_problem *prob);

/*
 * submit_nodes -- queue `count` nodes for bounding; non-blocking.  The nodes
 * are admitted into free batch slots as they free up (continuous batching)
 * and iterate on the device until their status is final.
 * Passage: Sec. 4.1 (assemble a batch of open nodes with constraints and
 * warm starts), Sec. 3 (node = (J0, J1), kbar = k - |J1|).
 * The whole call is validated first: indices in [0, p), no duplicates,
 * J0 and J1 disjoint, |J1| <= k, finite warm start; otherwise nothing is
 * queued and KBNB_E_INVALID_ARGUMENT is returned.
 */
int submit_nodes(kbnb_problem *prob, const kbnb_node_desc *nodes, int32_t count);

/*
 * poll_bounds -- collect up to `cap` completed nodes, in completion order.
 * Waits up to timeout_us microseconds for at least one (0 = do not wait,
 * negative = wait until one completes or nothing is queued or running).
 * out[i] receives the result; *n_out the number written.  If `supports` is
 * not NULL it receives, for result i, the rounding support (J1 plus the kbar
 * largest free |beta_j|, ties to the lowest index; Sec. 4.3) sorted ascending
 * in supports[i*k .. i*k+support_len-1], the rest set to -1.  If `betas` is
 * not NULL it receives the float64 iterate of result i in betas[i*p .. +p-1]:
 * the certified iterate with the least primal value, i.e. primal_value is
 * Phi_N at exactly this point, and the support and branch_index are its
 * rounding support and largest free coordinate.
 * Returns KBNB_OK, or KBNB_TIMEOUT if nothing completed in time.
 */
int poll_bounds(kbnb_problem *prob, kbnb_bound_result *out, int32_t cap,
                int32_t *n_out, int32_t *supports, double *betas, int32_t timeout_us);

typedef struct {
    double time_limit_s;     /* 0 -> no limit */
    double rel_gap_tol;      /* stop when (UB - LB) / UB <= tol; 0 -> 1e-6 */
    double node_rel_tol;     /* per-node relative gap; 0 -> 1e-6 */
    int32_t max_fista_iters; /* per node; 0 -> 20000 */
    int64_t max_nodes;       /* 0 -> unlimited */
    double log_every_s;      /* > 0: one progress line on stderr at this period; 0 -> silent */
    int32_t rashomon;        /* nonzero: also collect the support-level Rashomon set */
    int32_t rashomon_n;      /* keep only the best N supports (0 -> all) */
    double rashomon_eps;     /* set threshold (1 + eps) Phi*, eps >= 0 */
    int32_t node_order;      /* open-node order: 0 best bound (ties: deeper, then first in),
                                1 depth first (ties: smaller bound, then first in) */
    int32_t audit;           /* nonzero: record every leaf of the explored tree with the
                                certificate of its bound (bnb_audit_leaf); costs host
                                memory of p doubles per bounded node */
    int32_t support_path;    /* how supports are re-optimised (k <= 64): 0 automatic, 1 the
                                batched re-optimisation kernel (evaluate_supports), 2 the
                                node J1 = S, J0 = rest in the node engine.  Automatic takes
                                the kernel, except on tall instances where the device
                                cannot split a support's rows over several workgroups */
} kbnb_bnb_options;

typedef struct {
    double objective;   /* incumbent value v(S) = min over supp beta in S, |beta| <= M */
    double lower_bound; /* certified global lower bound: the least bound of any
                           pruned, closed or unexplored node, capped at objective */
    double rel_gap;
    int64_t nodes;      /* nodes bounded */
    int32_t status;     /* 0 optimal (gap <= tol), 1 time limit, 2 node limit,
                           3 tree exhausted with the gap above tol (nodes that hit
                           their iteration cap leave loose, still valid, bounds) */
    int32_t support_len;
    int32_t *support;   /* caller buffer of k entries: incumbent support (ascending) */
    double *beta;       /* caller buffer of p entries (or NULL): incumbent coefficients */
    int64_t incumbent_updates;
    double seconds;
    int64_t rashomon_size; /* entries of the collected set (0 unless collecting) */
    int64_t audit_leaves;  /* leaves recorded (0 unless opts->audit) */
} kbnb_bnb_result;

/*
 * cancel_nodes -- drop every node of the problem that is queued, running, or
 * completed but not yet polled: queued nodes are removed, running ones are
 * stopped at the end of the engine's current round, and none of their
 * results is ever returned by poll_bounds.  Blocks until every cancelled
 * node has left its slot, so the handle is idle when it returns (nodes
 * submitted by other threads meanwhile are not affected).  Passage: Sec. 4.1
 * (the host owns the frontier and may discard open nodes at any time).
 * KBNB_E_BAD_HANDLE on NULL; the engine's error if it has stopped.
 */
int cancel_nodes(kbnb_problem *prob);

/*
 * branch_and_bound -- blocking branch and bound built on submit_nodes /
 * poll_bounds (Sec. 4.1, Fig. 1): the host keeps the open-node queue (best
 * bound first, or depth first with opts->node_order = 1; the reported lower
 * bound is the least bound of the whole tree in either order); each batch of
 * open nodes is bounded on the device; a node is pruned
 * when its bound reaches the incumbent; otherwise its rounding support is
 * re-optimised (Sec. 4.3) to update the incumbent, and the node is branched
 * on the free coordinate with the largest |beta_j| into z_j = 0 / z_j = 1
 * children warm-started from the parent iterate.  The problem must have no
 * node queued, running or unpolled (KBNB_E_INVALID_ARGUMENT otherwise); nodes
 * still in flight when the search stops are cancelled (cancel_nodes), so the
 * handle is idle on return.  A node that reports KBNB_ERROR fails the call
 * with KBNB_E_DEVICE.  result->support must point to k int32 entries.
 */
int branch_and_bound(kbnb_problem *prob, const kbnb_bnb_options *opts,
                     kbnb_bnb_result *result);

/*
 * bnb_audit_leaf -- leaf i (0-based, in the order the search discarded them)
 * of the last branch_and_bound on `prob` run with opts->audit.  The leaves
 * partition the explored tree's discarded subtrees: every feasible support
 * lies in exactly one leaf or was left in no open node (Sec. 4.1).  A leaf is
 * the node (J1, J0) in leaf_state (p int8: 1 in, -1 out, 0 free) with
 *   kind 0: pruned: its bound reached the pruning threshold (Sec. 3, "Safe
 *           Lower Bound and Pruning"; Sec. 4.5 in Rashomon mode),
 *   kind 1: closed: its relaxation needs no branching (budget cannot bind,
 *           or every free coordinate is zero at a tight bound),
 *   kind 2: Rashomon leaf: the support J1 (J0 = the rest), bounded by its
 *           re-optimisation's certified bound,
 *   kind 3: left unexplored when the search stopped,
 * and *bound the value the search used for it.  Its certificate is a node
 * (cert_state) that contains the leaf -- the leaf itself or an ancestor --
 * and the float64 iterate cert_beta (p entries) whose dual point
 * zeta = -l'(X cert_beta) has dual value *cert_bound = Psi_cert(zeta) >= *bound
 * (eqs. prelim_fenchel_dual, dual_candidate_vector_form): replaying Psi at
 * that point checks the bound independently of the device arithmetic.  A
 * leaf with no certificate (bound -inf) gets zero arrays and -inf.  Any
 * output pointer may be NULL.  KBNB_E_INVALID_ARGUMENT when nothing was
 * audited or i is out of range.
 */
int bnb_audit_leaf(kbnb_problem *prob, int64_t i, int32_t *kind, double *bound, int8_t *leaf_state,
                   int8_t *cert_state, double *cert_beta, double *cert_bound);

/*
 * evaluate_supports -- batched re-optimisation of supports (Sec. 4.3): for
 * support S_i, the entries supports[i * k .. i * k + k) up to the first -1
 * (distinct features in [0, p), at most 64 of them),
 *   v(S_i) = min { F(X beta) + lambda2 ||beta||^2 : supp beta in S_i,
 *                  |beta_j| <= M },
 * the relaxation of the node J1 = S_i, J0 = the rest, which is exact.  On
 * the device in float64 from the stored instance values (gathered columns,
 * accelerated proximal gradient, the dual bound of the restricted problem
 * every 10 steps; on tall instances each support's rows are split over
 * several workgroups, see reopt_groups), blocking.  Outputs per
 * support: values[i] = the objective at the returned coefficients (attained
 * there), lower_bounds[i] = a certified lower bound of v(S_i) (weak
 * duality, <= values[i]), betas (NULL or count x p: the coefficients, 0 off
 * S_i), status (NULL or count: 0 when (value - bound) <= rel_tol |value|, 2
 * at the step limit) and iterations (NULL or count).  rel_tol 0 -> 1e-9;
 * max_iters 0 -> 20000.  branch_and_bound re-optimises through the same
 * kernel when k <= 64.  KBNB_E_INVALID_ARGUMENT for an index outside
 * [0, p), a repeated index or more than 64 features.
 */
int evaluate_supports(kbnb_problem *prob, int32_t count, const int32_t *supports, double rel_tol,
                      int32_t max_iters, double *values, double *lower_bounds, double *betas,
                      int32_t *status, int32_t *iterations);

/*
 * Support-level Rashomon set (Sec. 4.5, "Rashomon-set collection"): with
 * opts->rashomon set, branch_and_bound also collects every support S with
 * |S| <= k and v(S) <= (1 + rashomon_eps) Phi* (or the best rashomon_n of
 * them).  A node is then pruned only when its bound exceeds
 * tau = min((1 + eps) UB, v_(N)) (v_(N) the N-th best value found so far),
 * and is a leaf only when no indicator is undecided (kbar = 0 or nothing
 * free); the support J1 of every leaf and every re-optimised rounding
 * support are evaluated, and those within the final threshold form the set.
 * Values are certified to the re-optimisation tolerance
 * (min(1e-7, node_rel_tol / 10) relative), so a support whose value is that
 * close to the threshold may fall on either side.
 *
 * rashomon_entry -- entry i (0-based, by value, ties by the ascending index
 * sequence) of the set collected by the last such call on `prob`:
 * support (k entries, ascending, -1 padded), its length, beta (NULL or p
 * entries: the coefficients on the support, 0 elsewhere) and v(S).  The set
 * is stored compactly (a prefix trie of the supports, one flat coefficient
 * array) and freed with the problem.  KBNB_E_INVALID_ARGUMENT when i is out
 * of range or nothing was collected.
 */
int rashomon_entry(kbnb_problem *prob, int64_t i, int32_t *support, int32_t *support_len,
                   double *beta, double *value);

/*
 * Compact pool of supports (App. "compact Rashomon pool storage", with its
 * trie figure).  A pool holds N records; record m is (end node l_m, value
 * Phi_m) in a prefix trie of T nodes: node 0 is the root, node v >= 1 has
 * parent p(v) and edge label a(v) (a feature index), and the labels on the
 * path from the root to l_m are the support's insertion sequence.  Records
 * whose sequences share a prefix share its nodes; a record's end node may
 * be an inner node when its sequence is a prefix of another's.  The
 * coefficients of record m, ordered like its path labels, are
 * c[o_m .. o_{m+1}) of one flat vector c, with o_0 = 0 and
 * o_{m+1} = o_m + |S_m| (0-based).  Trie nodes are numbered in creation
 * order.  Host-only calls: none touches the device.  A pool is owned by its
 * caller and freed with pool_destroy; calls on one pool must not overlap.
 *
 * pool_create -- a new empty pool in *out (T = 1, N = 0).
 * pool_destroy -- frees the pool (NULL is accepted).
 * pool_add -- appends a record: seq[0..len) the insertion sequence (distinct
 *   indices >= 0; len 0 is the empty support, ending at the root), coef
 *   (len values, or NULL for zeros), value Phi.  KBNB_E_INVALID_ARGUMENT for
 *   a negative or repeated index.
 * pool_info -- N, T and o_N (any pointer may be NULL).
 * pool_export -- copies p(v), a(v) (T entries each, -1 for the root), the
 *   end nodes and values (N each), the offsets (N + 1) and c (o_N); any
 *   pointer may be NULL to skip that array.
 * pool_record -- record m (0-based): its path labels (root first; seq holds
 *   at least the record's length), their count, its coefficients in the
 *   same order and its value; seq, len, coef and value may be NULL.
 *   KBNB_E_INVALID_ARGUMENT when m is out of range.
 * rashomon_pool -- a copy of the set collected by the last Rashomon call of
 *   branch_and_bound on `prob` as a new pool (records by value as in
 *   rashomon_entry, each sequence ascending); the caller destroys it.
 *   KBNB_E_INVALID_ARGUMENT when nothing was collected.
 */
typedef struct kbnb_pool kbnb_pool;
int pool_create(kbnb_pool **out);
int pool_destroy(kbnb_pool *pool);
int pool_add(kbnb_pool *pool, const int32_t *seq, int32_t len, const double *coef, double value);
int pool_info(const kbnb_pool *pool, int64_t *records, int64_t *trie_nodes, int64_t *coefs);
int pool_export(const kbnb_pool *pool, int32_t *parent, int32_t *label, int32_t *end_node,
                double *values, int64_t *offsets, double *coef);
int pool_record(const kbnb_pool *pool, int64_t m, int32_t *seq, int32_t *len, double *coef,
                double *value);
int rashomon_pool(kbnb_problem *prob, kbnb_pool **out);

/*
 * Variable importance over a pool (App. "variable importance analysis based
 * on the Rashomon set").  Record m is the model beta^(m) with its stored
 * coefficients on its labels and 0 elsewhere.
 *
 * rashomon_reliance -- fixed-model reliance of every stored coefficient,
 *   R_j^(m) = (1/n) sum_i l(y_i, eta_i - x_ij beta_j) - (1/n) sum_i l(y_i, eta_i),
 *   eta = X beta^(m): the increase of the mean loss when feature j's fitted
 *   contribution is removed and the other coefficients are kept (the paper
 *   states it for the logistic loss; the squared loss takes its own l).  It
 *   runs on the device in float64 from the stored instance values of `prob`
 *   (one workgroup per record).  reliance: caller buffer of o_N doubles laid
 *   out like the pool's coefficient vector c (entry o_m + r belongs to the
 *   r-th path label of record m); R_j^(m) = 0 for j not in S_m and is not
 *   stored.  KBNB_E_INVALID_ARGUMENT when a label is not in [0, p).
 *
 * pool_summary -- per-feature summaries over the N records, host-only, into
 *   out[9][p] (rows, each p entries): support frequency (share of records
 *   whose support holds j), mean coefficient, mean |coefficient|, share of
 *   records with a positive coefficient, coefficient minimum and maximum,
 *   and, from `reliance` (o_N entries as written by rashomon_reliance, or
 *   NULL: rows of zeros), the reliance minimum, maximum and mean.  A record
 *   without j contributes coefficient 0 and reliance 0 to every row, so the
 *   [min, max] rows are the ranges over the whole pool.  All zeros when the
 *   pool is empty.  KBNB_E_INVALID_ARGUMENT when a label is not in [0, p).
 */
int rashomon_reliance(kbnb_problem *prob, const kbnb_pool *pool, double *reliance);
int pool_summary(const kbnb_pool *pool, int32_t p, const double *reliance, double *out);

typedef struct {
    const int32_t *widths;  /* candidate batch widths; NULL -> 64, 128, ..., 2048 */
    int32_t n_widths;
    const int32_t *periods; /* candidate certificate periods; NULL -> 4, 8, 16 */
    int32_t n_periods;
    int32_t sample_nodes;   /* nodes generated when none are given; 0 -> 2 x largest width */
    int32_t max_iters;      /* per sample node; 0 -> 2000 */
    double rel_tol;         /* per sample node; 0 -> 1e-6 */
    double time_limit_s;    /* no further candidate is started after this; 0 -> 60 */
    double tie_frac;        /* rates within this fraction of the best tie; 0 -> 0.03 */
    uint64_t seed;          /* generator seed of the sample nodes */
    int32_t tune_tiles;     /* nonzero: a second stage at the chosen width and period over
                               the tile height and the split depth of the contractions */
    int32_t refresh;        /* nonzero: measure even if a choice for this shape is cached */
} kbnb_tune_options;

typedef struct {
    int32_t batch_width;    /* the choice */
    int32_t cert_period;
    double rate;            /* node bounds per second of the choice on the sample */
    int32_t trials;         /* candidates measured */
    int32_t sample_nodes;   /* nodes bounded per candidate */
    double seconds;         /* total tuning time */
    int32_t tile_rows;      /* the choice of tile height (0: the launch-size rule) */
    int32_t split_rows;     /* the choice of split depth (0: the launch-size rule) */
    int32_t cached;         /* 1: returned from the cache without measuring */
    int32_t tile_trials;    /* second-stage candidates measured */
} kbnb_tune_result;

/*
 * autotune -- choose the batch width and certificate period for a problem
 * by measurement (the batch-size sweep of App. E.4, replaced by a timed
 * search on this device).  For each candidate (width, period) a problem is
 * created from `desc` with those values, the same sample of nodes is bounded
 * (the given `nodes`, tags ignored, or `sample_nodes` generated ones with
 * |J1| ~ U{0..k/2} and |J0| ~ U{0..p/10}, disjoint uniform subsets), and the
 * rate is sample size / wall time from the first submit to the last result.
 * Candidates that exceed the budget are skipped (rate 0).  The choice is the
 * smallest width whose best rate is within tie_frac of the overall best, at
 * its fastest period.  rates (nullable) receives n_widths x n_periods rates,
 * row-major by width (0 where skipped or not reached).  desc->batch_width and
 * desc->cert_period are ignored.  With opts->tune_tiles a second stage runs
 * at the chosen width and period over the tile height (the launch-size rule
 * and the explicit heights: 32 / 64 rows, or 64 / 128 / 256 for the streaming
 * kernel) and the split depth (the rule, half and twice its rows), and picks
 * the fastest (the rule on ties within tie_frac).  The choice is cached per
 * device and shape bucket (ceil(log2 n), ceil(log2 p), X dtype, loss,
 * iteration precision) for the life of the process; a later call for the same
 * bucket returns it with cached = 1 unless opts->refresh is set.
 */
int autotune(const kbnb_problem_desc *desc, const kbnb_node_desc *nodes, int32_t count,
             const kbnb_tune_options *opts, kbnb_tune_result *result, double *rates);

/* last_error -- thread-local description of the last failing call. */
const char *last_error(void);

/* ------------------------------------------------------------------------ */
/* Step-level entry points: one step of the hot path over a batch, on the    */
/* problem's device data, without the iteration loop.  They run the same     */
/* kernels as the engine and are synchronous.  All arrays are host arrays.    */
/* ------------------------------------------------------------------------ */

/*
 * prox_batch -- beta_b = prox_{eta G_Nb}(u_b) for m nodes (Sec. 4.2,
 * "Evaluating proximal operators with non-uniform node structure";
 * eq. pgd_step_vector_form; App. B PAVA).  states: m x p int8 (0 free,
 * 1 fixed in, -1 fixed out); u, beta_out: m x p float64 (node-major).
 * eta > 0.  Uses the problem's k, lambda2 and M.
 */
int prox_batch(kbnb_problem *prob, int32_t m, const int8_t *states, const double *u,
               double eta, double *beta_out);

/*
 * certify_batch -- float64 primal and dual values for m nodes at the points
 * beta_b (Sec. 4.4, eqs. batched_dual_candidate_matrix_form,
 * batched_primal_value_component, batched_dual_value_component):
 * zeta_b = -grad F(X beta_b), phi_b = F(X beta_b) + 2 lambda2 g_Nb(beta_b),
 * psi_b = -F*(-zeta_b) - 2 lambda2 g*_Nb(X^T zeta_b / (2 lambda2)).
 * states: m x p int8; betas: m x p float64.  Outputs phi, psi: m float64;
 * supports (nullable): m x k int32 rounding supports; branch (nullable): m.
 */
int certify_batch(kbnb_problem *prob, int32_t m, const int8_t *states,
                  const double *betas, double *phi, double *psi,
                  int32_t *supports, int32_t *branch);

/*
 * certify_batch_noalloc -- certify_batch for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The same float64 certificate kernels, with every
 * intermediate buffer (padded iterates and states, the dual points zeta, the
 * split-K partials of X^T zeta, the loss sums, per-node results) in a
 * fixed-size device array of the library (64 MiB, one copy per device, held
 * until the process ends); nothing is allocated, and no host-device copy or
 * synchronisation is made: the work is enqueued on `hip_stream` (NULL: the
 * problem's own stream) and the call returns.  All arrays are device arrays
 * on the problem's device: states m x p int8 (1 in, -1 out, 0 free), betas
 * m x p float64, outputs phi and psi (m float64), supports (nullable, m x k
 * int32) and branch (nullable, m int32), with certify_batch's meaning.  A
 * node whose states hold a value outside {-1, 0, 1} or more than k fixed-in
 * entries gets phi = psi = NaN, supports -1 and branch -1.  Calls that
 * overlap on one device race on the shared array: order them on one stream.
 * KBNB_E_INVALID_ARGUMENT when the call needs more than the array holds
 * (about 8 (n + (splits + 1) p) bytes per node, rounded up to 64 nodes) or
 * the stream belongs to another device.
 */
int certify_batch_noalloc(kbnb_problem *prob, int32_t m, const int8_t *states, const double *betas,
                          double *phi, double *psi, int32_t *supports, int32_t *branch, void *hip_stream);

/* Problem facts: i_out[0..10] = n, p, k, batch width, cert period, loss,
 * split-K count at full width, engine rounds so far, iteration precision
 * (KBNB_ITER_F32 / F64 / ANCHORED as resolved), tile rows and split rows of
 * the full-width iteration contractions (as resolved); d_out[0..3] =
 * smoothness constant L, lambda2, M, device bytes in use. */
int problem_info(kbnb_problem *prob, int64_t *i_out, double *d_out);

/*
 * kernel_stats -- instrumentation of the engine's kernels (for roofline
 * reporting).  mode 1: reset the counters and time every kernel of the
 * following rounds with a hipEvent pair on the engine stream (rounds are then
 * issued as direct launches instead of the captured graph); mode 0: stop
 * timing; mode -1: leave the mode unchanged.  out (nullable, 18 doubles)
 * receives the counters before the mode change: out[0..7] total milliseconds
 * of the kernel types {forward X Y, backward X^T R, prox, certificate X B,
 * certificate X^T zeta, certificate finish, admission, (unused, 0)},
 * out[8..15] their launch counts, out[16] the sum over timed iteration
 * launches of sum_b (p - |J0_b|) over the nodes in the batch, out[17] the sum
 * over timed iteration launches of the number of nodes in the batch.
 */
int kernel_stats(kbnb_problem *prob, int32_t mode, double *out);

#ifdef __cplusplus
}
#endif
#endif /* KBNB_H */
