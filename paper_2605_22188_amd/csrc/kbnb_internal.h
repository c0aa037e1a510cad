// kbnb_internal.h -- device-buffer layout and kernel launchers of the node-bound
// engine.  Internal to libkbnb: the public interface is include/kbnb.h.
//
// Layout in HBM (all node data is node-major: element (j, b) of a p x m batch
// matrix lives at [b * ldp + j], so one node's column is contiguous):
//   X   [npad][ldp]  instance storage type, row-major, zero padding
//   XT  [pm][npad]   the transpose of X (the X^T R products read it k-contiguous)
//   Yi  [mpad][ldp]  extrapolated point in the iteration type (MFMA operand)
//   R   [mpad][npad] l'(X Y) in the iteration type
//   Gp  [gsplit][mpad][ldp] split-K partials of X^T R;  G [mpad][ldp] their sum
//   B, Bprev [mpad][ldp] float64 iterates beta^t, beta^{t-1}
//   Z   [mpad][npad] float64 dual point zeta = -l'(X beta)
//   Qp  [qsplit][mpad][ldp] float64 split-K partials of X^T zeta;  Q their sum
//   lsum, csum [tiles_n][mpad] float64 per-row-tile sums of l(X beta) and l*(-zeta)
//   st  [mpad][ldp] int8 node coordinate state (0 free, 1 in, -1 out / padding)
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace kbnb {

constexpr int SLOT_EMPTY = -2;
constexpr int SLOT_RUNNING = -1;
// final statuses match kbnb.h: 0 converged, 1 pruned, 2 maxiter, 3 error

constexpr int GEMM_BM = 64;
constexpr int GEMM_BN = 64;
constexpr int GEMM_BK = 16;

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Padded column length of the per-node kernels: the power of two >= p, at
// least 256, at most 8192.  A node runs on pp / 256 waves (at most 16), so
// every thread holds 4 coordinates (8 at pp = 8192): the per-node chain of
// sort repair, scans and block search is short, and one workgroup per node
// still keeps a thin frontier's nodes on separate CUs.
__host__ __device__ constexpr int node_waves(int pp) { return pp <= 256 ? 1 : (pp / 256 < 16 ? pp / 256 : 16); }
// Split-K partials summed per load batch by the per-node kernels (pp: the
// coordinates one wave holds; element size in bytes), sized so a batch's
// loads fit in registers.
__host__ __device__ constexpr int split_batch(int pp, int elem_bytes)
{
    return (elem_bytes == 4) ? ((pp >= 2048) ? 4 : ((pp >= 1024) ? 8 : 16))
                             : ((pp >= 2048) ? 2 : ((pp >= 1024) ? 4 : ((pp >= 512) ? 8 : 16)));
}

// Per-slot scalar state (struct of arrays, device memory).
struct SlotState {
    double *theta;    // extrapolation weight for the next step
    double *tmom;     // FISTA t_k
    double *lb;       // best certified dual value
    double *phi;      // best primal value
    double *gap;      // relative gap at the last certificate
    double *ub;       // pruning incumbent
    double *tol;      // relative tolerance
    int32_t *status;  // SLOT_EMPTY / SLOT_RUNNING / final status
    int32_t *iter;    // iterations done
    int32_t *max_iter;
    int32_t *kbar;    // k - |J1|
    int32_t *jstar;   // branching index
    int32_t *early;   // nonzero: stop once the node cannot be pruned (primal < ub)
    int32_t *slen;    // rounding-support length
    int32_t *sup;     // [mpad][k] rounding support, ascending, -1 padded
    int32_t *perm;    // [mpad][pp] sorted order of the node's |u| at its last step
    double *blb;      // [mpad][ldp] iterate whose dual point gave the best certified bound
};

// Problem constants passed by value to kernels.
struct Consts {
    int n, p, k, loss;
    int ldp, npad, pm, mpad, m;
    int mact;  // columns the launches cover (multiple of 64, <= mpad); slots beyond are empty
    int pp;  // per-node sort width: next power of two >= max(p, 256)
    double lambda2, M, eta;
    // Plane mode (bfloat16 X with the float32 or anchored iteration): the
    // iteration's contractions stream tiled copies of X and X^T (k_gemm_stream),
    // and the point Y (or D) and R are kept as nb bfloat16 planes
    // (nb = 3: float32-exact; nb = 2: a 16-bit significand, enough for the
    // anchored iteration's increments).  yp is NULL outside plane mode.
    const uint16_t *xtile, *xttile;  // k_tile_bf16 layouts of X and X^T
    int nkb_x, nkb_xt;               // their 128-wide k blocks per 16-row block
    uint16_t *yp;                    // [nb][mpad][ldp]
    uint16_t *rp;                    // [nb][mpad][npad]
    int nb;
    // tile height of the iteration's contractions (0: the launch-size rule;
    // 32 / 64 for the per-tile kernels, 128 / 256 for the streaming kernel)
    int tile_rows;
};

// Staged node for admission into a slot (host -> device).
struct AdmitRec {
    int32_t slot, kbar, max_iter, has_warm;
    double ub, tol;
    int32_t early, pad;
};

enum XType { XT_F64 = 0, XT_F32 = 1, XT_BF16 = 2 };

// Anchored float32 iteration (all pointers NULL when it is off).  Each
// node's float64 certificate at beta_c also yields the exact gradient there;
// between certificates the float32 / bfloat16 contractions act on the
// change D = Y - beta_c only:  S = S_c + X D,  R = l'(S) - l'(S_c),
// grad F(Y) = grad F(beta_c) + X^T R, so their rounding shrinks with D.
struct Anchor {
    double *sc;        // [mpad][npad] S_c = X beta_c (float64)
    double *bc;        // [mpad][ldp]  beta_c
    double *gc;        // [mpad][ldp]  grad F(beta_c) (float64)
    const double *g0;  // [ldp]        grad F(0): the anchor of a newly admitted node
};

// When `start` is set, the next launch of the calling thread records the
// kernel's own start/end timestamps in (start, stop) (instrumentation).
struct KernelTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelTiming g_ktime;

// ---- launchers (kbnb_kernels.hip) -----------------------------------------
// iteration GEMMs (Ti = float for float32/bfloat16... instances, double for float64)
// `status` (nullable) lets a GEMM tile skip when none of its 64 nodes is running
// an.sc set: Yi holds D = Y - beta_c and R = l'(S_c + X D) - l'(S_c)
void launch_fwd_dloss(hipStream_t s, int xtype, bool iter_f64, const void *X, const void *Yi,
                      void *R, const double *y, const Consts &c, const int32_t *status,
                      const Anchor &an);
void launch_bwd(hipStream_t s, int xtype, bool iter_f64, const void *XT, const void *R,
                void *Gp, int gsplit, int gchunk, const Consts &c, const int32_t *status);
// the per-node kernels sum the split-K partials themselves (plus grad F(beta_c)
// when anchored, and then write D = Y - beta_c to Yi)
void launch_prox_iter(hipStream_t s, bool iter_f64, const void *Gp, int gsplit, double *B,
                      double *Bprev, void *Yi, const int8_t *st, SlotState ss, const Consts &c,
                      const Anchor &an);
// certificate
// sc_out (nullable): also store S = X B (float64), the anchored iteration's S_c
void launch_cert_fwd(hipStream_t s, int xtype, const void *X, const double *B, double *Z,
                     const double *y, double *lsum, double *csum, const Consts &c,
                     const int32_t *status, double *sc_out);
void launch_cert_bwd(hipStream_t s, int xtype, const void *XT, const double *Z, double *Qp,
                     int qsplit, int qchunk, const Consts &c, const int32_t *status);
// Bbest (engine only, nullable when update_state is 0): receives B of a
// certificate that improves the slot's best primal value.  Anchored (an.bc
// set, engine only): the certificate becomes the slot's new anchor, and the
// next step's D = theta (B - Bprev) is written to Yi (float32).
void launch_cert_finish(hipStream_t s, const double *Qp, int qsplit, const double *lsum,
                        const double *csum, int tiles_n, const double *B, double *Bbest,
                        const int8_t *st, SlotState ss, const Consts &c, int update_state,
                        const Anchor &an, const double *Bprev, float *Yi);
// admission of staged nodes into slots
void launch_admit(hipStream_t s, bool iter_f64, const uint8_t *stage, int count, int rec_bytes,
                  double *B, double *Bprev, double *Bbest, void *Yi, int8_t *st, SlotState ss,
                  const Consts &c, const Anchor &an);
// standalone prox over a batch (u given), for the step-level entry point
void launch_prox_batch(hipStream_t s, const double *U, const int8_t *st, const int32_t *kbar,
                       double *Bout, int m, double eta, const Consts &c);
// products of the Lanczos iteration for L: out[r] = sum_c A[r][c] v[c] in float64
void launch_matvec_f64(hipStream_t s, int xtype, const void *A, int64_t lda, int rows, int cols,
                       const double *v, double *out);
// fixed-model reliance of pool records (float64): record m's labels and
// coefficients are lab/coef[off[m] .. off[m + 1]); out has the same layout
void launch_reliance(hipStream_t s, int xtype, const void *XT, int64_t npad, int n, int loss, const double *y,
                     const int32_t *lab, const int64_t *off, const double *coef, int nrec, double *out);
// Batched support re-optimisation in float64 (supports of at most 64
// features): one batch of supports lab[off[i] .. off[i + 1]) with its
// outputs (coefficients in the layout of lab).  With a work area the rows of
// each support are split over `groups` workgroups (one or more): a set-up
// launch, then one launch per step, the supports' state kept in `work`
// between them; without one, one workgroup per support runs every step.
constexpr int SUPPORT_EVAL_MAX = 64;
struct SupportLaunch {
    int xtype = 0;
    const void *XT = nullptr;
    int64_t npad = 0;
    int n = 0, loss = 0;
    const double *y = nullptr;
    const int32_t *lab = nullptr;
    const int64_t *off = nullptr;
    int count = 0, maxlen = 0;
    const double *warm = nullptr;  // nullable
    double lambda2 = 0, M = 0, tol = 0;
    int max_iter = 0, cert_every = 10;
    double *beta_out = nullptr, *value = nullptr, *lower = nullptr;
    int32_t *status = nullptr, *iters = nullptr;
    double *beta_lb_out = nullptr;  // nullable
    int groups = 1;
    void *work = nullptr;
    size_t work_bytes = 0;
};
// Workgroups per support for a batch of `count` supports of at most maxlen
// features over n rows (want: 0 automatic, 1 the one-workgroup kernel,
// g >= 2 that many); *work_bytes gets the bytes of device work area the
// step-launch kernels need (0 for the one-workgroup kernel).
int support_eval_plan(int xtype, int n, int count, int maxlen, int want, size_t *work_bytes);
// Enqueue the batch: the whole of it on the one-workgroup kernel (no work
// area); otherwise the set-up and the first `steps` step launches.  -1 for a
// support longer than SUPPORT_EVAL_MAX or a work area too small.
int launch_support_start(hipStream_t s, const SupportLaunch &L, int steps);
// with a work area: `steps` more step launches (a launch leaves finished
// supports alone; every support has finished after max_iter + 1 of them)
int launch_support_steps(hipStream_t s, const SupportLaunch &L, int steps);
// with a work area: device counter of the supports that have finished
const int32_t *support_done_counter(const SupportLaunch &L);
// Arguments of the MFMA contraction kernels (kbnb_kernels.hip):
// C[col][row] = sum_k A[row][k] * B[col][k] over the workgroup's k split.
enum { EPI_DLOSS = 0, EPI_STORE = 1, EPI_CERT = 2, EPI_DLOSS_ANCHOR = 3 };

struct GemmArgs {
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
    int64_t split_stride;  // elements between split partial buffers
    int k_len;             // total k extent (multiple of 16)
    int k_chunk;           // k per split (multiple of 16)
    int tiles_m;
    int tiles_n;
    int nsplit;
    const int32_t *col_status;  // nullable: skip tiles with no running column
    int rows_valid;        // store rows < rows_valid (EPI_STORE)
    int n;                 // rows with data (EPI_DLOSS / EPI_CERT)
    int loss;
    const double *y;
    double *lsum;          // [tiles_m][ldsum]
    double *csum;
    int64_t ldsum;
    const double *sc;      // EPI_DLOSS_ANCHOR: S_c, same layout as C
    double *sc_out;        // EPI_CERT (nullable): also store S = acc, same layout as C
    // plane operands (k_gemm_stream): element distance between the bfloat16
    // planes of A, of B and of a plane output C; row counts of A and C
    int64_t a_plane, b_plane, c_plane;
    int rows_a, rows_c;
};
// streaming contraction for bfloat16 A (one plane) against nb = 2 or 3
// bfloat16 planes of B, tile (4 wr) x 64 with wr = 16, 32 or 64 rows per wave
// (k_gemm_stream; two-plane launches with 64-row wave tiles take the variant
// with one A register set, except a split-K launch of one column tile);
// modes EPI_DLOSS, EPI_DLOSS_ANCHOR (C: nb bfloat16 planes) or EPI_STORE
// (float32 split-K partials).  Returns -1 for an unsupported combination.
int launch_gemm_stream(hipStream_t s, int mode, GemmArgs g, int rows, int tiles_n, int splits, int wr, int nb);
// wave tile height (16, 32 or 64 rows) of a streaming launch over `rows`
// rows of A: tile_rows / 4 when given, else chosen by launch size
int stream_wave_rows(int tile_rows, int rows, int tiles_n, int splits);
// tiled copy of a rows x cols bfloat16 matrix for k_gemm_stream (whose A is
// this layout, with GemmArgs::lda = ceil(cols / 128)); dst holds
// ceil(rows / 16) * 16 x ceil(cols / 128) * 128 elements
void launch_tile_bf16(hipStream_t s, const uint16_t *src, int64_t lds, int rows, int cols, uint16_t *dst);
// convert/transposed copies
void launch_transpose(hipStream_t s, int xtype, const void *X, void *XT, int n, int p, int ldp,
                      int npad, int pm);

}  // namespace kbnb
