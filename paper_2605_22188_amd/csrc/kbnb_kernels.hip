// kbnb_kernels.hip -- gfx950 kernels of the batched node-bound hot path.
//
// One FISTA step over a batch of m nodes (paper Sec. 4.2, eqs.
// gradient_matrix_form and pgd_step_matrix_form) is three launches:
//   fwd   S = X Y (MFMA), epilogue R = l'(S, y)           (forward contraction + loss)
//   bwd   G = X^T R (MFMA, split-K partials)              (backward contraction)
//   prox  per node: U = Y - eta G, masked TopSum-Huber prox, momentum/restart
// and every few steps the float64 certificate (Sec. 4.4) is three more:
//   cfwd  S = X B in float64 (MFMA f64), epilogue zeta = -l'(S), column sums of
//         l(S) and l*(-zeta)
//   cbwd  Q = X^T zeta in float64 (MFMA f64, split-K partials)
//   cfin  per node: g*(Q / 2 lambda2) by TopSum selection, g(B) in closed form,
//         primal/dual values, status, rounding support and branching index.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>

#include "kbnb_internal.h"

namespace kbnb {

thread_local KernelTiming g_ktime;

// Every launch goes through this macro: when the calling thread has set a
// timing pair, the kernel is launched with hipExtLaunchKernelGGL so that the
// events carry the kernel's own start and end timestamps.
#define KBNB_LAUNCH(KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                        \
    do {                                                                                         \
        if (g_ktime.start)                                                                       \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, g_ktime.start, g_ktime.stop, \
                                  0, __VA_ARGS__);                                               \
        else                                                                                     \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                   \
    } while (0)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct V4;
template <> struct V4<float> { typedef f32x4 t; };
template <> struct V4<double> { typedef f64x4 t; };

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Global loads of 4 consecutive elements, converted to the compute type.
// bfloat16 storage is uint16 bit patterns; the conversion is exact.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ld4(const float *p, float o[4])
{
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const float *p, double o[4])
{
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const double *p, double o[4])
{
    double2 a = *reinterpret_cast<const double2 *>(p);
    double2 b = *reinterpret_cast<const double2 *>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void ld4(const double *p, float o[4])
{
    double2 a = *reinterpret_cast<const double2 *>(p);
    double2 b = *reinterpret_cast<const double2 *>(p + 2);
    o[0] = (float)a.x; o[1] = (float)a.y; o[2] = (float)b.x; o[3] = (float)b.y;
}
__device__ __forceinline__ float bf16_to_f(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}
__device__ __forceinline__ void ld4(const uint16_t *p, float o[4])
{
    uint2 v = *reinterpret_cast<const uint2 *>(p);
    o[0] = bf16_to_f((uint16_t)(v.x & 0xffff)); o[1] = bf16_to_f((uint16_t)(v.x >> 16));
    o[2] = bf16_to_f((uint16_t)(v.y & 0xffff)); o[3] = bf16_to_f((uint16_t)(v.y >> 16));
}
__device__ __forceinline__ void ld4(const uint16_t *p, double o[4])
{
    float f[4];
    ld4(p, f);
    o[0] = f[0]; o[1] = f[1]; o[2] = f[2]; o[3] = f[3];
}

// ---------------------------------------------------------------------------
// Scalar losses (paper Sec. 4.2 separable f; Sec. 4.4 l and l*).
//   squared  l = (y - s)^2, l' = 2 (s - y), l*(v) = v y + v^2 / 4
//   logistic l = log(1 + e^{-ys}), l' = -y / (1 + e^{ys}),
//            l*(-zeta) = t log t + (1 - t) log(1 - t), t = y zeta in [0, 1]
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dloss_f(int loss, float s, float y)
{
    if (loss == 0) return 2.0f * (s - y);
    return -y / (1.0f + __expf(y * s));
}
__device__ __forceinline__ double dloss_d(int loss, double s, double y)
{
    if (loss == 0) return 2.0 * (s - y);
    return -y / (1.0 + exp(y * s));
}
__device__ __forceinline__ double loss_d(int loss, double s, double y)
{
    if (loss == 0) {
        double r = y - s;
        return r * r;
    }
    double z = -y * s;
    return fmax(z, 0.0) + log1p(exp(-fabs(z)));
}
// l*(-zeta, y)
__device__ __forceinline__ double conj_neg_d(int loss, double zeta, double y)
{
    if (loss == 0) return -zeta * y + 0.25 * zeta * zeta;
    double t = y * zeta;
    if (t < 0.0 || t > 1.0) return INFINITY;
    double a = (t > 0.0) ? t * log(t) : 0.0;
    double b = (t < 1.0) ? (1.0 - t) * log1p(-t) : 0.0;
    return a + b;
}

// Certificate terms at one entry s of X beta: zeta = -l'(s), l(s) and
// l*(-zeta).  Logistic, with z = y s, e = exp(-|z|), L1 = log1p(e):
//   t = sigma(-z) = (z >= 0 ? e : 1) / (1 + e),  zeta = y t,
//   l(s) = max(-z, 0) + L1,
//   log t = -(max(z, 0) + L1),  log(1 - t) = -(max(-z, 0) + L1),
//   l*(-zeta) = t log t + (1 - t) log(1 - t)
//             = -L1 - t max(z, 0) - (1 - t) max(-z, 0),
// one exp and one log1p per entry.
__device__ __forceinline__ void cert_terms(int loss, double s, double y, double &zeta,
                                           double &lval, double &cval)
{
    if (loss == 0) {
        const double r = y - s;
        zeta = 2.0 * r;
        lval = r * r;
        cval = -zeta * y + 0.25 * zeta * zeta;
        return;
    }
    const double z = y * s;
    const double e = exp(-fabs(z));
    const double L1 = log1p(e);
    const double t = ((z >= 0.0) ? e : 1.0) / (1.0 + e);
    zeta = y * t;
    const double zp = fmax(z, 0.0), zn = fmax(-z, 0.0);
    lval = zn + L1;
    cval = -L1 - t * zp - (1.0 - t) * zn;
}

template <typename T> __device__ __forceinline__ T dloss_t(int loss, T s, T y);
template <> __device__ __forceinline__ float dloss_t<float>(int loss, float s, float y) { return dloss_f(loss, s, y); }
template <> __device__ __forceinline__ double dloss_t<double>(int loss, double s, double y) { return dloss_d(loss, s, y); }

// ---------------------------------------------------------------------------
// MFMA contraction  C[col][row] = sum_k A[row][k] * Bm[col][k]
// over k in this workgroup's split range, both operands k-contiguous.
// Tile 64 x 64 x 16, 256 threads as 2 x 2 waves of 32 x 32 (2 x 2 MFMA
// 16x16x4 blocks).  Within a 16-wide k chunk, lane group g = lane / 16 owns
// k = 4g .. 4g+3, so each lane reads its four A (and B) values of a chunk
// with one LDS vector read; MFMA step s contracts k in {s, 4+s, 8+s, 12+s}.
// Epilogue modes:
//   EPI_DLOSS  C = l'(acc, y[row]) for row < n, 0 otherwise  (R of the step)
//   EPI_STORE  C[split] = acc for row < rows_valid            (split-K partials)
//   EPI_CERT   C = zeta = -l'(acc, y[row]) for row < n, plus per-column sums
//              of l(acc) and l*(-zeta) over this tile's rows.
// ---------------------------------------------------------------------------
// (the epilogue modes and GemmArgs are declared in kbnb_internal.h)

// XCD-aware tile order shared by the contraction kernels: workgroups are
// dealt round-robin to the 8 XCDs (blockIdx % 8), each with its own L2.
//  - split-K: every tile of one k-split goes to the same XCD, so both operand
//    chunks of the split are fetched into one L2 and read there;
//  - otherwise, with >= 8 row tiles, the column tiles of one row tile go to
//    the same XCD back to back, so the A row tile is reused from one L2.
// Returns false for a workgroup past the end of the grid.
__device__ __forceinline__ bool map_tile(const GemmArgs &g, int &tm, int &tn, int &split)
{
    if (g.nsplit > 1) {
        const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
        const int T = g.tiles_m * g.tiles_n;
        split = xcd + 8 * (q / T);
        const int t = q % T;
        // the column tiles that share a row block of A run next to each other
        // on one XCD, so its L2 serves A to all of them
        tn = t % g.tiles_n;
        tm = t / g.tiles_n;
        return split < g.nsplit;
    }
    split = 0;
    if (g.tiles_m >= 8) {
        const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
        tn = q % g.tiles_n;
        tm = (q / g.tiles_n) * 8 + xcd;
        return tm < g.tiles_m;
    }
    tm = blockIdx.x % g.tiles_m;
    tn = blockIdx.x / g.tiles_m;
    return true;
}

// Epilogues EPI_DLOSS and EPI_STORE of a BM x 64 tile whose accumulators
// acc[i][j][r] hold C at row = row0 + wm*BM/2 + i*16 + lg*4 + r,
// col = col0 + wn*32 + j*16 + lr (the layout of both the f32 and the bf16
// 16x16 MFMA, and of the f64 one after the A-row permutation).
template <typename TC, int MODE, int FI>
__device__ __forceinline__ void epi_store(const GemmArgs &g, const typename V4<TC>::t (&acc)[FI][2],
                                          const double (&yv)[FI][4], int row0, int col0, int wm,
                                          int wn, int lg, int lr, int split)
{
    typedef typename V4<TC>::t acc_t;
    constexpr int BM = FI * 32;
    if constexpr (MODE == EPI_DLOSS) {
        TC *C = reinterpret_cast<TC *>(g.C);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = col0 + wn * 32 + j * 16 + lr;
#pragma unroll
            for (int i = 0; i < FI; ++i) {
                const int rb0 = row0 + wm * (BM / 2) + i * 16 + lg * 4;
                acc_t o;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const TC d = dloss_t<TC>(g.loss, acc[i][j][r], (TC)yv[i][r]);
                    o[r] = (rb0 + r < g.n) ? d : (TC)0;
                }
                *reinterpret_cast<acc_t *>(C + (int64_t)col * g.ldc + rb0) = o;
            }
        }
    } else if constexpr (MODE == EPI_DLOSS_ANCHOR) {
        // acc = X D; S = S_c + acc and R = l'(S) - l'(S_c), formed in float64
        // (squared loss: exactly 2 acc)
        TC *C = reinterpret_cast<TC *>(g.C);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = col0 + wn * 32 + j * 16 + lr;
#pragma unroll
            for (int i = 0; i < FI; ++i) {
                const int rb0 = row0 + wm * (BM / 2) + i * 16 + lg * 4;
                acc_t o;
                if (g.loss == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = (rb0 + r < g.n) ? (TC)(2.0 * (double)acc[i][j][r]) : (TC)0;
                } else {
                    double sc[4];
                    ld4(g.sc + (int64_t)col * g.ldc + rb0, sc);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double s = sc[r] + (double)acc[i][j][r];
                        const double d = dloss_d(g.loss, s, yv[i][r]) - dloss_d(g.loss, sc[r], yv[i][r]);
                        o[r] = (rb0 + r < g.n) ? (TC)d : (TC)0;
                    }
                }
                *reinterpret_cast<acc_t *>(C + (int64_t)col * g.ldc + rb0) = o;
            }
        }
    } else {
        TC *C = reinterpret_cast<TC *>(g.C) + (int64_t)split * g.split_stride;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = col0 + wn * 32 + j * 16 + lr;
#pragma unroll
            for (int i = 0; i < FI; ++i) {
                const int rb0 = row0 + wm * (BM / 2) + i * 16 + lg * 4;
                if (rb0 + 3 < g.rows_valid) {
                    *reinterpret_cast<acc_t *>(C + (int64_t)col * g.ldc + rb0) = acc[i][j];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (rb0 + r < g.rows_valid)
                            C[(int64_t)col * g.ldc + rb0 + r] = acc[i][j][r];
                }
            }
        }
    }
}

template <typename TA, typename TB, typename TC, int MODE, int BM>
__global__ __launch_bounds__(256) void k_gemm_tn(GemmArgs g)
{
    // tile BM x 64 (BM = 32 or 64); the 4 waves form a 2 x 2 grid of
    // (BM / 2) x 32 wave tiles, i.e. FI x 2 MFMA blocks of 16 x 16
    constexpr int BN = GEMM_BN;
    constexpr int FI = BM / 32;
    // k depth of one LDS stage: 64 (float) or 32 (double) so that a stage's
    // MFMA work (64 or 32 instructions per wave) covers the next stage's
    // global-load latency.  A stage is NH sub-blocks of 16; in sub-block h
    // lane group lg holds k = 16 h + 4 lg .. + 3 (one vector LDS read), and
    // MFMA step s contracts k in {16 h + 4 g + s : g = 0..3}.
    constexpr int BK = (sizeof(TC) == 8) ? 32 : 64;
    constexpr int NH = BK / 16;
    constexpr int PAD = (sizeof(TC) == 8) ? 2 : 4;
    constexpr int LS = BK + PAD;                      // LDS row stride (elements)
    constexpr int GPR = BK / 4;                       // 4-element groups per row
    constexpr int LPA = (BM * GPR) / 256;             // A groups per thread per stage
    constexpr int LPB = (BN * GPR) / 256;             // B groups per thread per stage
    typedef typename V4<TC>::t acc_t;
    __shared__ TC As[2][BM * LS];
    __shared__ TC Bs[2][BN * LS];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lg = lane >> 4;
    // The f64 16x16x4 MFMA returns row g + 4r of its block in lane group g,
    // register r (the f32 one returns row 4g + r).  Feeding A row
    // 4 (i % 4) + i / 4 into row slot i makes both layouts "lane group g,
    // register r holds row 4g + r", so one epilogue serves both.
    const int arow = (sizeof(TC) == 8) ? ((lr & 3) * 4 + (lr >> 2)) : lr;
    int tm, tn, split;
    if (!map_tile(g, tm, tn, split)) return;
    const int row0 = tm * BM, col0 = tn * BN;
    const int kbeg = split * g.k_chunk;
    const int kend = max(kbeg, min(g.k_len, kbeg + g.k_chunk));  // an empty split stores zeros
    // nodes that finished keep their columns, but a tile whose 64 nodes are
    // all finished (or empty) has nothing to compute; the check is read
    // beside the first stage's loads, not before them
    const int run = (g.col_status && tid < BN) ? (g.col_status[col0 + tid] == SLOT_RUNNING) : (g.col_status ? 0 : 1);
    const TA *A = reinterpret_cast<const TA *>(g.A);
    const TB *Bg = reinterpret_cast<const TB *>(g.B);

    acc_t acc[FI][2];
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = acc_t{0, 0, 0, 0};
    // the epilogue's y values (rows row0 + wm*BM/2 + i*16 + lg*4 + r), loaded
    // now so their latency is hidden behind the contraction (y has npad rows)
    double yv[FI][4];
    if constexpr (MODE != EPI_STORE) {
#pragma unroll
        for (int i = 0; i < FI; ++i) ld4(g.y + row0 + wm * (BM / 2) + i * 16 + lg * 4, yv[i]);
    }

    // staging: thread t loads groups t, t + 256, ... of each operand tile;
    // group x covers row x / GPR, k = 4 (x % GPR) .. + 3 of the stage
    TC ra[LPA][4], rb[LPB][4];
    bool rka[LPA], rkb[LPB];
    // loads only: a group past kend re-reads k = kbeg (always valid); its
    // zeroing happens at the LDS store, so no instruction consumes the loaded
    // registers before the stage's MFMA work has been issued
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int v = 0; v < LPA; ++v) {
            const int x = tid + 256 * v;
            const int r = x / GPR, kq = 4 * (x % GPR);
            rka[v] = k0 + kq < kend;
            ld4(A + (int64_t)(row0 + r) * g.lda + (rka[v] ? k0 + kq : kbeg), ra[v]);
        }
#pragma unroll
        for (int v = 0; v < LPB; ++v) {
            const int x = tid + 256 * v;
            const int r = x / GPR, kq = 4 * (x % GPR);
            rkb[v] = k0 + kq < kend;
            ld4(Bg + (int64_t)(col0 + r) * g.ldb + (rkb[v] ? k0 + kq : kbeg), rb[v]);
        }
    };
    auto store_stage = [&](int bufi) {
#pragma unroll
        for (int v = 0; v < LPA; ++v) {
            const int x = tid + 256 * v;
            const int r = x / GPR, kq = 4 * (x % GPR);
#pragma unroll
            for (int e = 0; e < 4; ++e) As[bufi][r * LS + kq + e] = rka[v] ? ra[v][e] : (TC)0;
        }
#pragma unroll
        for (int v = 0; v < LPB; ++v) {
            const int x = tid + 256 * v;
            const int r = x / GPR, kq = 4 * (x % GPR);
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[bufi][r * LS + kq + e] = rkb[v] ? rb[v][e] : (TC)0;
        }
    };

    // contract sub-blocks [0, nh) of the LDS stage in buffer bi
    auto compute = [&](int bi, int h) {
        TC av[FI][4], bv[2][4];
#pragma unroll
        for (int f = 0; f < FI; ++f) {
            const TC *pa = &As[bi][(wm * (BM / 2) + f * 16 + arow) * LS + 16 * h + 4 * lg];
#pragma unroll
            for (int s = 0; s < 4; ++s) av[f][s] = pa[s];
        }
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const TC *pb = &Bs[bi][(wn * 32 + f * 16 + lr) * LS + 16 * h + 4 * lg];
#pragma unroll
            for (int s = 0; s < 4; ++s) bv[f][s] = pb[s];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < FI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = mfma16(av[i][s], bv[j][s], acc[i][j]);
    };

    // full stages (no conditions inside), then a partial last stage whose
    // depth is a multiple of 16
    const int nfull = (kend - kbeg) / BK;
    const int ntail = ((kend - kbeg) % BK) / 16;
    const int nstage = nfull + (ntail > 0 ? 1 : 0);
    if (nstage > 0) load_stage(kbeg);
    if (!__syncthreads_or(run)) return;
    if (nstage > 0) store_stage(0);
    __syncthreads();
    int buf = 0;
    for (int st = 0; st < nstage; ++st) {
        const bool more = st + 1 < nstage;
        if (more) load_stage(kbeg + (st + 1) * BK);
        if (st < nfull) {
#pragma unroll
            for (int h = 0; h < NH; ++h) compute(buf, h);
        } else {
            for (int h = 0; h < ntail; ++h) compute(buf, h);
        }
        if (more) store_stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    // ---- epilogue ----------------------------------------------------------
    // acc[i][j][r] holds C at row = row0 + wm*BM/2 + i*16 + lg*4 + r,
    //                        col = col0 + wn*32 + j*16 + lr.
    if constexpr (MODE != EPI_CERT) {
        epi_store<TC, MODE, FI>(g, acc, yv, row0, col0, wm, wn, lg, lr, split);
    } else {  // EPI_CERT (TC is double)
        double *C = reinterpret_cast<double *>(g.C);
        __shared__ double red_l[2][64];
        __shared__ double red_c[2][64];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = col0 + wn * 32 + j * 16 + lr;
            double sl = 0.0, sc = 0.0;
#pragma unroll
            for (int i = 0; i < FI; ++i) {
                const int rb0 = row0 + wm * (BM / 2) + i * 16 + lg * 4;
                f64x4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rb0 + r;
                    double z, lv, cv;
                    cert_terms(g.loss, acc[i][j][r], yv[i][r], z, lv, cv);
                    const bool in = row < g.n;
                    o[r] = in ? z : 0.0;
                    sl += in ? lv : 0.0;
                    sc += in ? cv : 0.0;
                }
                *reinterpret_cast<f64x4 *>(C + (int64_t)col * g.ldc + rb0) = o;
                if (g.sc_out) {
                    f64x4 sv;
#pragma unroll
                    for (int r = 0; r < 4; ++r) sv[r] = (rb0 + r < g.n) ? (double)acc[i][j][r] : 0.0;
                    *reinterpret_cast<f64x4 *>(g.sc_out + (int64_t)col * g.ldc + rb0) = sv;
                }
            }
            // reduce over the 4 lane groups holding this column
            sl += __shfl_xor(sl, 16);
            sl += __shfl_xor(sl, 32);
            sc += __shfl_xor(sc, 16);
            sc += __shfl_xor(sc, 32);
            if (lg == 0) {
                red_l[wm][wn * 32 + j * 16 + lr] = sl;
                red_c[wm][wn * 32 + j * 16 + lr] = sc;
            }
        }
        __syncthreads();
        // the sums are indexed in 32-row units whatever the tile height, so
        // launches with either height leave no stale entry behind
        if (tid < 64) {
            const int col = col0 + tid;
            const int64_t t32 = (int64_t)tm * (BM / 32);
            g.lsum[t32 * g.ldsum + col] = red_l[0][tid] + red_l[1][tid];
            g.csum[t32 * g.ldsum + col] = red_c[0][tid] + red_c[1][tid];
            if constexpr (BM == 64) {
                g.lsum[(t32 + 1) * g.ldsum + col] = 0.0;
                g.csum[(t32 + 1) * g.ldsum + col] = 0.0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// bfloat16 helpers: round to nearest even, and the three-term split of a
// float32 value b into bfloat16 hi = bf16(b), mid = bf16(b - hi),
// lo = bf16(b - hi - mid) (both differences are exact in float32), whose sum
// carries b's 24-bit significand.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t bf16_rne_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
// b -> three bfloat16 bit patterns (hi, mid, lo) with hi + mid + lo ~= b
__device__ __forceinline__ void split3(float b, uint16_t &h, uint16_t &m, uint16_t &l)
{
    const uint32_t hb = bf16_rne_bits(b);
    const float r1 = b - __uint_as_float(hb << 16);
    const uint32_t mb = bf16_rne_bits(r1);
    const float r2 = r1 - __uint_as_float(mb << 16);
    h = (uint16_t)hb;
    m = (uint16_t)mb;
    l = (uint16_t)bf16_rne_bits(r2);
}


// ---------------------------------------------------------------------------
// bfloat16 planes.  A float32 value v is stored as planes v1 = bf16(v),
// v2 = bf16(v - v1), v3 = bf16(v - v1 - v2) (round to nearest even): three
// planes carry v's 24-bit significand, two planes 16 bits.  Products of
// planes are exact in float32, so a bfloat16 matrix times the planes of a
// float32 one is a sum of exact bfloat16 MFMA products.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint2 pack4(const uint16_t (&v)[4])
{
    return make_uint2(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16));
}

// the first NP (2 or 3) planes of 4 consecutive float32 values at element
// offset o (planes `plane` elements apart)
template <int NP = 3>
__device__ __forceinline__ void store_planes4(uint16_t *C, int64_t plane, int64_t o, const float (&d)[4])
{
    uint16_t h[4], m[4], l[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) split3(d[r], h[r], m[r], l[r]);
    *reinterpret_cast<uint2 *>(C + o) = pack4(h);
    *reinterpret_cast<uint2 *>(C + plane + o) = pack4(m);
    if constexpr (NP > 2) *reinterpret_cast<uint2 *>(C + 2 * plane + o) = pack4(l);
}

// ---------------------------------------------------------------------------
// Streaming bfloat16 contraction for bfloat16 A against NB planes of B (the
// bound of tall instances is the HBM stream of X).  Tile 4 WR x 64: wave w
// owns rows row0 + WR w .. + WR - 1 and all 64 columns (WR/16 x 4 MFMA
// blocks of 16 x 16, float32 accumulate).  The k loop runs in super-steps of
// 128.  Each lane loads its A rows straight into registers in the MFMA
// operand layout, from the tiled copy of k_tile_bf16 in which every load
// instruction of a wave reads 1 KB of contiguous memory, one super-step
// ahead of the MFMAs (no LDS traffic for A).  B is staged through LDS,
// prefetched into registers one super-step ahead.  MFMA k-step h of a
// super-step contracts, in lane group g, k = 32 g + 8 h .. + 7 of A and B
// alike (a fixed permutation of the k order inside the super-step).
// Epilogues: EPI_DLOSS (R = l'(S, y) written as NB planes), EPI_DLOSS_ANCHOR
// (R = l'(S_c + S) - l'(S_c) formed in float64, NB planes), EPI_STORE
// (split-K float32 partials).  Rows of A past rows_a repeat the last row
// block and are not stored (rows_c / rows_valid).
// ---------------------------------------------------------------------------
template <int MODE, int WR, int NB, bool ADB = true>
__global__ __launch_bounds__(256, ADB ? 1 : 2) void k_gemm_stream(GemmArgs g)
{
    constexpr int BM = 4 * WR, BN = GEMM_BN, SK = 128;
    constexpr int FI = WR / 16, FJ = 4;
    constexpr int LSB = SK + 8;                 // LDS row stride (bf16): 272 bytes
    constexpr int CPR = SK / 8;                 // 16-byte chunks per B row and super-step
    constexpr int LPB = (BN * CPR) / 256;       // B chunks per thread and plane (4)
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NB][BN * LSB];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    int tm, tn, split;
    if (!map_tile(g, tm, tn, split)) return;
    const int row0 = tm * BM, col0 = tn * BN;
    const int wrow = row0 + WR * wave;
    const int kbeg = split * g.k_chunk;
    const int kend = max(kbeg, min(g.k_len, kbeg + g.k_chunk));
    const uint16_t *A = reinterpret_cast<const uint16_t *>(g.A);
    const uint16_t *Bg = reinterpret_cast<const uint16_t *>(g.B);
    const int run = (g.col_status && tid < BN) ? (g.col_status[col0 + tid] == SLOT_RUNNING) : 1;

    f32x4 acc[FI][FJ];
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

    // A is in the tiled layout of k_tile_bf16 (g.lda = 128-wide k blocks per
    // 16-row block): the 16 x 128 block of row block rb and k block kb is
    // 2048 contiguous elements, in which instruction q of lane l reads the 16
    // bytes at (64 q + l) * 8, i.e. row l % 16, k = 32 (l / 16) + 8 q: each
    // load instruction of a wave reads 1 KB of contiguous memory.  A row
    // block past the last one reads the last (its outputs are not stored);
    // the layout is zero beyond the k extent, and B is zeroed past kend when
    // staged, so split boundaries need no guard on A (they are multiples of
    // 128).
    const int nrb = (g.rows_a + 15) / 16;
    const uint16_t *pa[FI];
#pragma unroll
    for (int f = 0; f < FI; ++f)
        pa[f] = A + (int64_t)min(wrow / 16 + f, nrb - 1) * g.lda * 2048 + (int64_t)lane * 8;
    // A: two register sets (the super-step being contracted and the next);
    // B: one register set, loaded two super-steps ahead and staged into the
    // LDS buffer of the next super-step while the current one is contracted
    uint4 ra0[FI][4], ra1[FI][4], rb[NB][LPB];
    auto load_a = [&](int k0, uint4 (&ra)[FI][4]) {
        const int64_t kb = (int64_t)(k0 / 128) * 2048;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int f = 0; f < FI; ++f) ra[f][q] = *reinterpret_cast<const uint4 *>(pa[f] + kb + 512 * q);
        }
    };
    auto load_b = [&](int k0) {
#pragma unroll
        for (int v = 0; v < LPB; ++v) {
            const int x = tid + 256 * v;
            const int cl = x / CPR, k = k0 + 8 * (x % CPR);
            const int64_t o = (int64_t)(col0 + cl) * g.ldb + ((k < kend) ? k : kbeg);
#pragma unroll
            for (int pb = 0; pb < NB; ++pb) rb[pb][v] = *reinterpret_cast<const uint4 *>(Bg + pb * g.b_plane + o);
        }
    };
    auto stage_b = [&](int bi, int k0) {
#pragma unroll
        for (int v = 0; v < LPB; ++v) {
            const int x = tid + 256 * v;
            const int cl = x / CPR, kq = 8 * (x % CPR);
            const bool ok = k0 + kq < kend;
#pragma unroll
            for (int pb = 0; pb < NB; ++pb)
                *reinterpret_cast<uint4 *>(&Bs[bi][pb][cl * LSB + kq]) = ok ? rb[pb][v] : make_uint4(0, 0, 0, 0);
        }
    };
    // B operands of MFMA k-step h, read from LDS one k-step ahead of their use
    auto read_b = [&](int bi, int h, bf16x8 (&bv)[NB][FJ]) {
#pragma unroll
        for (int pb = 0; pb < NB; ++pb)
#pragma unroll
            for (int j = 0; j < FJ; ++j)
                bv[pb][j] = *reinterpret_cast<const bf16x8 *>(&Bs[bi][pb][(16 * j + lr) * LSB + 32 * lg + 8 * h]);
    };
    auto mfmas = [&](const uint4 (&ra)[FI][4], int h, const bf16x8 (&bv)[NB][FJ]) {
#pragma unroll
        for (int t = NB - 1; t >= 0; --t)  // small terms first
#pragma unroll
            for (int f = 0; f < FI; ++f) {
                const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&ra[f][h]);
#pragma unroll
                for (int j = 0; j < FJ; ++j)
                    acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[t][j], acc[f][j], 0, 0, 0);
            }
    };
    auto compute = [&](const uint4 (&ra)[FI][4], int bi) {
        bf16x8 b0[NB][FJ], b1[NB][FJ];
        read_b(bi, 0, b0);
        read_b(bi, 1, b1);
        mfmas(ra, 0, b0);
        read_b(bi, 2, b0);
        mfmas(ra, 1, b1);
        read_b(bi, 3, b1);
        mfmas(ra, 2, b0);
        mfmas(ra, 3, b1);
    };
    // super-step s contracts LDS buffer s & 1
    auto step = [&](int s, const uint4 (&ra)[FI][4], uint4 (&ra_next)[FI][4], int nss) {
        if (s + 1 < nss) load_a(kbeg + (s + 1) * SK, ra_next);
        compute(ra, s & 1);
        if (s + 1 < nss) {
            stage_b((s + 1) & 1, kbeg + (s + 1) * SK);
            if (s + 2 < nss) load_b(kbeg + (s + 2) * SK);
        }
        __syncthreads();
    };

    const int nss = (kend - kbeg + SK - 1) / SK;
    if (nss > 0) {
        load_a(kbeg, ra0);
        load_b(kbeg);
    }
    if (!__syncthreads_or(run)) return;  // every node of the tile has finished
    if (nss > 0) {
        stage_b(0, kbeg);
        if (nss > 1) load_b(kbeg + SK);
    }
    __syncthreads();
    if constexpr (ADB) {
        // two super-steps per trip, so the A register sets are fixed at compile time
        for (int s = 0; s < nss; s += 2) {
            step(s, ra0, ra1, nss);
            if (s + 1 >= nss) break;
            step(s + 1, ra1, ra0, nss);
        }
    } else {
        // one A register set, loaded at the start of its own super-step: the
        // freed registers let a second workgroup share the CU and cover that
        // load's latency
        for (int s = 0; s < nss; ++s) {
            if (s > 0) load_a(kbeg + s * SK, ra0);
            compute(ra0, s & 1);
            if (s + 1 < nss) {
                stage_b((s + 1) & 1, kbeg + (s + 1) * SK);
                if (s + 2 < nss) load_b(kbeg + (s + 2) * SK);
            }
            __syncthreads();
        }
    }

    // ---- epilogue: acc[f][j][r] holds C at row = wrow + 16 f + 4 lg + r,
    //                col = col0 + 16 j + lr
    if constexpr (MODE == EPI_STORE) {
        float *C = reinterpret_cast<float *>(g.C) + (int64_t)split * g.split_stride;
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const int col = col0 + 16 * j + lr;
#pragma unroll
            for (int f = 0; f < FI; ++f) {
                const int rb = wrow + 16 * f + 4 * lg;
                if (rb + 3 < g.rows_valid) {
                    *reinterpret_cast<f32x4 *>(C + (int64_t)col * g.ldc + rb) = acc[f][j];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (rb + r < g.rows_valid) C[(int64_t)col * g.ldc + rb + r] = acc[f][j][r];
                }
            }
        }
    } else {
        uint16_t *C = reinterpret_cast<uint16_t *>(g.C);
#pragma unroll
        for (int f = 0; f < FI; ++f) {
            const int rb = wrow + 16 * f + 4 * lg;
            if (rb >= g.rows_c) continue;  // rows_c is a multiple of 4
            double yv[4];
            ld4(g.y + rb, yv);
#pragma unroll
            for (int j = 0; j < FJ; ++j) {
                const int col = col0 + 16 * j + lr;
                float d[4];
                if constexpr (MODE == EPI_DLOSS) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        d[r] = (rb + r < g.n) ? dloss_f(g.loss, acc[f][j][r], (float)yv[r]) : 0.0f;
                } else {  // EPI_DLOSS_ANCHOR
                    if (g.loss == 0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) d[r] = (rb + r < g.n) ? 2.0f * acc[f][j][r] : 0.0f;
                    } else {
                        double sc[4];
                        ld4(g.sc + (int64_t)col * g.ldc + rb, sc);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const double sv = sc[r] + (double)acc[f][j][r];
                            const double dd = dloss_d(g.loss, sv, yv[r]) - dloss_d(g.loss, sc[r], yv[r]);
                            d[r] = (rb + r < g.n) ? (float)dd : 0.0f;
                        }
                    }
                }
                store_planes4<NB>(C, g.c_plane, (int64_t)col * g.ldc + rb, d);
            }
        }
    }
}

// Tiled copy of a row-major bfloat16 matrix for k_gemm_stream: 16-row by
// 128-column blocks of 2048 contiguous elements (row block rb, column block
// kb at (rb * nkb + kb) * 2048), inside a block element (r, k) at
// ((4 (k % 32 / 8) + k / 32) * 16 + r) * 8 + k % 8; zero outside rows x cols.
// One thread per 8-element chunk.
__global__ __launch_bounds__(256) void k_tile_bf16(const uint16_t *__restrict__ src, int64_t lds, int rows, int cols,
                                                   int nrb, int nkb, uint16_t *__restrict__ dst)
{
    const int64_t nch = (int64_t)nrb * nkb * 256;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = c / 256;
        const int w = (int)(c % 256);
        const int q = w / 64, l = w % 64;
        const int rb = (int)(b / nkb), kb = (int)(b % nkb);
        const int row = rb * 16 + (l & 15), k = kb * 128 + 32 * (l >> 4) + 8 * q;
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (row < rows && k + e < cols) ? src[(int64_t)row * lds + k + e] : (uint16_t)0;
        uint4 o;
        o.x = v[0] | ((uint32_t)v[1] << 16);
        o.y = v[2] | ((uint32_t)v[3] << 16);
        o.z = v[4] | ((uint32_t)v[5] << 16);
        o.w = v[6] | ((uint32_t)v[7] << 16);
        *reinterpret_cast<uint4 *>(dst + c * 8) = o;
    }
}

void launch_tile_bf16(hipStream_t s, const uint16_t *src, int64_t lds, int rows, int cols, uint16_t *dst)
{
    const int nrb = (rows + 15) / 16, nkb = (cols + 127) / 128;
    const int64_t nch = (int64_t)nrb * nkb * 256;
    const int blocks = (int)std::min<int64_t>((nch + 255) / 256, 16384);
    if (blocks > 0) KBNB_LAUNCH(k_tile_bf16, dim3(blocks), dim3(256), 0, s, src, lds, rows, cols, nrb, nkb, dst);
}

// Wave tile height of a streaming launch: the explicit tile (4 waves per
// workgroup tile), else the tallest of 64 / 32 / 16 rows that still gives
// the launch 256 workgroups (a thin frontier on a short X needs the smaller
// tiles to occupy the CUs; tall tiles reuse each B super-step longer).
int stream_wave_rows(int tile_rows, int rows, int tiles_n, int splits)
{
    if (tile_rows) return tile_rows / 4;
    int wr = 64;
    while (wr > 16 && (int64_t)((rows + 4 * wr - 1) / (4 * wr)) * tiles_n * splits < 256) wr /= 2;
    return wr;
}

int launch_gemm_stream(hipStream_t s, int mode, GemmArgs g, int rows, int tiles_n, int splits, int wr, int nb)
{
    const int bm = 4 * wr;
    g.tiles_n = tiles_n;
    g.nsplit = splits;
    g.tiles_m = (rows + bm - 1) / bm;
    int nblocks;
    if (splits > 1) nblocks = 8 * g.tiles_m * tiles_n * ((splits + 7) / 8);
    else if (g.tiles_m >= 8) nblocks = (g.tiles_m + 7) / 8 * 8 * tiles_n;
    else nblocks = g.tiles_m * tiles_n;
    const dim3 grid(nblocks, 1);
    if ((wr != 16 && wr != 32 && wr != 64) || (nb != 2 && nb != 3)) return -1;
    // two-plane launches with 64-row wave tiles run with one A register set
    // at two workgroups per CU: the forward always (5-9% faster at 100000 x
    // 5000), the split-K backward from two column tiles up (4-10% at widths
    // 128-512; a single column tile keeps the prefetch); three planes do not
    // fit two workgroups and keep the prefetching A set
#define KBNB_STREAM_1A(M)                                                                       \
    do {                                                                                         \
        if (wr == 64 && nb == 3) KBNB_LAUNCH((k_gemm_stream<M, 64, 3>), grid, dim3(256), 0, s, g); \
        else if (wr == 64) KBNB_LAUNCH((k_gemm_stream<M, 64, 2, false>), grid, dim3(256), 0, s, g);       \
        else if (wr == 32 && nb == 3) KBNB_LAUNCH((k_gemm_stream<M, 32, 3>), grid, dim3(256), 0, s, g); \
        else if (wr == 32) KBNB_LAUNCH((k_gemm_stream<M, 32, 2>), grid, dim3(256), 0, s, g);       \
        else if (nb == 3) KBNB_LAUNCH((k_gemm_stream<M, 16, 3>), grid, dim3(256), 0, s, g);        \
        else KBNB_LAUNCH((k_gemm_stream<M, 16, 2>), grid, dim3(256), 0, s, g);                     \
    } while (0)
#define KBNB_STREAM(M)                                                                           \
    do {                                                                                         \
        if (wr == 64 && nb == 3) KBNB_LAUNCH((k_gemm_stream<M, 64, 3>), grid, dim3(256), 0, s, g); \
        else if (wr == 64) KBNB_LAUNCH((k_gemm_stream<M, 64, 2>), grid, dim3(256), 0, s, g);       \
        else if (wr == 32 && nb == 3) KBNB_LAUNCH((k_gemm_stream<M, 32, 3>), grid, dim3(256), 0, s, g); \
        else if (wr == 32) KBNB_LAUNCH((k_gemm_stream<M, 32, 2>), grid, dim3(256), 0, s, g);       \
        else if (nb == 3) KBNB_LAUNCH((k_gemm_stream<M, 16, 3>), grid, dim3(256), 0, s, g);        \
        else KBNB_LAUNCH((k_gemm_stream<M, 16, 2>), grid, dim3(256), 0, s, g);                     \
    } while (0)
    if (mode == EPI_DLOSS) KBNB_STREAM_1A(EPI_DLOSS);
    else if (mode == EPI_DLOSS_ANCHOR) KBNB_STREAM_1A(EPI_DLOSS_ANCHOR);
    else if (mode == EPI_STORE && tiles_n >= 2) KBNB_STREAM_1A(EPI_STORE);
    else if (mode == EPI_STORE) KBNB_STREAM(EPI_STORE);
    else return -1;
#undef KBNB_STREAM
#undef KBNB_STREAM_1A
    return 0;
}


// ---------------------------------------------------------------------------
// Wavefront and workgroup helpers.  A per-node workgroup has W waves; with
// W = 1 the block-level helpers are the plain wave operations.  Every block
// helper must be reached by all threads of the workgroup.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// argmax with ties to the lowest index; (v, i) pairs, i = INT_MAX for none
__device__ __forceinline__ void wave_argmax(double &v, int &i)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double v2 = __shfl_xor(v, o);
        int i2 = __shfl_xor(i, o);
        if (v2 > v || (v2 == v && i2 < i)) {
            v = v2;
            i = i2;
        }
    }
}
// inclusive prefix sum over the lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int ln = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(v, o);
        if (ln >= o) v += t;
    }
    return v;
}

// Sums reduce the per-wave totals in wave order, so every thread gets the
// same bits.
template <int W>
__device__ __forceinline__ double blk_sum(double v)
{
    v = wave_sum(v);
    if constexpr (W == 1) {
        return v;
    } else {
        __shared__ double red[W];
        __syncthreads();
        if (lane_id() == 0) red[wave_id()] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) s += red[q];
        return s;
    }
}
template <int W>
__device__ __forceinline__ int blk_sum_i(int v)
{
    v = wave_sum_i(v);
    if constexpr (W == 1) {
        return v;
    } else {
        __shared__ int red[W];
        __syncthreads();
        if (lane_id() == 0) red[wave_id()] = v;
        __syncthreads();
        int s = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) s += red[q];
        return s;
    }
}
template <int W>
__device__ __forceinline__ int blk_max_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    if constexpr (W == 1) {
        return v;
    } else {
        __shared__ int red[W];
        __syncthreads();
        if (lane_id() == 0) red[wave_id()] = v;
        __syncthreads();
        int s = red[0];
#pragma unroll
        for (int q = 1; q < W; ++q) s = max(s, red[q]);
        return s;
    }
}
template <int W>
__device__ __forceinline__ bool blk_any(bool pred)
{
    if constexpr (W == 1) return __ballot(pred) != 0ull;
    else return __syncthreads_or(pred) != 0;
}
template <int W>
__device__ __forceinline__ void blk_argmax(double &v, int &i)
{
    wave_argmax(v, i);
    if constexpr (W > 1) {
        __shared__ double rv[W];
        __shared__ int ri[W];
        __syncthreads();
        if (lane_id() == 0) {
            rv[wave_id()] = v;
            ri[wave_id()] = i;
        }
        __syncthreads();
        v = rv[0];
        i = ri[0];
#pragma unroll
        for (int q = 1; q < W; ++q)
            if (rv[q] > v || (rv[q] == v && ri[q] < i)) {
                v = rv[q];
                i = ri[q];
            }
    }
}
// exclusive prefix sum over the workgroup's threads (in thread order)
template <int W, typename T>
__device__ __forceinline__ T blk_excl_scan(T v)
{
    const T incl = wave_incl_scan(v);
    if constexpr (W == 1) {
        return incl - v;
    } else {
        __shared__ T tot[W];
        __syncthreads();
        if (lane_id() == 63) tot[wave_id()] = incl;
        __syncthreads();
        T off = 0;
        for (int q = 0; q < wave_id(); ++q) off += tot[q];
        return off + incl - v;
    }
}

// Huber prox: argmin_v 1/2 (v - x)^2 + c H_M(v)
__device__ __forceinline__ double prox_huber(double x, double c, double M)
{
    if (fabs(x) <= M * (1.0 + c)) return x / (1.0 + c);
    return (x > 0.0) ? x - c * M : x + c * M;
}
__device__ __forceinline__ double huber(double q, double M)
{
    const double a = fabs(q);
    return (a <= M) ? 0.5 * q * q : M * a - 0.5 * M * M;
}

// Bitonic sort of PP (key, idx) pairs in LDS by the whole workgroup:
// key descending, idx ascending on equal keys (a strict total order).
template <int PP, typename TI>
__device__ void bitonic_desc(double *key, TI *idx)
{
    for (int size = 2; size <= PP; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < PP / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const double ki = key[i], kj = key[j];
                const TI ii = idx[i], ij = idx[j];
                const bool i_first = (ki > kj) || (ki == kj && ii < ij);
                const bool want_desc = ((i & size) == 0);
                if (want_desc != i_first) {
                    key[i] = kj; key[j] = ki;
                    idx[i] = ij; idx[j] = ii;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Per-node kernels run one workgroup of W waves per node (W = PP / 256, at
// most 16).  Thread t owns the contiguous coordinates
// j = E t .. E t + E - 1 (E = PP / (64 W); PP >= 256 a power of two >= p),
// i.e. E / 4 whole groups of four, so a node's column is read and written
// with 16-byte vector accesses.  Groups at or beyond ldp (the padded column
// length, a multiple of 16) are not touched.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ld4_i8(const int8_t *p, int o[4])
{
    const char4 v = *reinterpret_cast<const char4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void st4(float *p, const double v[4])
{
    *reinterpret_cast<float4 *>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
}
__device__ __forceinline__ void st4(double *p, const double v[4])
{
    *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2 *>(p + 2) = make_double2(v[2], v[3]);
}

// The next point of the iteration, 4 consecutive entries at element offset o
// of a node-major [mpad][ldp] array: float32 / float64 Yi, or in plane mode
// its nb bfloat16 planes.
template <typename Ti>
__device__ __forceinline__ void store_y4(const Consts &c, Ti *Yi, int64_t o, const double (&v)[4])
{
    if (c.yp) {
        uint16_t hh[4], mm[4], ll[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) split3((float)v[r], hh[r], mm[r], ll[r]);
        const int64_t pl = (int64_t)c.mpad * c.ldp;
        *reinterpret_cast<uint2 *>(c.yp + o) = pack4(hh);
        *reinterpret_cast<uint2 *>(c.yp + pl + o) = pack4(mm);
        if (c.nb > 2) *reinterpret_cast<uint2 *>(c.yp + 2 * pl + o) = pack4(ll);
    } else {
        st4(Yi + o, v);
    }
}

// Registers a split batch may hold in a workgroup of W waves.
__host__ __device__ constexpr int split_regs(int w) { return w >= 16 ? 32 : (w >= 8 ? 64 : 128); }

// Sum of split-K partials for a thread's chunk: acc[e] += sum_s col[s * stride + j0 + e].
// Splits are taken in batches of SB with no conditions inside, so all SB * NQ
// 16-byte loads of a batch are in flight together; the remaining splits
// (nsplit is the same for the whole workgroup) go one at a time.  A batch
// holds at most RB registers (the workgroup size caps a wave's registers:
// 1024 threads leave 128, and a larger batch spills to scratch).  Group
// addresses are clamped into the column with min(): a group past ldp reads
// valid memory and its (unused) value belongs to a padding coordinate.
template <typename T, int NQ, int RB>
__device__ __forceinline__ void sum_splits(const T *__restrict__ col, int nsplit, int64_t stride,
                                           int j0, int ldp, double (&acc)[4 * NQ])
{
    constexpr int SB0 = split_batch(4 * NQ * 64, (int)sizeof(T));
    constexpr int SBR = RB / (4 * NQ * ((int)sizeof(T) / 4));
    constexpr int SB = SBR < 1 ? 1 : (SBR < SB0 ? SBR : SB0);
    int go[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) go[q] = min(j0 + 4 * q, ldp - 4);
    int s0 = 0;
    for (; s0 + SB <= nsplit; s0 += SB) {
        T v[SB][4 * NQ];
#pragma unroll
        for (int i = 0; i < SB; ++i)
#pragma unroll
            for (int q = 0; q < NQ; ++q) ld4(col + (int64_t)(s0 + i) * stride + go[q], &v[i][4 * q]);
#pragma unroll
        for (int i = 0; i < SB; ++i)
#pragma unroll
            for (int e = 0; e < 4 * NQ; ++e) acc[e] += (double)v[i][e];
    }
    for (; s0 < nsplit; ++s0) {
        T v[4 * NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) ld4(col + (int64_t)s0 * stride + go[q], &v[4 * q]);
#pragma unroll
        for (int e = 0; e < 4 * NQ; ++e) acc[e] += (double)v[e];
    }
}

// Waves per node workgroup for a padded column length PP.
template <int PP> struct NodeWaves { static constexpr int W = node_waves(PP); };

// ---------------------------------------------------------------------------
// Masked prox of one node (paper Sec. 4.2 "Evaluating proximal operators with
// non-uniform node structure", eq. pgd_step_vector_form; App. B):
//   J0 -> 0;  J1 -> u / (1 + 2 eta lambda2) clipped to [-M, M];
//   free coordinates: keys |u| (non-free and padding -1, below every free key),
//   descending sort, then the PAVA of App. B with weights rho on the first
//   kbar positions and 0 after.  Violations can only start at the kbar/kbar+1
//   boundary, so a single pooled block [a, b] forms there; positions before
//   it keep the ridge-and-clip value, block positions get |u| - V / rho
//   (V the block value in rho-scaled units), positions after it exactly 0.
// The block is found in parallel.  With P the prefix sums of w = rho * key,
// the pooled value of [a, b] is
//   V(a, b) = prox_{c H_M}(S / cnt),  S = P[b+1] - P[a], cnt = b - a + 1,
//                                     c = rho (kbar - a) / cnt.
// For a fixed left end the block grows right while V(a, b) < w_{b+1}; that
// test is monotone in b, so all (a, b) pairs are tested at once and the
// smallest passing b, b(a), is kept per a.  The left end is the largest a
// whose left neighbour's value prox_{rho H_M}(w_{a-1}) is not below
// V(a, b(a)).  This is the block the one-step expansion of App. B reaches.
// The right test is written without divisions:
//   S <= M (cnt + wa):  V = S / (cnt + wa)      ->  S >= w (cnt + wa)
//   otherwise:          V = (S - wa M) / cnt    ->  S - wa M >= w cnt
// with wa = rho (kbar - a).
// ---------------------------------------------------------------------------
template <int PP>
struct ProxLds {
    double key[PP];       // free magnitudes in sorted (descending) order
    uint16_t rank[PP];    // sorted position of each free coordinate
    double psum[PP + 1];  // prefix sums of rho * key
    int bmin[128];        // per left end a: smallest passing right end
    double vblk[128];     // per left end a: block value V(a, b(a))
};

// Register bitonic sort of one wave's 64 E (key, idx) pairs; lane l holds
// positions l E .. l E + E - 1.  Order: key descending, idx ascending on equal
// keys (strict).  Strides below E are compare-exchanges inside a lane; larger
// strides pair lane l with lane l ^ (stride / E) through shuffles.
template <int PP>
__device__ __forceinline__ void reg_bitonic_desc(double (&key)[PP / 64], int (&idx)[PP / 64])
{
    constexpr int E = PP / 64;
    const int l = lane_id();
#pragma unroll
    for (int size = 2; size <= PP; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= E) {
                const int lm = stride / E;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const double pk = __shfl_xor(key[e], lm);
                    const int pi = __shfl_xor(idx[e], lm);
                    const int i = l * E + e;
                    const bool lower = (i & stride) == 0;
                    const bool desc = (i & size) == 0;
                    const bool mine_first = (key[e] > pk) || (key[e] == pk && idx[e] < pi);
                    const bool keep = (lower == desc) ? mine_first : !mine_first;
                    if (!keep) { key[e] = pk; idx[e] = pi; }
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e & stride) continue;
                    const int e2 = e | stride;
                    const int i = l * E + e;
                    const bool desc = (i & size) == 0;
                    const bool first = (key[e] > key[e2]) || (key[e] == key[e2] && idx[e] < idx[e2]);
                    if (desc != first) {
                        const double tk = key[e]; key[e] = key[e2]; key[e2] = tk;
                        const int ti = idx[e]; idx[e] = idx[e2]; idx[e2] = ti;
                    }
                }
            }
        }
    }
}

// Descending order with index tie-break, as in the sort.
__device__ __forceinline__ bool before(double ka, int ia, double kb, int ib)
{
    return (ka > kb) || (ka == kb && ia < ib);
}

// perm (nullable): the node's sorted order from its previous step (PP
// entries, free coordinates first); when given, the new keys are gathered in
// that order and repaired by odd-even transposition rounds, which is cheap
// because the order of |u| changes little between steps; the full sort runs
// only if 8 rounds leave it unsorted.  The new order is written back.
template <int PP, int W>
__device__ void masked_prox(ProxLds<PP> &L, const double (&u)[PP / (64 * W)],
                            const int (&sv)[PP / (64 * W)], int p, int kbar, double eta,
                            double lambda2, double M, double (&bet)[PP / (64 * W)],
                            int32_t *perm, bool have_prev, const int (&pv)[PP / (64 * W)])
{
    constexpr int E = PP / (64 * W);
    constexpr int T = 64 * W;
    const int t = threadIdx.x;
    const int ln = lane_id();
    const int j0 = t * E;
    const double rho = 1.0 / (2.0 * eta * lambda2);
    const double shrink = 1.0 + 2.0 * eta * lambda2;
    double key[E];
    int idx[E];
    int nfree = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = j0 + e;
        const bool fr = (j < p) && sv[e] == 0;
        key[e] = fr ? fabs(u[e]) : -1.0;
        idx[e] = j;
        nfree += fr ? 1 : 0;
    }
    const int pf = blk_sum_i<W>(nfree);
    bool sorted = false;
    if (perm && have_prev) {
        // keys by coordinate into LDS, then gathered in the previous order
        // (pv: this thread's entries of the previous order, loaded by the caller)
#pragma unroll
        for (int e = 0; e < E; ++e) L.key[j0 + e] = key[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            idx[e] = pv[e];
            key[e] = L.key[pv[e]];
        }
        for (int round = 0; round < 8; ++round) {
            int swaps = 0;
            // even pairs (2i, 2i + 1) lie inside a thread
#pragma unroll
            for (int e = 0; e + 1 < E; e += 2) {
                if (!before(key[e], idx[e], key[e + 1], idx[e + 1])) {
                    const double tk = key[e]; key[e] = key[e + 1]; key[e + 1] = tk;
                    const int ti = idx[e]; idx[e] = idx[e + 1]; idx[e + 1] = ti;
                    ++swaps;
                }
            }
            // odd pairs: inside a thread, plus (last of thread t, first of t + 1)
#pragma unroll
            for (int e = 1; e + 1 < E; e += 2) {
                if (!before(key[e], idx[e], key[e + 1], idx[e + 1])) {
                    const double tk = key[e]; key[e] = key[e + 1]; key[e + 1] = tk;
                    const int ti = idx[e]; idx[e] = idx[e + 1]; idx[e + 1] = ti;
                    ++swaps;
                }
            }
            double nk = __shfl_down(key[0], 1);
            int ni = __shfl_down(idx[0], 1);
            double pk = __shfl_up(key[E - 1], 1);
            int pi = __shfl_up(idx[E - 1], 1);
            if constexpr (W > 1) {
                // neighbours across a wave boundary go through LDS; the
                // barrier of blk_any below orders these reads before the
                // next round's writes
                __shared__ double xk_first[W], xk_last[W];
                __shared__ int xi_first[W], xi_last[W];
                const int w = wave_id();
                if (ln == 0) { xk_first[w] = key[0]; xi_first[w] = idx[0]; }
                if (ln == 63) { xk_last[w] = key[E - 1]; xi_last[w] = idx[E - 1]; }
                __syncthreads();
                if (ln == 63 && w + 1 < W) { nk = xk_first[w + 1]; ni = xi_first[w + 1]; }
                if (ln == 0 && w > 0) { pk = xk_last[w - 1]; pi = xi_last[w - 1]; }
            }
            const bool swap_hi = (t < T - 1) && !before(key[E - 1], idx[E - 1], nk, ni);
            const bool swap_lo = (t > 0) && !before(pk, pi, key[0], idx[0]);
            if (swap_hi) { key[E - 1] = nk; idx[E - 1] = ni; ++swaps; }
            if (swap_lo) { key[0] = pk; idx[0] = pi; ++swaps; }
            if (!blk_any<W>(swaps != 0)) {
                sorted = true;
                break;
            }
        }
        __syncthreads();
    }
    if (sorted) {
        // repaired in place
    } else if constexpr (W == 1 && E <= 4) {
        reg_bitonic_desc<PP>(key, idx);
    } else {
        // wide chunks: sort through LDS (the register network would be too
        // large to unroll); L.key and L.rank serve as the pair arrays
        double *sk = L.key;
        uint16_t *si = L.rank;
#pragma unroll
        for (int e = 0; e < E; ++e) { sk[j0 + e] = key[e]; si[j0 + e] = (uint16_t)idx[e]; }
        __syncthreads();
        bitonic_desc<PP, uint16_t>(sk, si);
#pragma unroll
        for (int e = 0; e < E; ++e) { key[e] = sk[j0 + e]; idx[e] = si[j0 + e]; }
        __syncthreads();
    }
    if (perm) {
#pragma unroll
        for (int q = 0; q < E / 4; ++q)
            *reinterpret_cast<int4 *>(perm + j0 + 4 * q) =
                make_int4(idx[4 * q], idx[4 * q + 1], idx[4 * q + 2], idx[4 * q + 3]);
    }
    // sorted keys, ranks and prefix sums of w = rho * key
    double acc = 0.0, loc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int r = j0 + e;
        L.key[r] = key[e];
        if (r < pf) L.rank[idx[e]] = (uint16_t)r;
        acc += (r < pf) ? rho * key[e] : 0.0;
        loc[e] = acc;
    }
    const double excl = blk_excl_scan<W, double>(acc);
#pragma unroll
    for (int e = 0; e < E; ++e) L.psum[j0 + e + 1] = excl + loc[e];
    if (t == 0) L.psum[0] = 0.0;
    __syncthreads();

    int ba = 0, bb_end = -1, top;
    double V = 0.0;
    if (kbar <= 0) {
        top = 0;
    } else if (kbar >= pf) {
        top = pf;
    } else {
        top = kbar;
        const double wl = rho * L.key[kbar - 1], wr = rho * L.key[kbar];
        if (prox_huber(wl, rho, M) < wr) {
            // thread a finds b(a) by binary search (the right test is
            // monotone in b), then V(a, b(a)) and the left test; the left end
            // is the largest a that passes
            int found = -1;
            for (int a0 = ((kbar - 1) / T) * T; a0 >= 0 && found < 0; a0 -= T) {
                const int a = a0 + t;
                bool left = false;
                if (a < kbar) {
                    const double pa = L.psum[a];
                    const double wa = rho * (double)(kbar - a);
                    int lo = kbar, hi = pf - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        const double cnt = (double)(mid - a + 1);
                        const double S = L.psum[mid + 1] - pa;
                        const double w = rho * L.key[mid + 1];
                        const bool pass = (S <= M * (cnt + wa)) ? (S >= w * (cnt + wa))
                                                                : (S - wa * M >= w * cnt);
                        if (pass) hi = mid;
                        else lo = mid + 1;
                    }
                    const double cnt = (double)(lo - a + 1);
                    const double Va = prox_huber((L.psum[lo + 1] - pa) / cnt, wa / cnt, M);
                    L.bmin[a] = lo;
                    L.vblk[a] = Va;
                    left = (a == 0) || (prox_huber(rho * L.key[a - 1], rho, M) >= Va);
                }
                found = blk_max_i<W>(left ? a : -1);
            }
            __syncthreads();
            if (found >= 0) {
                ba = found;
                bb_end = L.bmin[found];
                V = L.vblk[found];
                top = found;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = j0 + e;
        const double au = fabs(u[e]), sg = (u[e] > 0.0) ? 1.0 : ((u[e] < 0.0) ? -1.0 : 0.0);
        double bj = 0.0;
        if (j < p && sv[e] >= 0) {
            if (sv[e] > 0) {
                bj = sg * fmin(au / shrink, M);
            } else {
                const int r = L.rank[j];
                if (r < top) bj = sg * fmin(au / shrink, M);
                else if (r >= ba && r <= bb_end) bj = sg * (au - V / rho);
            }
        }
        bet[e] = bj;
    }
}

// ---------------------------------------------------------------------------
// Prox + FISTA momentum for every running slot (one workgroup per slot).  The
// gradient is the sum of the split-K partials of X^T R, read here directly:
// all loads of a thread's chunk are independent, so they are in flight together.
// ---------------------------------------------------------------------------
template <typename Ti, int PP, int W>
__global__ __launch_bounds__(64 * W) void k_prox_iter(const Ti *__restrict__ Gp, int gsplit,
                                                       double *__restrict__ B, double *__restrict__ Bprev,
                                                       Ti *__restrict__ Yi, const int8_t *__restrict__ stg,
                                                       SlotState ss, Consts c, Anchor an)
{
    constexpr int E = PP / (64 * W), NQ = E / 4;
    __shared__ ProxLds<PP> L;
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    if (ss.status[b] != SLOT_RUNNING) return;
    const int64_t off = (int64_t)b * c.ldp;
    const int64_t gstride = (int64_t)c.mpad * c.ldp;
    const int j0 = t * E;
    // every load of the step is issued here, before any result is needed
    const double th = ss.theta[b];
    const double tm = ss.tmom[b];
    const int itn = ss.iter[b];
    const int kbar = ss.kbar[b];
    int32_t *perm = ss.perm + (int64_t)b * c.pp;
    int pv[E];
#pragma unroll
    for (int q = 0; q < E / 4; ++q) {
        const int4 v = *reinterpret_cast<const int4 *>(perm + j0 + 4 * q);
        pv[4 * q] = v.x; pv[4 * q + 1] = v.y; pv[4 * q + 2] = v.z; pv[4 * q + 3] = v.w;
    }

    double g[E], bo[E], bp[E], u[E], y[E], bet[E], bcv[E];
    int sv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) { g[e] = 0.0; bo[e] = 0.0; bp[e] = 0.0; sv[e] = -1; bcv[e] = 0.0; }
    const bool anchored = an.gc != nullptr;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = j0 + 4 * q;
        const bool ok = j < c.ldp;
        const int jj = ok ? j : 0;
        ld4(B + off + jj, &bo[4 * q]);
        ld4(Bprev + off + jj, &bp[4 * q]);
        ld4_i8(stg + off + jj, &sv[4 * q]);
        if (anchored) {
            ld4(an.gc + off + jj, &g[4 * q]);
            ld4(an.bc + off + jj, &bcv[4 * q]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            bo[4 * q + e] = ok ? bo[4 * q + e] : 0.0;
            bp[4 * q + e] = ok ? bp[4 * q + e] : 0.0;
            sv[4 * q + e] = ok ? sv[4 * q + e] : -1;
            g[4 * q + e] = ok ? g[4 * q + e] : 0.0;
        }
    }
    // grad F(Y) = (grad F(beta_c) when anchored) + sum of the partials
    sum_splits<Ti, NQ, split_regs(W)>(Gp + off, gsplit, gstride, j0, c.ldp, g);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        y[e] = bo[e] + th * (bo[e] - bp[e]);
        u[e] = y[e] - c.eta * g[e];
    }
    masked_prox<PP, W>(L, u, sv, c.p, kbar, c.eta, c.lambda2, c.M, bet, perm, itn > 0, pv);
    // restart test (y - beta+)^T (beta+ - beta) > 0, then momentum
    double dot = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) dot += (y[e] - bet[e]) * (bet[e] - bo[e]);
    dot = blk_sum<W>(dot);
    double tn, thn;
    if (dot > 0.0) {
        tn = 1.0;
        thn = 0.0;
    } else {
        tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tm * tm));
        thn = (tm - 1.0) / tn;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = j0 + 4 * q;
        if (j < c.ldp) {
            double yn[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                yn[e] = bet[4 * q + e] + thn * (bet[4 * q + e] - bo[4 * q + e]) - bcv[4 * q + e];
            st4(Bprev + off + j, &bo[4 * q]);
            st4(B + off + j, &bet[4 * q]);
            store_y4(c, Yi, off + j, yn);
        }
    }
    if (t == 0) {
        ss.tmom[b] = tn;
        ss.theta[b] = thn;
        ss.iter[b] = itn + 1;
    }
}

// Standalone prox over a batch (step-level entry point).
template <int PP, int W>
__global__ __launch_bounds__(64 * W) void k_prox_batch(const double *__restrict__ U, const int8_t *__restrict__ stg,
                                                        const int32_t *__restrict__ kbar, double *__restrict__ Bout,
                                                        double eta, Consts c)
{
    constexpr int E = PP / (64 * W), NQ = E / 4;
    __shared__ ProxLds<PP> L;
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t off = (int64_t)b * c.ldp;
    const int j0 = t * E;
    double u[E], bet[E];
    int sv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) { u[e] = 0.0; sv[e] = -1; }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = j0 + 4 * q;
        const bool ok = j < c.ldp;
        const int jj = ok ? j : 0;
        ld4(U + off + jj, &u[4 * q]);
        ld4_i8(stg + off + jj, &sv[4 * q]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            u[4 * q + e] = ok ? u[4 * q + e] : 0.0;
            sv[4 * q + e] = ok ? sv[4 * q + e] : -1;
        }
    }
    int pv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) pv[e] = 0;  // no previous order
    masked_prox<PP, W>(L, u, sv, c.p, kbar[b], eta, c.lambda2, c.M, bet, nullptr, false, pv);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = j0 + 4 * q;
        if (j < c.ldp) st4(Bout + off + j, &bet[4 * q]);
    }
}

// ---------------------------------------------------------------------------
// Certificate finish (one workgroup per slot): paper Sec. 4.4,
// eqs. batched_primal_value_component / batched_dual_value_component.
//   q = (sum of the split-K partials of X^T zeta) / (2 lambda2)
//   g*(q) = sum_{J1} H_M(q_j) + TopSum_kbar{H_M(q_j)}_{free}  (kbar rounds of
//           argmax; fewer free entries than kbar sums them all)
//   g(beta) by Thm. 4.1: J1 contributes beta^2/2; on the free set with
//           a = |beta| sorted descending (top kbar by the same selection),
//           at most kbar nonzeros -> sum a^2/2; otherwise the first s in
//           0..kbar-1 with a_(s) >= tau >= a_(s+1), tau = (sum_{r>s} a_r)/(kbar-s)
//           gives sum_{r<=s} a_r^2/2 + tau (sum_{r>s} a_r)/2.  Points outside
//           dom g (|beta_j| > M, beta on J0, free sum > M kbar, relative slack
//           1e-9) give +inf.
//   Phi = sum l(X beta) + 2 lambda2 g(beta);  Psi = -sum l*(-zeta) - 2 lambda2 g*(q)
//   LB = max(LB, Psi), Phi_best = min(Phi_best, Phi); status update.
//   Rounding support = J1 + the kbar selected free indices (ascending);
//   branching index = the first selected (argmax |beta_j| over free, lowest
//   index on ties) -- Sec. 4.3.
// ---------------------------------------------------------------------------
template <int PP>
struct CertLds {
    double h[PP];
    double a[PP];
    double topa[128];
    int topi[128];
    int sup[256];
};

template <int PP, int W>
__global__ __launch_bounds__(64 * W) void k_cert_finish(const double *__restrict__ Qp, int qsplit,
                                                         const double *__restrict__ lsum,
                                                         const double *__restrict__ csum, int tiles_n,
                                                         const double *__restrict__ B,
                                                         double *__restrict__ Bbest,
                                                         const int8_t *__restrict__ stg, SlotState ss,
                                                         Consts c, int update_state, Anchor an,
                                                         const double *__restrict__ Bprev,
                                                         float *__restrict__ Yi)
{
    constexpr int E = PP / (64 * W), NQ = E / 4;
    constexpr int T = 64 * W;
    __shared__ CertLds<PP> L;
    const int b = blockIdx.x, t = threadIdx.x;
    if (update_state && ss.status[b] != SLOT_RUNNING) return;
    const int p = c.p;
    const int64_t off = (int64_t)b * c.ldp;
    const int64_t qstride = (int64_t)c.mpad * c.ldp;
    const int j0 = t * E;
    const int kbar = ss.kbar[b];
    const double inv2l = 1.0 / (2.0 * c.lambda2);
    const double slack = 1.0 + 1e-9;
    const double phi_prev = update_state ? ss.phi[b] : INFINITY;
    const double lb_prev = update_state ? ss.lb[b] : -INFINITY;

    double qv[E], bv[E];
    int sv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) { qv[e] = 0.0; bv[e] = 0.0; sv[e] = -1; }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = j0 + 4 * q;
        const bool ok = j < c.ldp;
        const int jj = ok ? j : 0;
        ld4(B + off + jj, &bv[4 * q]);
        ld4_i8(stg + off + jj, &sv[4 * q]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            bv[4 * q + e] = ok ? bv[4 * q + e] : 0.0;
            sv[4 * q + e] = ok ? sv[4 * q + e] : -1;
        }
    }
    sum_splits<double, NQ, split_regs(W)>(Qp + off, qsplit, qstride, j0, c.ldp, qv);
    // smooth parts
    double fl = 0.0, fc = 0.0;
    for (int q = t; q < tiles_n; q += T) {
        fl += lsum[(int64_t)q * c.mpad + b];
        fc += csum[(int64_t)q * c.mpad + b];
    }
    fl = blk_sum<W>(fl);
    fc = blk_sum<W>(fc);

    double gin = 0.0, g1 = 0.0, sum_a = 0.0, sum_a2 = 0.0;
    int nnz = 0, bad = 0, cin = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = j0 + e;
        double hj = -1.0, aj = -1.0;
        if (j < p) {
            const double q = qv[e] * inv2l;
            const double bj = bv[e];
            const double ab = fabs(bj);
            const int s = sv[e];
            if (s < 0) {
                if (bj != 0.0) bad = 1;
            } else {
                if (ab > c.M * slack) bad = 1;
                if (s > 0) {
                    ++cin;
                    gin += huber(q, c.M);
                    g1 += 0.5 * bj * bj;
                } else {
                    hj = huber(q, c.M);
                    aj = ab;
                    sum_a += ab;
                    sum_a2 += ab * ab;
                    nnz += (ab > 0.0) ? 1 : 0;
                }
            }
        }
        L.h[j] = hj;
        L.a[j] = aj;
    }
    // J1 indices in ascending order: exclusive scan of the per-thread counts
    {
        int pos = blk_excl_scan<W, int>(cin);
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (j0 + e < p && sv[e] > 0 && pos < 256) L.sup[pos++] = j0 + e;
    }
    const int nin = min(256, blk_sum_i<W>(cin));
    gin = blk_sum<W>(gin);
    g1 = blk_sum<W>(g1);
    sum_a = blk_sum<W>(sum_a);
    sum_a2 = blk_sum<W>(sum_a2);
    nnz = blk_sum_i<W>(nnz);
    bad = blk_sum_i<W>(bad);
    __syncthreads();

    // TopSum_kbar of H over the free set
    double topsum = 0.0;
    for (int r = 0; r < kbar; ++r) {
        double v = -1.0;
        int vi = 0x7fffffff;
        for (int j = t; j < PP; j += T) {
            const double hv = L.h[j];
            if (hv > v) { v = hv; vi = j; }
        }
        blk_argmax<W>(v, vi);
        if (v < 0.0) break;
        topsum += v;
        if (t == 0) L.h[vi] = -1.0;
        __syncthreads();
    }
    // kbar largest |beta| over the free set (ties to the lowest index)
    int ntop = 0;
    const int kcap = kbar < 128 ? kbar : 128;
    for (int r = 0; r < kcap; ++r) {
        double v = -1.0;
        int vi = 0x7fffffff;
        for (int j = t; j < PP; j += T) {
            const double av = L.a[j];
            if (av > v) { v = av; vi = j; }
        }
        blk_argmax<W>(v, vi);
        if (v < 0.0) break;
        if (t == 0) {
            L.topa[r] = v;
            L.topi[r] = vi;
            L.a[vi] = -1.0;
        }
        ++ntop;
        __syncthreads();
    }
    __syncthreads();
    // branching index: the largest free |beta|
    int jstar = -1;
    if (kbar > 0) {
        jstar = (ntop > 0) ? L.topi[0] : -1;
    } else {
        double v = -1.0;
        int vi = 0x7fffffff;
        for (int j = t; j < PP; j += T) {
            const double av = L.a[j];
            if (av > v) { v = av; vi = j; }
        }
        blk_argmax<W>(v, vi);
        jstar = (v >= 0.0) ? vi : -1;
    }

    // g on the free set (Thm. 4.1): with the free magnitudes sorted
    // descending, a_(0) >= a_(1) >= ..., the budget equation
    // sum_j min(1, a_j / tau) = kbar has the solution tau = tail(s) / (kbar - s)
    // for the s with a_(s-1) >= tau >= a_(s), where tail(s) = sum_{r >= s} a_(r);
    // then g_free = (1/2) sum_{r < s} a_(r)^2 + (1/2) tau tail(s).  The tails
    // are sums of non-negative terms (the entries outside the top kbar plus a
    // suffix of the top kbar), so no cancellation enters tau.
    double rest = 0.0;  // free magnitudes outside the selected top kbar
    for (int j = t; j < PP; j += T) rest += fmax(L.a[j], 0.0);
    rest = blk_sum<W>(rest);
    double gfree;
    if (bad) {
        gfree = INFINITY;
    } else if (nnz <= kbar) {
        gfree = 0.5 * sum_a2;
    } else if (kbar <= 0 || sum_a > c.M * kbar * slack) {
        gfree = INFINITY;
    } else {
        // the smallest s whose threshold lies in [a_(s), a_(s-1)] (relative
        // slack 1e-10 for the rounding of the sums; at a tie both sides give
        // the same value)
        int sel = -1;
        double tail = rest, tsel = 0.0;
        for (int s = kbar - 1; s >= 0; --s) {
            tail += L.topa[s];
            const double tau = tail / (double)(kbar - s);
            const double up = (s == 0) ? INFINITY : L.topa[s - 1];
            if (up >= tau * (1.0 - 1e-10) && tau >= L.topa[s] * (1.0 - 1e-10)) {
                sel = s;
                tsel = tail;
            }
        }
        if (sel >= 0) {
            double head2 = 0.0;
            for (int r = 0; r < sel; ++r) head2 += L.topa[r] * L.topa[r];
            gfree = 0.5 * head2 + 0.5 * (tsel / (double)(kbar - sel)) * tsel;
        } else {
            // not reached in exact arithmetic (a solution exists whenever
            // more than kbar entries are nonzero): solve the budget equation
            // by bisection over tau instead
            double tlo = 0.0, thi = fmax(L.topa[0], tail / (double)kbar);  // tail = every free magnitude
            for (int it = 0; it < 200; ++it) {
                const double tm = 0.5 * (tlo + thi);
                double h = 0.0;
                for (int r = t; r < kbar; r += T) h += fmin(1.0, L.topa[r] / tm);
                for (int j = t; j < PP; j += T) h += (L.a[j] > 0.0) ? fmin(1.0, L.a[j] / tm) : 0.0;
                h = blk_sum<W>(h);
                if (h > (double)kbar) tlo = tm;
                else thi = tm;
            }
            const double tau = 0.5 * (tlo + thi);
            double v = 0.0;
            for (int r = t; r < kbar; r += T) {
                const double a = L.topa[r];
                v += (a >= tau) ? 0.5 * a * a : 0.5 * tau * a;
            }
            for (int j = t; j < PP; j += T) {
                const double a = L.a[j];
                v += (a <= 0.0) ? 0.0 : ((a >= tau) ? 0.5 * a * a : 0.5 * tau * a);
            }
            gfree = blk_sum<W>(v);
        }
    }
    const double phi = fl + 2.0 * c.lambda2 * (g1 + gfree);
    const double psi = -fc - 2.0 * c.lambda2 * (gin + topsum);
    // In the engine the node's reported iterate is the one with the best
    // primal value, with its rounding support and branching index: they are
    // replaced only when this certificate improves that value.
    const bool nan = (psi != psi) || (phi != phi);
    const bool improved = !update_state || (!nan && phi < phi_prev);
    if (update_state && an.bc) {
        // this certificate becomes the anchor: beta_c = B, grad F(beta_c) =
        // -X^T zeta (the partial sums above), and the next step's
        // D = Y - beta_c = theta (B - Bprev)
        const double th = ss.theta[b];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = j0 + 4 * q;
            if (j < c.ldp) {
                double bp[4], gq[4], dq[4];
                ld4(Bprev + off + j, bp);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    gq[e] = -qv[4 * q + e];
                    dq[e] = th * (bv[4 * q + e] - bp[e]);
                }
                st4(an.bc + off + j, &bv[4 * q]);
                st4(an.gc + off + j, gq);
                store_y4(c, Yi, off + j, dq);
            }
        }
    }
    if (update_state && improved) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = j0 + 4 * q;
            if (j < c.ldp) st4(Bbest + off + j, &bv[4 * q]);
        }
    }
    // the iterate whose dual point certifies the node's bound (audits replay it)
    if (update_state && !nan && psi > lb_prev) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = j0 + 4 * q;
            if (j < c.ldp) st4(ss.blb + off + j, &bv[4 * q]);
        }
    }

    // rounding support: J1 (already ascending in L.sup) plus the selected free
    // indices, merged into ascending order
    if (t == 0 && improved) {
        int len = nin;
        for (int r = 0; r < ntop && len < 256; ++r) {
            const int v = L.topi[r];
            int y = len - 1;
            while (y >= 0 && L.sup[y] > v) { L.sup[y + 1] = L.sup[y]; --y; }
            L.sup[y + 1] = v;
            ++len;
        }
        int32_t *so = ss.sup + (int64_t)b * c.k;
        for (int r = 0; r < c.k; ++r) so[r] = (r < len) ? L.sup[r] : -1;
        ss.slen[b] = len < c.k ? len : c.k;
        ss.jstar[b] = jstar;
    }
    if (t == 0) {
        if (update_state) {
            // a NaN value means the iterate broke down: the node keeps its last
            // certified bound and stops with status ERROR
            double LB = ss.lb[b], PH = phi_prev;
            if (!nan && psi > LB) LB = psi;
            if (!nan && phi < PH) PH = phi;
            const double gap = (PH < INFINITY && LB > -INFINITY) ? (PH - LB) / fmax(fabs(PH), 1e-12) : INFINITY;
            ss.lb[b] = LB;
            ss.phi[b] = PH;
            ss.gap[b] = gap;
            const double ub = ss.ub[b];
            int stt = SLOT_RUNNING;
            if (nan) stt = 3;
            else if (LB >= ub - 1e-6 * fabs(ub)) stt = 1;
            else if (gap <= ss.tol[b]) stt = 0;
            // the node value lies below PH < ub - 1e-6 |ub|: no bound can prune it
            else if (ss.early[b] && isfinite(ub) && PH < ub - 1e-6 * fabs(ub)) stt = 4;
            else if (ss.iter[b] >= ss.max_iter[b]) stt = 2;
            ss.status[b] = stt;
        } else {
            ss.lb[b] = psi;
            ss.phi[b] = phi;
        }
    }
}

// ---------------------------------------------------------------------------
// Admission: scatter staged node records into their slots.
// Record: AdmitRec, then st[ldp] int8, then (aligned to 8) warm[ldp] float64.
// ---------------------------------------------------------------------------
template <typename Ti>
__global__ __launch_bounds__(64) void k_admit(const uint8_t *__restrict__ stage, int rec_bytes,
                                               double *B, double *Bprev, double *Bbest, Ti *Yi,
                                               int8_t *stg, SlotState ss, Consts c, Anchor an)
{
    const uint8_t *rec = stage + (int64_t)blockIdx.x * rec_bytes;
    const AdmitRec h = *reinterpret_cast<const AdmitRec *>(rec);
    const int8_t *sst = reinterpret_cast<const int8_t *>(rec + sizeof(AdmitRec));
    const int64_t woff = round_up((int64_t)sizeof(AdmitRec) + c.ldp, 8);
    const double *warm = reinterpret_cast<const double *>(rec + woff);
    const int b = h.slot;
    const int64_t off = (int64_t)b * c.ldp;
    for (int j = threadIdx.x; j < c.ldp; j += 64) {
        const int8_t s = sst[j];
        const double w = (h.has_warm && s >= 0 && j < c.p) ? warm[j] : 0.0;
        stg[off + j] = s;
        B[off + j] = w;
        Bprev[off + j] = w;
        Bbest[off + j] = w;
        ss.blb[off + j] = w;
        if (c.yp) {  // plane mode: the planes of w
            uint16_t hh, mm, ll;
            split3((float)w, hh, mm, ll);
            const int64_t pl = (int64_t)c.mpad * c.ldp;
            c.yp[off + j] = hh;
            c.yp[pl + off + j] = mm;
            if (c.nb > 2) c.yp[2 * pl + off + j] = ll;
        } else {
            Yi[off + j] = (Ti)w;
        }
        if (an.bc) {  // anchored at beta_c = 0 (D = w)
            an.bc[off + j] = 0.0;
            an.gc[off + j] = an.g0[j];
        }
    }
    if (an.sc) {
        double *scs = an.sc + (int64_t)b * c.npad;
        for (int i = threadIdx.x; i < c.npad; i += 64) scs[i] = 0.0;
    }
    if (threadIdx.x == 0) {
        ss.theta[b] = 0.0;
        ss.tmom[b] = 1.0;
        ss.lb[b] = -INFINITY;
        ss.phi[b] = INFINITY;
        ss.gap[b] = INFINITY;
        ss.ub[b] = h.ub;
        ss.tol[b] = h.tol;
        ss.early[b] = h.early;
        ss.iter[b] = 0;
        ss.max_iter[b] = h.max_iter;
        ss.kbar[b] = h.kbar;
        ss.jstar[b] = -1;
        ss.slen[b] = 0;
        ss.status[b] = SLOT_RUNNING;
    }
}

// ---------------------------------------------------------------------------
// Float64 matrix-vector product (power iteration): out[r] = sum_c A[r][c] v[c].
// One wave per row.
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(256) void k_matvec(const TA *__restrict__ A, int64_t lda, int rows,
                                                 int cols, const double *__restrict__ v,
                                                 double *__restrict__ out)
{
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (r >= rows) return;
    const TA *a = A + (int64_t)r * lda;
    double s = 0.0;
    for (int j = l; j < cols; j += 64) {
        double aj;
        if constexpr (sizeof(TA) == 2) aj = (double)bf16_to_f(a[j]);
        else aj = (double)a[j];
        s += aj * v[j];
    }
    s = wave_sum(s);
    if (l == 0) out[r] = s;
}

// Transposed copy XT[j][i] = X[i][j] (padding stays zero: XT is pre-zeroed).
template <typename TA>
__global__ __launch_bounds__(256) void k_transpose(const TA *__restrict__ X, TA *__restrict__ XT,
                                                    int n, int p, int ldp, int npad)
{
    __shared__ TA tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx over j, by over i
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        tile[r][tx] = (i < n && j < p) ? X[(int64_t)i * ldp + j] : (TA)0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;
        if (j < p && i < n) XT[(int64_t)j * npad + i] = tile[tx][r];
    }
}


// ===========================================================================
// Launchers
// ===========================================================================
// rows: the A operand's (padded) row count, a multiple of 64.  BM = 32 when
// 64-row tiles would leave fewer than two workgroups per CU (256 CUs), so
// that resident workgroups hide each other's load latency.
template <typename TA, typename TB, typename TC, int MODE>
static void gemm(hipStream_t s, GemmArgs g, int rows, int tiles_n, int splits, int bm_force = 0)
{
    g.tiles_n = tiles_n;
    g.nsplit = splits;
    const bool small = (int64_t)(rows / 64) * tiles_n * splits < 512;
    const int bm = (bm_force == 32 || bm_force == 64) ? bm_force : (small ? 32 : 64);
    g.tiles_m = rows / bm;
    int nblocks;
    if (splits > 1) nblocks = 8 * g.tiles_m * tiles_n * ((splits + 7) / 8);
    else if (g.tiles_m >= 8) nblocks = (g.tiles_m + 7) / 8 * 8 * tiles_n;
    else nblocks = g.tiles_m * tiles_n;
    dim3 grid(nblocks, 1);
    if (bm == 32) KBNB_LAUNCH((k_gemm_tn<TA, TB, TC, MODE, 32>), grid, dim3(256), 0, s, g);
    else KBNB_LAUNCH((k_gemm_tn<TA, TB, TC, MODE, 64>), grid, dim3(256), 0, s, g);
}


void launch_fwd_dloss(hipStream_t s, int xtype, bool iter_f64, const void *X, const void *Yi,
                      void *R, const double *y, const Consts &c, const int32_t *status,
                      const Anchor &an)
{
    GemmArgs g{};
    g.col_status = status;
    g.A = X; g.lda = c.ldp; g.B = Yi; g.ldb = c.ldp; g.C = R; g.ldc = c.npad;
    g.k_len = c.ldp; g.k_chunk = c.ldp;
    g.n = c.n; g.loss = c.loss; g.y = y;
    g.sc = an.sc;
    const int tn = c.mact / GEMM_BN;
    if (c.yp) {  // plane mode: stream the tiled X against the planes of Y
        g.A = c.xtile; g.lda = c.nkb_x; g.rows_a = c.npad;
        g.B = c.yp; g.b_plane = (int64_t)c.mpad * c.ldp;
        g.C = c.rp; g.c_plane = (int64_t)c.mpad * c.npad; g.rows_c = c.npad;
        (void)launch_gemm_stream(s, an.sc ? EPI_DLOSS_ANCHOR : EPI_DLOSS, g, c.npad, tn, 1,
                                 stream_wave_rows(c.tile_rows, c.npad, tn, 1), c.nb);
        return;
    }
    // outside plane mode a float32 iteration has float32 X
    if (an.sc && !iter_f64) {
        gemm<float, float, float, EPI_DLOSS_ANCHOR>(s, g, c.npad, tn, 1, c.tile_rows);
    } else if (iter_f64) {
        if (xtype == XT_F64) gemm<double, double, double, EPI_DLOSS>(s, g, c.npad, tn, 1, c.tile_rows);
        else if (xtype == XT_F32) gemm<float, double, double, EPI_DLOSS>(s, g, c.npad, tn, 1, c.tile_rows);
        else gemm<uint16_t, double, double, EPI_DLOSS>(s, g, c.npad, tn, 1, c.tile_rows);
    } else {
        gemm<float, float, float, EPI_DLOSS>(s, g, c.npad, tn, 1, c.tile_rows);
    }
}

void launch_bwd(hipStream_t s, int xtype, bool iter_f64, const void *XT, const void *R,
                void *Gp, int gsplit, int gchunk, const Consts &c, const int32_t *status)
{
    GemmArgs g{};
    g.col_status = status;
    g.A = XT; g.lda = c.npad; g.B = R; g.ldb = c.npad; g.C = Gp; g.ldc = c.ldp;
    g.split_stride = (int64_t)c.mpad * c.ldp;
    g.k_len = c.npad; g.k_chunk = gchunk; g.rows_valid = c.ldp;
    const int tn = c.mact / GEMM_BN;
    if (c.yp) {  // plane mode: stream the tiled X^T against the planes of R
        g.A = c.xttile; g.lda = c.nkb_xt; g.rows_a = c.pm;
        g.B = c.rp; g.b_plane = (int64_t)c.mpad * c.npad;
        (void)launch_gemm_stream(s, EPI_STORE, g, c.pm, tn, gsplit, stream_wave_rows(c.tile_rows, c.pm, tn, gsplit),
                                 c.nb);
        return;
    }
    if (iter_f64) {
        if (xtype == XT_F64) gemm<double, double, double, EPI_STORE>(s, g, c.pm, tn, gsplit, c.tile_rows);
        else if (xtype == XT_F32) gemm<float, double, double, EPI_STORE>(s, g, c.pm, tn, gsplit, c.tile_rows);
        else gemm<uint16_t, double, double, EPI_STORE>(s, g, c.pm, tn, gsplit, c.tile_rows);
    } else {
        gemm<float, float, float, EPI_STORE>(s, g, c.pm, tn, gsplit, c.tile_rows);
    }
}

void launch_cert_fwd(hipStream_t s, int xtype, const void *X, const double *B, double *Z,
                     const double *y, double *lsum, double *csum, const Consts &c,
                     const int32_t *status, double *sc_out)
{
    GemmArgs g{};
    g.col_status = status;
    g.sc_out = sc_out;
    g.A = X; g.lda = c.ldp; g.B = B; g.ldb = c.ldp; g.C = Z; g.ldc = c.npad;
    g.k_len = c.ldp; g.k_chunk = c.ldp;
    g.n = c.n; g.loss = c.loss; g.y = y; g.lsum = lsum; g.csum = csum; g.ldsum = c.mpad;
    const int tn = c.mact / GEMM_BN;
    if (xtype == XT_F64) gemm<double, double, double, EPI_CERT>(s, g, c.npad, tn, 1);
    else if (xtype == XT_F32) gemm<float, double, double, EPI_CERT>(s, g, c.npad, tn, 1);
    else gemm<uint16_t, double, double, EPI_CERT>(s, g, c.npad, tn, 1);
}

void launch_cert_bwd(hipStream_t s, int xtype, const void *XT, const double *Z, double *Qp,
                     int qsplit, int qchunk, const Consts &c, const int32_t *status)
{
    GemmArgs g{};
    g.col_status = status;
    g.A = XT; g.lda = c.npad; g.B = Z; g.ldb = c.npad; g.C = Qp; g.ldc = c.ldp;
    g.split_stride = (int64_t)c.mpad * c.ldp;
    g.k_len = c.npad; g.k_chunk = qchunk; g.rows_valid = c.ldp;
    const int tn = c.mact / GEMM_BN;
    if (xtype == XT_F64) gemm<double, double, double, EPI_STORE>(s, g, c.pm, tn, qsplit);
    else if (xtype == XT_F32) gemm<float, double, double, EPI_STORE>(s, g, c.pm, tn, qsplit);
    else gemm<uint16_t, double, double, EPI_STORE>(s, g, c.pm, tn, qsplit);
}

// PP: padded column length of the per-node kernels; W: waves per node.
#define KBNB_PP_DISPATCH(P, CALL)                                                  \
    do {                                                                           \
        if ((P) <= 256) { constexpr int PP = 256, W = NodeWaves<PP>::W; CALL; }    \
        else if ((P) <= 512) { constexpr int PP = 512, W = NodeWaves<PP>::W; CALL; } \
        else if ((P) <= 1024) { constexpr int PP = 1024, W = NodeWaves<PP>::W; CALL; } \
        else if ((P) <= 2048) { constexpr int PP = 2048, W = NodeWaves<PP>::W; CALL; } \
        else if ((P) <= 4096) { constexpr int PP = 4096, W = NodeWaves<PP>::W; CALL; } \
        else { constexpr int PP = 8192, W = NodeWaves<PP>::W; CALL; }              \
    } while (0)

void launch_prox_iter(hipStream_t s, bool iter_f64, const void *Gp, int gsplit, double *B,
                      double *Bprev, void *Yi, const int8_t *st, SlotState ss, const Consts &c,
                      const Anchor &an)
{
    if (iter_f64) {
        KBNB_PP_DISPATCH(c.p, KBNB_LAUNCH((k_prox_iter<double, PP, W>), dim3(min(c.m, c.mact)), dim3(64 * W), 0, s,
                                                 (const double *)Gp, gsplit, B, Bprev, (double *)Yi, st, ss, c, an));
    } else {
        KBNB_PP_DISPATCH(c.p, KBNB_LAUNCH((k_prox_iter<float, PP, W>), dim3(min(c.m, c.mact)), dim3(64 * W), 0, s,
                                                 (const float *)Gp, gsplit, B, Bprev, (float *)Yi, st, ss, c, an));
    }
}

void launch_prox_batch(hipStream_t s, const double *U, const int8_t *st, const int32_t *kbar,
                       double *Bout, int m, double eta, const Consts &c)
{
    KBNB_PP_DISPATCH(c.p, KBNB_LAUNCH((k_prox_batch<PP, W>), dim3(m), dim3(64 * W), 0, s, U, st, kbar,
                                             Bout, eta, c));
}

void launch_cert_finish(hipStream_t s, const double *Qp, int qsplit, const double *lsum,
                        const double *csum, int tiles_n, const double *B, double *Bbest,
                        const int8_t *st, SlotState ss, const Consts &c, int update_state,
                        const Anchor &an, const double *Bprev, float *Yi)
{
    KBNB_PP_DISPATCH(c.p, KBNB_LAUNCH((k_cert_finish<PP, W>), dim3(min(c.m, c.mact)), dim3(64 * W), 0, s, Qp, qsplit,
                                             lsum, csum, tiles_n, B, Bbest, st, ss, c, update_state,
                                             an, Bprev, Yi));
}

void launch_admit(hipStream_t s, bool iter_f64, const uint8_t *stage, int count, int rec_bytes,
                  double *B, double *Bprev, double *Bbest, void *Yi, int8_t *st, SlotState ss,
                  const Consts &c, const Anchor &an)
{
    if (count <= 0) return;
    if (iter_f64)
        KBNB_LAUNCH((k_admit<double>), dim3(count), dim3(64), 0, s, stage, rec_bytes, B, Bprev,
                           Bbest, (double *)Yi, st, ss, c, an);
    else
        KBNB_LAUNCH((k_admit<float>), dim3(count), dim3(64), 0, s, stage, rec_bytes, B, Bprev,
                           Bbest, (float *)Yi, st, ss, c, an);
}

void launch_matvec_f64(hipStream_t s, int xtype, const void *A, int64_t lda, int rows, int cols,
                       const double *v, double *out)
{
    dim3 grid((rows + 3) / 4);
    if (xtype == XT_F64)
        KBNB_LAUNCH((k_matvec<double>), grid, dim3(256), 0, s, (const double *)A, lda, rows, cols, v, out);
    else if (xtype == XT_F32)
        KBNB_LAUNCH((k_matvec<float>), grid, dim3(256), 0, s, (const float *)A, lda, rows, cols, v, out);
    else
        KBNB_LAUNCH((k_matvec<uint16_t>), grid, dim3(256), 0, s, (const uint16_t *)A, lda, rows, cols, v, out);
}

// ---------------------------------------------------------------------------
// Fixed-model reliance over a pool of sparse models (appendix on variable
// importance over the Rashomon set): for record m with coefficients c on the
// labels lab of its support,
//   R = (1/n) sum_i [ l(eta_i - x_{i,lab_r} c_r, y_i) - l(eta_i, y_i) ],
//   eta = X_{:,lab} c,
// one workgroup per record, float64 from the stored values of X^T (rows of
// X^T are columns of X, contiguous over i).  Labels are taken in groups of
// 16 (eta is recomputed per group).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cvt_d(double v) { return v; }
__device__ __forceinline__ double cvt_d(float v) { return (double)v; }
__device__ __forceinline__ double cvt_d(uint16_t v) { return (double)bf16_to_f(v); }

template <typename TA>
__global__ __launch_bounds__(256) void k_reliance(const TA *__restrict__ XT, int64_t npad, int n, int loss,
                                                  const double *__restrict__ y, const int32_t *__restrict__ lab,
                                                  const int64_t *__restrict__ off, const double *__restrict__ coef,
                                                  double *__restrict__ out)
{
    constexpr int RG = 16;
    __shared__ double red[4][RG];
    const int m = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t o0 = off[m];
    const int kl = (int)(off[m + 1] - o0);
    const int32_t *L = lab + o0;
    const double *C = coef + o0;
    for (int g0 = 0; g0 < kl; g0 += RG) {
        double acc[RG];
#pragma unroll
        for (int r = 0; r < RG; ++r) acc[r] = 0.0;
        for (int i = tid; i < n; i += 256) {
            double eta = 0.0;
            for (int r = 0; r < kl; ++r) eta += cvt_d(XT[(int64_t)L[r] * npad + i]) * C[r];
            const double yi = y[i];
            const double base = loss_d(loss, eta, yi);
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                if (g0 + r < kl) {
                    const double xv = cvt_d(XT[(int64_t)L[g0 + r] * npad + i]);
                    acc[r] += loss_d(loss, eta - xv * C[g0 + r], yi) - base;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            double v = wave_sum(acc[r]);
            if (lane == 0) red[wave][r] = v;
        }
        __syncthreads();
        if (tid < RG && g0 + tid < kl)
            out[o0 + g0 + tid] = (red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]) / (double)n;
        __syncthreads();
    }
}

void launch_reliance(hipStream_t s, int xtype, const void *XT, int64_t npad, int n, int loss, const double *y,
                     const int32_t *lab, const int64_t *off, const double *coef, int nrec, double *out)
{
    if (nrec <= 0) return;
    dim3 grid(nrec);
    if (xtype == XT_F64)
        KBNB_LAUNCH((k_reliance<double>), grid, dim3(256), 0, s, (const double *)XT, npad, n, loss, y, lab, off, coef, out);
    else if (xtype == XT_F32)
        KBNB_LAUNCH((k_reliance<float>), grid, dim3(256), 0, s, (const float *)XT, npad, n, loss, y, lab, off, coef, out);
    else
        KBNB_LAUNCH((k_reliance<uint16_t>), grid, dim3(256), 0, s, (const uint16_t *)XT, npad, n, loss, y, lab, off, coef, out);
}

// ---------------------------------------------------------------------------
// Batched support re-optimisation (Sec. 4.3): for each support S of at most
// KB features,
//   v(S) = min { F(X_S beta) + lambda2 ||beta||^2 : |beta_j| <= M },
// the relaxation of the node J1 = S, J0 = the rest, which is exact.  One
// workgroup (256 threads) per support, float64 throughout, from the stored
// values of the support's rows of X^T (columns of X, contiguous over i):
//   1. the Gram matrix X_S^T X_S in one pass over LDS row tiles; the step
//      1 / L uses L = c_l min(||G||_F, max_r sum_q |G_rq|) >= c_l lambda_max;
//   2. accelerated proximal gradient on the |S| coordinates (prox of
//      lambda2 beta^2 plus the box: clip(u / (1 + 2 eta lambda2), +-M)),
//      gradient restart, one pass over X_S per step;
//   3. every `cert_every` steps the certificate at beta: Phi = F(X_S beta) +
//      lambda2 ||beta||^2 and the dual value at zeta = -l'(X_S beta),
//      Psi = -sum l*(-zeta) - 2 lambda2 sum_j H_M(x_j^T zeta / (2 lambda2)),
//      a lower bound of v(S) by weak duality; stop when
//      (Phi_best - Psi_best) <= tol |Phi_best|.
// Returns the best certified beta (it attains value = Phi_best), the best
// Psi, status (0 converged, 2 iteration limit) and the steps taken.
// ---------------------------------------------------------------------------
struct SupportArgs {
    // split-row version (k_support_mw_init, k_support_mw_step): workgroups
    // per support, and the state of each support kept between step launches
    int groups;
    int init_groups;    // workgroups per support of the set-up (Gram matrix) launch
    double *part;       // [count][groups][KB + 2] partial sums of the current step
    double *gram;       // [count][init_groups][KB (KB + 1) / 2] partial Gram matrices
    double *st;         // [count][8] eta, theta, t, best primal, best dual, finished
    double *vec;        // [count][4][KB] beta, Y, best-primal beta, best-dual beta
    int32_t *step;      // [count] step index
    int32_t *arrive;    // [count] workgroups through the current launch (0 between launches)
    int32_t *ndone;     // supports finished
    const void *XT;
    int64_t npad;
    int n, loss;
    const double *y;
    const int32_t *lab;    // labels of support m: lab[off[m] .. off[m + 1])
    const int64_t *off;
    const double *warm;    // nullable: starting coefficients, same layout
    double lambda2, M, c_loss, tol;
    int max_iter, cert_every;
    double *beta_out;      // same layout as lab
    double *beta_lb_out;   // nullable: coefficients whose dual point gave `lower`
    double *value, *lower;
    int32_t *status, *iters;
};

template <typename TA, int KB>
__global__ __launch_bounds__(256) void k_support_eval(SupportArgs a)
{
    constexpr int TR = 2048 / KB;  // rows per Gram tile (128, 64 or 32)
    constexpr int NPAIR = KB * (KB + 1) / 2;
    constexpr int PT = (NPAIR + 255) / 256;
    __shared__ int32_t L[KB];
    __shared__ double Bv[KB], Bp[KB], Yv[KB], Bb[KB], Bn[KB], Bd[KB];
    __shared__ double G[KB][KB + 1];
    __shared__ double tile[TR][KB + 1];
    __shared__ double red[4][KB + 2];
    __shared__ double sc[8];  // eta, theta, tmom, phi_best, psi_best, done, new best primal, new best dual
    const TA *XT = reinterpret_cast<const TA *>(a.XT);
    const int m = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t o0 = a.off[m];
    const int kl = (int)(a.off[m + 1] - o0);
    if (tid < KB) {
        L[tid] = (tid < kl) ? a.lab[o0 + tid] : 0;
        double w = (a.warm && tid < kl) ? a.warm[o0 + tid] : 0.0;
        w = fmin(fmax(w, -a.M), a.M);
        Bv[tid] = w;
        Bp[tid] = w;
        Yv[tid] = w;
        Bb[tid] = w;
        Bd[tid] = w;
    }
    __syncthreads();

    // 1. Gram matrix: thread t owns pairs t + 256 v, (r, q) with r <= q
    int pr[PT], pq[PT];
    double gacc[PT];
#pragma unroll
    for (int v = 0; v < PT; ++v) {
        int pi = tid + 256 * v, r = 0;
        const int np = kl * (kl + 1) / 2;
        if (pi < np) {
            while (pi >= kl - r) { pi -= kl - r; ++r; }
            pr[v] = r;
            pq[v] = r + pi;
        } else {
            pr[v] = -1;
            pq[v] = 0;
        }
        gacc[v] = 0.0;
    }
    for (int i0 = 0; i0 < a.n && kl > 0; i0 += TR) {
        for (int e = tid; e < TR * kl; e += 256) {
            const int r = e / TR, row = e - r * TR, i = i0 + row;
            tile[row][r] = (i < a.n) ? cvt_d(XT[(int64_t)L[r] * a.npad + i]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < PT; ++v) {
            if (pr[v] >= 0) {
                double acc = 0.0;
                for (int row = 0; row < TR; ++row) acc += tile[row][pr[v]] * tile[row][pq[v]];
                gacc[v] += acc;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < PT; ++v) {
        if (pr[v] >= 0) {
            G[pr[v]][pq[v]] = gacc[v];
            G[pq[v]][pr[v]] = gacc[v];
        }
    }
    __syncthreads();
    if (tid < 64) {
        double rs = 0.0, fr = 0.0;
        if (tid < kl)
            for (int q = 0; q < kl; ++q) {
                rs += fabs(G[tid][q]);
                fr += G[tid][q] * G[tid][q];
            }
        double gmax = rs;
        for (int o = 32; o > 0; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o));
        fr = wave_sum(fr);
        if (tid == 0) {
            double lam = fmin(sqrt(fr), gmax);
            const double Lc = a.c_loss * lam;
            sc[0] = (Lc > 0.0) ? 1.0 / (Lc * 1.000001) : 1.0;
            sc[1] = 0.0;        // theta
            sc[2] = 1.0;        // t
            sc[3] = INFINITY;   // best primal
            sc[4] = -INFINITY;  // best dual
            sc[5] = 0.0;        // done
        }
    }
    __syncthreads();
    const double eta = sc[0];
    const double shrink = 1.0 / (1.0 + 2.0 * eta * a.lambda2);
    int it = 0;
    for (;; ++it) {
        const bool cert = (it % a.cert_every) == 0 || it >= a.max_iter;
        // pass over the rows: gradient at Y, or (cert) the certificate at beta
        double g[KB];
#pragma unroll
        for (int r = 0; r < KB; ++r) g[r] = 0.0;
        double al = 0.0, ac = 0.0;
        const double *pt = cert ? Bv : Yv;
        // U rows per thread at a time (rows past n read row 0 and contribute
        // 0), so their loads are in flight together; U shrinks as KB grows to
        // keep the row values the two passes share in registers
        constexpr int U = (KB <= 16) ? 4 : ((KB <= 32) ? 2 : 1);
        for (int i0 = tid; i0 < a.n; i0 += 256 * U) {
            int64_t ri[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ok[u] = i0 + 256 * u < a.n;
                ri[u] = ok[u] ? i0 + 256 * u : 0;
            }
            double sv[U], yv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                sv[u] = 0.0;
                yv[u] = a.y[ri[u]];
            }
            // every column slot is read (slots past the support hold column
            // 0 with weight 0), so all U * KB loads are issued together
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                const TA *col = XT + (int64_t)L[r] * a.npad;
#pragma unroll
                for (int u = 0; u < U; ++u) sv[u] += cvt_d(col[ri[u]]) * pt[r];
            }
            double dv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double yi = yv[u];
                if (cert) {
                    double z, lv, cv;
                    cert_terms(a.loss, sv[u], yi, z, lv, cv);
                    al += ok[u] ? lv : 0.0;
                    ac += ok[u] ? cv : 0.0;
                    dv[u] = ok[u] ? z : 0.0;
                } else {
                    dv[u] = ok[u] ? dloss_d(a.loss, sv[u], yi) : 0.0;
                }
            }
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                const TA *col = XT + (int64_t)L[r] * a.npad;
                double acc = 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u) acc += cvt_d(col[ri[u]]) * dv[u];
                g[r] += acc;  // unused past the support
            }
        }
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            if (r < kl) {
                const double v = wave_sum(g[r]);
                if (lane == 0) red[wave][r] = v;
            }
        }
        if (cert) {
            al = wave_sum(al);
            ac = wave_sum(ac);
            if (lane == 0) {
                red[wave][KB] = al;
                red[wave][KB + 1] = ac;
            }
        }
        __syncthreads();
        if (cert) {
            if (tid < 64) {
                // q_r = x_r^T zeta / (2 lambda2); penalty and dual terms over r < kl
                double pen = 0.0, dterm = 0.0;
                if (tid < kl) {
                    const double qv = (red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]) / (2.0 * a.lambda2);
                    pen = Bv[tid] * Bv[tid];
                    dterm = huber(qv, a.M);
                }
                pen = wave_sum(pen);
                dterm = wave_sum(dterm);
                if (tid == 0) {
                    const double fl = red[0][KB] + red[1][KB] + red[2][KB] + red[3][KB];
                    const double fc = red[0][KB + 1] + red[1][KB + 1] + red[2][KB + 1] + red[3][KB + 1];
                    const double phi = fl + a.lambda2 * pen;
                    const double psi = -fc - 2.0 * a.lambda2 * dterm;
                    if (phi < sc[3]) {
                        sc[3] = phi;
                        sc[6] = 1.0;  // take beta as the best
                    } else {
                        sc[6] = 0.0;
                    }
                    sc[7] = (psi > sc[4]) ? 1.0 : 0.0;
                    if (psi > sc[4]) sc[4] = psi;
                    const double den = fmax(fabs(sc[3]), 1e-12);
                    sc[5] = ((sc[3] - sc[4]) <= a.tol * den || it >= a.max_iter) ? 1.0 : 0.0;
                }
            }
            __syncthreads();
            if (tid < kl && sc[6] != 0.0) Bb[tid] = Bv[tid];
            if (tid < kl && sc[7] != 0.0) Bd[tid] = Bv[tid];
            if (sc[5] != 0.0) break;
            __syncthreads();
            continue;  // the certificate pass takes no step
        }
        // proximal step from Y, restart test, momentum
        if (tid < 64) {
            double dot = 0.0;
            if (tid < kl) {
                const double gr = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
                const double u = Yv[tid] - eta * gr;
                const double bn = fmin(fmax(u * shrink, -a.M), a.M);
                Bn[tid] = bn;
                dot = (Yv[tid] - bn) * (bn - Bv[tid]);
            }
            dot = wave_sum(dot);
            if (tid == 0) {
                const double tm = sc[2];
                if (dot > 0.0) {
                    sc[2] = 1.0;
                    sc[1] = 0.0;
                } else {
                    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tm * tm));
                    sc[1] = (tm - 1.0) / tn;
                    sc[2] = tn;
                }
            }
        }
        __syncthreads();
        if (tid < kl) {
            const double th = sc[1];
            Bp[tid] = Bv[tid];
            Bv[tid] = Bn[tid];
            Yv[tid] = Bn[tid] + th * (Bn[tid] - Bp[tid]);
        }
        __syncthreads();
    }
    if (tid < kl) a.beta_out[o0 + tid] = Bb[tid];
    if (tid < kl && a.beta_lb_out) a.beta_lb_out[o0 + tid] = Bd[tid];
    if (tid == 0) {
        a.value[m] = sc[3];
        a.lower[m] = fmin(sc[4], sc[3]);
        a.status[m] = (sc[3] - sc[4] <= a.tol * fmax(fabs(sc[3]), 1e-12)) ? 0 : 2;
        a.iters[m] = it;
    }
}

// ---------------------------------------------------------------------------
// Re-optimisation with the rows of each support split over a.groups
// workgroups (tall instances, where one workgroup walking every row per step
// is latency-bound).  Workgroup g of support m owns a contiguous block of
// rows.  k_support_mw_init forms the Gram matrix from the groups' partial
// sums and sets up each support's state; then each launch of
// k_support_mw_step is one step: every workgroup makes one pass over its
// rows forming s_i = x_{i,S} . pt and, in the same pass, its part of the
// gradient (or, at a certificate, of q = X_S^T zeta and the loss sums); the
// last workgroup of the support to finish (an atomic arrival count) adds
// the parts in group order and applies the update of k_support_eval.  No
// workgroup ever waits for another, so the launch needs no residency
// guarantee.  A finished support's workgroups return at once; a support
// finishes at step max_iter at the latest, so max_iter + 1 step launches
// finish every support.
// ---------------------------------------------------------------------------
// rows [r0, r1) of workgroup gg of ng; block starts are multiples of RT
template <int RT = 1>
__device__ __forceinline__ void support_rows(const SupportArgs &a, int ng, int gg, int &r0, int &r1)
{
    const int per = ((a.n + ng - 1) / ng + RT - 1) / RT * RT;
    r0 = min(a.n, gg * per);
    r1 = min(a.n, r0 + per);
}

// Rows per lane and load in the split-row step: the lane reads RT consecutive
// rows of each of the KB column slots with one vector load, 256 bytes of
// registers for the KB loads together (128 above 16 slots, where the KB
// gradient sums take the rest of the registers).
template <typename TA, int KB> struct MwRows {
    static constexpr int B = (KB <= 16 ? 256 : 128) / (KB * (int)sizeof(TA));
    static constexpr int RT = B < 1 ? 1 : B;
};
template <int NB> struct RawVec;
template <> struct RawVec<16> { typedef uint4 t; };
template <> struct RawVec<8> { typedef uint2 t; };
template <> struct RawVec<4> { typedef uint32_t t; };
template <> struct RawVec<2> { typedef uint16_t t; };
// element j of RT consecutive stored values loaded as one raw vector
template <typename TA, typename RV> __device__ __forceinline__ double raw_elem(const RV &v, int j)
{
    return cvt_d(reinterpret_cast<const TA *>(&v)[j]);
}

// sum_{q < ng} v[q * stride], added in q order, with eight loads in flight
__device__ __forceinline__ double sum_in_order(const double *v, int ng, int64_t stride)
{
    double t = 0.0;
    int q = 0;
    for (; q + 8 <= ng; q += 8) {
        double w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = v[(q + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) t += w[u];
    }
    for (; q < ng; ++q) t += v[q * stride];
    return t;
}

// every thread: true in the workgroup that arrives last of the ng of support m
__device__ __forceinline__ bool support_last_arrival(const SupportArgs &a, int m, int ng, int *flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's partial sums before its arrival
        *flag = atomicAdd(&a.arrive[m], 1) == ng - 1;
    }
    __syncthreads();
    const bool last = *flag != 0;
    if (last) __threadfence();  // ... and every other workgroup's after it
    return last;
}

template <typename TA, int KB>
__global__ __launch_bounds__(256) void k_support_mw_init(SupportArgs a)
{
    constexpr int TR = 2048 / KB;
    constexpr int NPAIR = KB * (KB + 1) / 2;
    constexpr int PT = (NPAIR + 255) / 256;
    __shared__ int32_t L[KB];
    __shared__ double G[KB][KB + 1];
    __shared__ double tile[TR][KB + 1];
    __shared__ int s_last;
    const TA *XT = reinterpret_cast<const TA *>(a.XT);
    const int ng = a.init_groups, m = blockIdx.x / ng, gg = blockIdx.x % ng;
    const int tid = threadIdx.x;
    const int64_t o0 = a.off[m];
    const int kl = (int)(a.off[m + 1] - o0);
    int r0, r1;
    support_rows(a, ng, gg, r0, r1);
    if (tid < KB) L[tid] = (tid < kl) ? a.lab[o0 + tid] : 0;
    if (blockIdx.x == 0 && tid == 0) *a.ndone = 0;
    __syncthreads();
    // partial Gram matrix of this workgroup's rows: thread t owns pairs t + 256 v
    int pr[PT], pq[PT];
    double gacc[PT];
#pragma unroll
    for (int v = 0; v < PT; ++v) {
        int pi = tid + 256 * v, r = 0;
        const int np = kl * (kl + 1) / 2;
        if (pi < np) {
            while (pi >= kl - r) { pi -= kl - r; ++r; }
            pr[v] = r;
            pq[v] = r + pi;
        } else {
            pr[v] = -1;
            pq[v] = 0;
        }
        gacc[v] = 0.0;
    }
    for (int i0 = r0; i0 < r1 && kl > 0; i0 += TR) {
        for (int e = tid; e < TR * kl; e += 256) {
            const int r = e / TR, row = e - r * TR, i = i0 + row;
            tile[row][r] = (i < r1) ? cvt_d(XT[(int64_t)L[r] * a.npad + i]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < PT; ++v) {
            if (pr[v] >= 0) {
                double acc = 0.0;
                for (int row = 0; row < TR; ++row) acc += tile[row][pr[v]] * tile[row][pq[v]];
                gacc[v] += acc;
            }
        }
        __syncthreads();
    }
    double *gp = a.gram + ((int64_t)m * ng + gg) * NPAIR;
#pragma unroll
    for (int v = 0; v < PT; ++v)
        if (tid + 256 * v < NPAIR) gp[tid + 256 * v] = gacc[v];
    if (!support_last_arrival(a, m, ng, &s_last)) return;
    // the last workgroup: the Gram matrix in group order, the step size and
    // the starting state
#pragma unroll
    for (int v = 0; v < PT; ++v) {
        if (pr[v] >= 0) {
            const double t = sum_in_order(a.gram + (int64_t)m * ng * NPAIR + tid + 256 * v, ng, NPAIR);
            G[pr[v]][pq[v]] = t;
            G[pq[v]][pr[v]] = t;
        }
    }
    __syncthreads();
    double *st = a.st + 8 * (int64_t)m;
    if (tid < 64) {
        double rs = 0.0, fr = 0.0;
        if (tid < kl)
            for (int q = 0; q < kl; ++q) {
                rs += fabs(G[tid][q]);
                fr += G[tid][q] * G[tid][q];
            }
        double gmax = rs;
        for (int o = 32; o > 0; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o));
        fr = wave_sum(fr);
        if (tid == 0) {
            const double Lc = a.c_loss * fmin(sqrt(fr), gmax);
            st[0] = (Lc > 0.0) ? 1.0 / (Lc * 1.000001) : 1.0;
            st[1] = 0.0;        // theta
            st[2] = 1.0;        // t
            st[3] = INFINITY;   // best primal
            st[4] = -INFINITY;  // best dual
            st[5] = 0.0;        // finished
            a.step[m] = 0;
            a.arrive[m] = 0;
        }
    }
    if (tid < KB) {
        double w = (a.warm && tid < kl) ? a.warm[o0 + tid] : 0.0;
        w = (tid < kl) ? fmin(fmax(w, -a.M), a.M) : 0.0;
        double *vec = a.vec + (int64_t)m * 4 * KB;
#pragma unroll
        for (int c = 0; c < 4; ++c) vec[c * KB + tid] = w;
    }
}

template <typename TA, int KB>
__global__ __launch_bounds__(256) void k_support_mw_step(SupportArgs a)
{
    __shared__ int32_t L[KB];
    __shared__ double Pt[KB], Bv[KB], Yv[KB], Bb[KB], Bd[KB], Bn[KB];
    __shared__ double red[4][KB + 2];
    __shared__ double rsum[256];
    __shared__ double sc[8];
    __shared__ int s_last;
    const TA *XT = reinterpret_cast<const TA *>(a.XT);
    const int ng = a.groups, m = blockIdx.x / ng, gg = blockIdx.x % ng;
    double *st = a.st + 8 * (int64_t)m;
    if (st[5] != 0.0) return;  // finished (the same for the whole workgroup)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int it = a.step[m];
    const bool cert = (it % a.cert_every) == 0 || it >= a.max_iter;
    const int64_t o0 = a.off[m];
    const int kl = (int)(a.off[m + 1] - o0);
    constexpr int RT = MwRows<TA, KB>::RT;
    typedef typename RawVec<RT * (int)sizeof(TA)>::t RV;
    int r0, r1;
    support_rows<RT>(a, ng, gg, r0, r1);
    double *vec = a.vec + (int64_t)m * 4 * KB;
    if (tid < KB) {
        L[tid] = (tid < kl) ? a.lab[o0 + tid] : 0;
        Pt[tid] = vec[(cert ? 0 : 1) * KB + tid];
    }
    __syncthreads();
    // this workgroup's rows: gradient at Y, or (cert) the certificate terms
    // at beta.  Lane t takes rows i0 .. i0 + RT - 1 (i0 a multiple of RT, so
    // the loads are aligned; rows up to npad exist and are zero past n, and
    // rows at or past r1 are masked).  Every column slot is read (slots past
    // the support hold column 0 with weight 0), so the KB loads are issued
    // together.
    {
        double g[KB];
#pragma unroll
        for (int r = 0; r < KB; ++r) g[r] = 0.0;
        double al = 0.0, ac = 0.0;
        for (int i0 = r0 + tid * RT; i0 < r1; i0 += 256 * RT) {
            RV xr[KB];
#pragma unroll
            for (int r = 0; r < KB; ++r) xr[r] = *reinterpret_cast<const RV *>(XT + (int64_t)L[r] * a.npad + i0);
            bool ok[RT];
            double yv[RT], sv[RT];
#pragma unroll
            for (int u = 0; u < RT; ++u) {
                ok[u] = i0 + u < r1;
                yv[u] = ok[u] ? a.y[i0 + u] : 0.0;
                sv[u] = 0.0;
            }
#pragma unroll
            for (int r = 0; r < KB; ++r)
#pragma unroll
                for (int u = 0; u < RT; ++u) sv[u] += raw_elem<TA>(xr[r], u) * Pt[r];
            double dv[RT];
#pragma unroll
            for (int u = 0; u < RT; ++u) {
                if (cert) {
                    double z, lv, cv;
                    cert_terms(a.loss, sv[u], yv[u], z, lv, cv);
                    al += ok[u] ? lv : 0.0;
                    ac += ok[u] ? cv : 0.0;
                    dv[u] = ok[u] ? z : 0.0;
                } else {
                    dv[u] = ok[u] ? dloss_d(a.loss, sv[u], yv[u]) : 0.0;
                }
            }
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int u = 0; u < RT; ++u) acc += raw_elem<TA>(xr[r], u) * dv[u];
                g[r] += acc;  // unused past the support
            }
        }
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            if (r < kl) {
                const double v = wave_sum(g[r]);
                if (lane == 0) red[wave][r] = v;
            }
        }
        al = wave_sum(al);
        ac = wave_sum(ac);
        if (lane == 0) {
            red[wave][KB] = al;
            red[wave][KB + 1] = ac;
        }
    }
    __syncthreads();
    double *pp = a.part + ((int64_t)m * ng + gg) * (KB + 2);
    if (tid < KB + 2 && (tid < kl || tid >= KB)) pp[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    if (!support_last_arrival(a, m, ng, &s_last)) return;
    // the last workgroup: the step's sums in group order, then the update
    {
        // the groups' partials in a fixed order: thread (c, h) adds groups
        // h, h + H, ... of column c, then the H sums are added in h order
        constexpr int C = KB + 2, H = 256 / C;
        const int c = tid % C, h = tid / C;
        double t = 0.0;
        if (h < H && (c < kl || c >= KB)) {
            const double *src = a.part + (int64_t)m * ng * C + c;
#pragma unroll 4
            for (int q = h; q < ng; q += H) t += src[(int64_t)q * C];
        }
        rsum[tid] = t;
        __syncthreads();
        if (tid < C && (tid < kl || tid >= KB)) {
            double u = 0.0;
            for (int q = 0; q < H; ++q) u += rsum[q * C + tid];
            red[0][tid] = u;
        }
    }
    if (tid < KB) {
        Bv[tid] = vec[tid];
        Yv[tid] = vec[KB + tid];
        Bb[tid] = vec[2 * KB + tid];
        Bd[tid] = vec[3 * KB + tid];
    }
    if (tid < 8) sc[tid] = st[tid];
    __syncthreads();
    const double eta = sc[0];
    if (cert) {
        if (tid < 64) {
            double pen = 0.0, dterm = 0.0;
            if (tid < kl) {
                const double qv = red[0][tid] / (2.0 * a.lambda2);
                pen = Bv[tid] * Bv[tid];
                dterm = huber(qv, a.M);
            }
            pen = wave_sum(pen);
            dterm = wave_sum(dterm);
            if (tid == 0) {
                const double phi = red[0][KB] + a.lambda2 * pen;
                const double psi = -red[0][KB + 1] - 2.0 * a.lambda2 * dterm;
                sc[6] = (phi < sc[3]) ? 1.0 : 0.0;
                if (phi < sc[3]) sc[3] = phi;
                sc[7] = (psi > sc[4]) ? 1.0 : 0.0;
                if (psi > sc[4]) sc[4] = psi;
                const double den = fmax(fabs(sc[3]), 1e-12);
                sc[5] = ((sc[3] - sc[4]) <= a.tol * den || it >= a.max_iter) ? 1.0 : 0.0;
            }
        }
        __syncthreads();
        if (tid < kl && sc[6] != 0.0) Bb[tid] = Bv[tid];
        if (tid < kl && sc[7] != 0.0) Bd[tid] = Bv[tid];
    } else {
        // proximal step from Y, restart test, momentum
        const double shrink = 1.0 / (1.0 + 2.0 * eta * a.lambda2);
        if (tid < 64) {
            double dot = 0.0;
            if (tid < kl) {
                const double u = Yv[tid] - eta * red[0][tid];
                const double bn = fmin(fmax(u * shrink, -a.M), a.M);
                Bn[tid] = bn;
                dot = (Yv[tid] - bn) * (bn - Bv[tid]);
            }
            dot = wave_sum(dot);
            if (tid == 0) {
                const double tm = sc[2];
                if (dot > 0.0) {
                    sc[2] = 1.0;
                    sc[1] = 0.0;
                } else {
                    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tm * tm));
                    sc[1] = (tm - 1.0) / tn;
                    sc[2] = tn;
                }
            }
        }
        __syncthreads();
        if (tid < kl) {
            const double bp = Bv[tid];
            Bv[tid] = Bn[tid];
            Yv[tid] = Bn[tid] + sc[1] * (Bn[tid] - bp);
        }
    }
    __syncthreads();
    if (tid < KB) {
        vec[tid] = Bv[tid];
        vec[KB + tid] = Yv[tid];
        vec[2 * KB + tid] = Bb[tid];
        vec[3 * KB + tid] = Bd[tid];
    }
    if (tid < 6) st[tid] = sc[tid];
    const bool fin = sc[5] != 0.0;
    if (fin && tid < kl) {
        a.beta_out[o0 + tid] = Bb[tid];
        if (a.beta_lb_out) a.beta_lb_out[o0 + tid] = Bd[tid];
    }
    if (tid == 0) {
        a.arrive[m] = 0;
        if (fin) {
            a.value[m] = sc[3];
            a.lower[m] = fmin(sc[4], sc[3]);
            a.status[m] = (sc[3] - sc[4] <= a.tol * fmax(fabs(sc[3]), 1e-12)) ? 0 : 2;
            a.iters[m] = it;
            atomicAdd(a.ndone, 1);
        } else {
            a.step[m] = it + 1;
        }
    }
}
static int support_kb(int maxlen) { return maxlen <= 16 ? 16 : (maxlen <= 32 ? 32 : 64); }

// The automatic split: at most SUPPORT_MW_ROWS rows per workgroup (one
// vectorised sweep of the workgroup), and about one workgroup per CU over
// the batch (a step is a latency-bound chain per workgroup, so a second wave
// of workgroups costs a second chain; measured at 100000 rows: 49 groups for
// one support, 16 for 16, 2 for 128).  Below SUPPORT_MW_MIN_N rows the
// one-workgroup kernel with its internal step loop is kept.
constexpr int SUPPORT_MW_ROWS = 2048;
constexpr int SUPPORT_MW_BLOCKS = 256;
constexpr int SUPPORT_MW_MIN_N = 8192;

struct MwLayout {
    size_t part, gram, st, vec, step, arrive, ndone, total;
};

// the set-up launch forms the Gram matrix over workgroups of at most
// SUPPORT_MW_ROWS rows whatever the step's split
static int mw_init_groups(int n, int groups)
{
    return std::max(groups, (n + SUPPORT_MW_ROWS - 1) / SUPPORT_MW_ROWS);
}

static MwLayout mw_layout(int count, int groups, int init_groups, int KB)
{
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t blocks = (size_t)count * groups, c = (size_t)count;
    MwLayout l;
    size_t o = 0;
    l.part = o;   o += al(blocks * (KB + 2) * 8);
    l.gram = o;   o += al((size_t)count * init_groups * (size_t)KB * (KB + 1) / 2 * 8);
    l.st = o;     o += al(c * 8 * 8);
    l.vec = o;    o += al(c * 4 * KB * 8);
    l.step = o;   o += al(c * 4);
    l.arrive = o; o += al(c * 4);
    l.ndone = o;  o += 256;
    l.total = o;
    return l;
}

int support_eval_plan(int xtype, int n, int count, int maxlen, int want, size_t *work_bytes)
{
    (void)xtype;
    *work_bytes = 0;
    if (count <= 0 || maxlen > SUPPORT_EVAL_MAX || want == 1) return 1;
    if (want == 0 && n < SUPPORT_MW_MIN_N) return 1;
    int g = (want > 0) ? want
                       : std::min((n + SUPPORT_MW_ROWS - 1) / SUPPORT_MW_ROWS,
                                  std::max(1, SUPPORT_MW_BLOCKS / count));
    g = std::min(g, std::max(n, 1));  // no more workgroups than rows
    g = std::max(1, (int)std::min<int64_t>(g, INT32_MAX / count));
    if ((int64_t)count * mw_init_groups(n, g) > INT32_MAX) return 1;
    // the step-launch kernels, with g workgroups per support (also for g = 1)
    *work_bytes = mw_layout(count, g, mw_init_groups(n, g), support_kb(maxlen)).total;
    return g;
}

static SupportArgs support_args(const SupportLaunch &L)
{
    SupportArgs a{};
    a.groups = L.groups;
    a.XT = L.XT; a.npad = L.npad; a.n = L.n; a.loss = L.loss; a.y = L.y; a.lab = L.lab; a.off = L.off;
    a.warm = L.warm; a.lambda2 = L.lambda2; a.M = L.M; a.c_loss = (L.loss == 0) ? 2.0 : 0.25; a.tol = L.tol;
    a.max_iter = L.max_iter; a.cert_every = L.cert_every;
    a.beta_out = L.beta_out; a.beta_lb_out = L.beta_lb_out; a.value = L.value; a.lower = L.lower;
    a.status = L.status; a.iters = L.iters;
    if (L.work) {
        a.init_groups = mw_init_groups(L.n, L.groups);
        const MwLayout l = mw_layout(L.count, L.groups, a.init_groups, support_kb(L.maxlen));
        char *w = (char *)L.work;
        a.part = (double *)(w + l.part);
        a.gram = (double *)(w + l.gram);
        a.st = (double *)(w + l.st);
        a.vec = (double *)(w + l.vec);
        a.step = (int32_t *)(w + l.step);
        a.arrive = (int32_t *)(w + l.arrive);
        a.ndone = (int32_t *)(w + l.ndone);
    }
    return a;
}

const int32_t *support_done_counter(const SupportLaunch &L)
{
    const MwLayout l = mw_layout(L.count, L.groups, mw_init_groups(L.n, L.groups), support_kb(L.maxlen));
    return (const int32_t *)((const char *)L.work + l.ndone);
}

#define KBNB_SUP_DISPATCH(KERNEL, GRID)                                          \
    do {                                                                         \
        const int kb_ = support_kb(L.maxlen);                                    \
        if (L.xtype == XT_F64) {                                                 \
            if (kb_ == 16) KBNB_LAUNCH((KERNEL<double, 16>), GRID, dim3(256), 0, s, a);   \
            else if (kb_ == 32) KBNB_LAUNCH((KERNEL<double, 32>), GRID, dim3(256), 0, s, a); \
            else KBNB_LAUNCH((KERNEL<double, 64>), GRID, dim3(256), 0, s, a);             \
        } else if (L.xtype == XT_F32) {                                          \
            if (kb_ == 16) KBNB_LAUNCH((KERNEL<float, 16>), GRID, dim3(256), 0, s, a);    \
            else if (kb_ == 32) KBNB_LAUNCH((KERNEL<float, 32>), GRID, dim3(256), 0, s, a); \
            else KBNB_LAUNCH((KERNEL<float, 64>), GRID, dim3(256), 0, s, a);              \
        } else {                                                                 \
            if (kb_ == 16) KBNB_LAUNCH((KERNEL<uint16_t, 16>), GRID, dim3(256), 0, s, a); \
            else if (kb_ == 32) KBNB_LAUNCH((KERNEL<uint16_t, 32>), GRID, dim3(256), 0, s, a); \
            else KBNB_LAUNCH((KERNEL<uint16_t, 64>), GRID, dim3(256), 0, s, a);           \
        }                                                                        \
    } while (0)

int launch_support_steps(hipStream_t s, const SupportLaunch &L, int steps)
{
    if (L.count <= 0 || !L.work) return 0;
    const SupportArgs a = support_args(L);
    const dim3 grid((unsigned)((size_t)L.count * L.groups));
    for (int i = 0; i < steps; ++i) KBNB_SUP_DISPATCH(k_support_mw_step, grid);
    return 0;
}

int launch_support_start(hipStream_t s, const SupportLaunch &L, int steps)
{
    if (L.count <= 0) return 0;
    if (L.maxlen > SUPPORT_EVAL_MAX) return -1;
    const SupportArgs a = support_args(L);
    if (!L.work_bytes) {
        KBNB_SUP_DISPATCH(k_support_eval, dim3(L.count));
        return 0;
    }
    const MwLayout l = mw_layout(L.count, L.groups, a.init_groups, support_kb(L.maxlen));
    if (!L.work || L.work_bytes < l.total) return -1;
    // arrival counts start at zero (each launch's last workgroup clears its own)
    if (hipMemsetAsync(a.arrive, 0, (size_t)L.count * 4, s) != hipSuccess) return -2;
    KBNB_SUP_DISPATCH(k_support_mw_init, dim3((unsigned)((size_t)L.count * a.init_groups)));
    return launch_support_steps(s, L, steps);
}
#undef KBNB_SUP_DISPATCH
void launch_transpose(hipStream_t s, int xtype, const void *X, void *XT, int n, int p, int ldp,
                      int npad, int pm)
{
    (void)pm;
    dim3 grid((p + 31) / 32, (n + 31) / 32);
    if (xtype == XT_F64)
        KBNB_LAUNCH((k_transpose<double>), grid, dim3(256), 0, s, (const double *)X, (double *)XT, n, p, ldp, npad);
    else if (xtype == XT_F32)
        KBNB_LAUNCH((k_transpose<float>), grid, dim3(256), 0, s, (const float *)X, (float *)XT, n, p, ldp, npad);
    else
        KBNB_LAUNCH((k_transpose<uint16_t>), grid, dim3(256), 0, s, (const uint16_t *)X, (uint16_t *)XT, n, p, ldp, npad);
}

}  // namespace kbnb
