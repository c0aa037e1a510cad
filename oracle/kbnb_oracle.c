/*
 * kbnb_oracle.c -- plain, sequential float64 CPU reference (the oracle).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code; the GPU library never
 * does.  It is written for a reader holding the paper ("From Sequential Nodes
 * to GPU Batches: Parallel Branch and Bound for Optimal k-Sparse GLMs"):
 * every routine cites the section or equation it writes out, and no routine
 * blocks, fuses or reorders work beyond what that passage states.
 *
 * Where the paper is silent the following readings are used:
 *   - squared loss is (y - s)^2, with no 1/2 and no 1/n;
 *   - H_M(q) = q^2/2 for |q| <= M, M|q| - M^2/2 otherwise (the scaling that
 *     makes the node conjugate g*_N the conjugate of g_N);
 *   - the FISTA step is 1/L with L = c_l * lambda_max(X^T X) (c_l = 2 for the
 *     squared loss, 1/4 for the logistic loss), momentum t+ = (1+sqrt(1+4t^2))/2,
 *     restarted when (y - beta+)^T (beta+ - beta) > 0;
 *   - the relative gap is (Phi_best - LB) / max(|Phi_best|, 1e-12);
 *   - a node is pruned when LB >= UB - prune_rel * |UB|;
 *   - ties in sorting, rounding and branching go to the lowest index.
 */
#include "kbnb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Scalar losses (Sec. 4.2, separable form of f; Sec. 4.4 for l*).          */
/* ------------------------------------------------------------------------ */

double orc_loss(int loss, double s, double y)
{
    if (loss == ORC_SQUARED) {
        double r = y - s;
        return r * r;
    }
    /* log(1 + exp(z)), z = -y s, written without overflow */
    double z = -y * s;
    if (z > 0.0)
        return z + log1p(exp(-z));
    return log1p(exp(z));
}

double orc_dloss(int loss, double s, double y)
{
    if (loss == ORC_SQUARED)
        return 2.0 * (s - y);
    /* d/ds log(1 + exp(-y s)) = -y / (1 + exp(y s)) */
    return -y / (1.0 + exp(y * s));
}

double orc_loss_conj(int loss, double v, double y)
{
    if (loss == ORC_SQUARED) {
        /* sup_s v s - (y - s)^2 is attained at s = y + v/2 */
        return v * y + 0.25 * v * v;
    }
    /* logistic: with t = -v y in [0, 1], l*(v) = t log t + (1 - t) log(1 - t) */
    double t = -v * y;
    if (t < 0.0 || t > 1.0)
        return INFINITY;
    double a = (t > 0.0) ? t * log(t) : 0.0;
    double b = (t < 1.0) ? (1.0 - t) * log1p(-t) : 0.0;
    return a + b;
}

/* ------------------------------------------------------------------------ */
/* Huber function and its prox (Sec. 3, eq. prelim_node_conjugate).          */
/* ------------------------------------------------------------------------ */

double orc_huber(double q, double M)
{
    double a = fabs(q);
    if (a <= M)
        return 0.5 * q * q;
    return M * a - 0.5 * M * M;
}

/* argmin_v 1/2 (v - x)^2 + c H_M(v) */
double orc_prox_huber(double x, double c, double M)
{
    if (fabs(x) <= M * (1.0 + c))
        return x / (1.0 + c);
    return (x > 0.0) ? x - c * M : x + c * M;
}

/* ------------------------------------------------------------------------ */
/* Helpers: sorting (key descending, ties to the lowest index).              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double key;
    int idx;
} orc_kv;

static int cmp_desc(const void *a, const void *b)
{
    const orc_kv *x = (const orc_kv *)a, *y = (const orc_kv *)b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

int orc_kbar(const orc_problem *P, const signed char *st)
{
    int kb = P->k;
    for (int j = 0; j < P->p; ++j)
        if (st[j] == ORC_IN)
            --kb;
    return kb;
}

static double sgn(double x) { return (x > 0.0) ? 1.0 : ((x < 0.0) ? -1.0 : 0.0); }

/* ------------------------------------------------------------------------ */
/* g_N (Sec. 3, definition of g_N) evaluated by minimising over z.           */
/*                                                                          */
/* On J1 z = 1 gives beta_j^2 / 2.  On the free set the z-problem is solved  */
/* through its optimality conditions (Thm. 4.1 and its proof): when at most  */
/* kbar free entries are nonzero every nonzero entry takes z = 1; otherwise  */
/* z_j = min(1, |beta_j| / tau) with tau the root of the budget equation     */
/* sum_j min(1, |beta_j| / tau) = kbar (eq. tau_budget_equation), found here */
/* by bisection.  Outside the domain (beta_J0 != 0, |beta_j| > M, or         */
/* sum |beta_Jf| > M kbar) g is +infinity; a relative slack of 1e-9 absorbs  */
/* the rounding of iterates that lie on the boundary.                        */
/* ------------------------------------------------------------------------ */

double orc_g(const orc_problem *P, const signed char *st, const double *b)
{
    const int p = P->p;
    const double M = P->M, slack = 1.0 + 1e-9;
    int kbar = orc_kbar(P, st);
    double val = 0.0, sum_free = 0.0, amax = 0.0;
    int nnz = 0;
    for (int j = 0; j < p; ++j) {
        if (st[j] == ORC_OUT) {
            if (b[j] != 0.0)
                return INFINITY;
            continue;
        }
        double a = fabs(b[j]);
        if (a > M * slack)
            return INFINITY;
        if (st[j] == ORC_IN) {
            val += 0.5 * b[j] * b[j];
        } else if (a > 0.0) {
            ++nnz;
            sum_free += a;
            if (a > amax) amax = a;
        }
    }
    if (nnz <= kbar) {
        for (int j = 0; j < p; ++j)
            if (st[j] == ORC_FREE)
                val += 0.5 * b[j] * b[j];
        return val;
    }
    if (kbar <= 0 || sum_free > M * kbar * slack)
        return INFINITY;
    /* budget equation: c(tau) = sum min(1, a/tau) is nonincreasing in tau */
    double lo = 0.0, hi = amax;
    if (sum_free / kbar > hi)
        hi = sum_free / kbar;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        double c = 0.0;
        for (int j = 0; j < p; ++j)
            if (st[j] == ORC_FREE && b[j] != 0.0) {
                double a = fabs(b[j]);
                c += (a >= mid) ? 1.0 : a / mid;
            }
        if (c > kbar)
            lo = mid;
        else
            hi = mid;
    }
    double tau = hi;
    for (int j = 0; j < p; ++j)
        if (st[j] == ORC_FREE && b[j] != 0.0) {
            double a = fabs(b[j]);
            double z = (a >= tau) ? 1.0 : a / tau;
            val += 0.5 * a * a / z;
        }
    return val;
}

/* ------------------------------------------------------------------------ */
/* g*_N (eq. prelim_node_conjugate): sum over J1 of H_M(q_j) plus the sum of */
/* the kbar largest H_M(q_j) over the free set (all of them if fewer).       */
/* ------------------------------------------------------------------------ */

double orc_gstar(const orc_problem *P, const signed char *st, const double *q)
{
    const int p = P->p;
    int kbar = orc_kbar(P, st);
    double val = 0.0;
    orc_kv *h = (orc_kv *)malloc(sizeof(orc_kv) * (size_t)(p > 0 ? p : 1));
    int pf = 0;
    for (int j = 0; j < p; ++j) {
        if (st[j] == ORC_IN)
            val += orc_huber(q[j], P->M);
        else if (st[j] == ORC_FREE) {
            h[pf].key = orc_huber(q[j], P->M);
            h[pf].idx = j;
            ++pf;
        }
    }
    qsort(h, (size_t)pf, sizeof(orc_kv), cmp_desc);
    for (int r = 0; r < pf && r < kbar; ++r)
        val += h[r].key;
    free(h);
    return val;
}

/* ------------------------------------------------------------------------ */
/* prox_{eta G_N}(u) = u - rho^{-1} prox_{rho g*_N}(rho u), rho = 1/(2 eta    */
/* lambda2) (eq. pgd_step_vector_form).                                       */
/*                                                                          */
/* prox_{rho g*_N} separates: J0 coordinates carry no g* term (prox is the    */
/* identity, so beta_j = 0); J1 coordinates carry rho H_M (scalar Huber prox);*/
/* the free set carries rho TopSum_kbar(H_M(.)), computed by Alg. 1 (sort the */
/* magnitudes descending, weights rho on the first kbar positions and 0 after,*/
/* scalar Huber prox per position, then pool adjacent blocks while the left   */
/* block's value is below the right block's; a pooled block takes            */
/* prox_{mean weight * H_M}(mean magnitude)).  This is the stack form of     */
/* PAVA.  A block of zero total weight is left unshrunk, so its coefficients */
/* are exactly zero.                                                          */
/* ------------------------------------------------------------------------ */

void orc_prox(const orc_problem *P, const signed char *st, double eta,
              const double *u, double *beta)
{
    const int p = P->p;
    const double M = P->M;
    const double rho = 1.0 / (2.0 * eta * P->lambda2);
    int kbar = orc_kbar(P, st);

    orc_kv *w = (orc_kv *)malloc(sizeof(orc_kv) * (size_t)(p > 0 ? p : 1));
    int pf = 0;
    for (int j = 0; j < p; ++j) {
        if (st[j] == ORC_OUT) {
            beta[j] = 0.0;
        } else if (st[j] == ORC_IN) {
            double a = fabs(u[j]);
            double v = orc_prox_huber(rho * a, rho, M);
            beta[j] = sgn(u[j]) * (a - v / rho);
        } else {
            w[pf].key = rho * fabs(u[j]);
            w[pf].idx = j;
            ++pf;
        }
    }
    qsort(w, (size_t)pf, sizeof(orc_kv), cmp_desc);

    /* stack of blocks */
    int *bstart = (int *)malloc(sizeof(int) * (size_t)(pf + 1));
    int *bcnt = (int *)malloc(sizeof(int) * (size_t)(pf + 1));
    double *bsumw = (double *)malloc(sizeof(double) * (size_t)(pf + 1));
    double *bsumr = (double *)malloc(sizeof(double) * (size_t)(pf + 1));
    double *bval = (double *)malloc(sizeof(double) * (size_t)(pf + 1));
    int nb = 0;
    for (int r = 0; r < pf; ++r) {
        double wr = (r < kbar) ? rho : 0.0;
        bstart[nb] = r;
        bcnt[nb] = 1;
        bsumw[nb] = w[r].key;
        bsumr[nb] = wr;
        bval[nb] = orc_prox_huber(w[r].key, wr, M);
        ++nb;
        while (nb >= 2 && bval[nb - 2] < bval[nb - 1]) {
            int a = nb - 2, c = nb - 1;
            bcnt[a] += bcnt[c];
            bsumw[a] += bsumw[c];
            bsumr[a] += bsumr[c];
            bval[a] = orc_prox_huber(bsumw[a] / bcnt[a], bsumr[a] / bcnt[a], M);
            --nb;
        }
    }
    for (int bi = 0; bi < nb; ++bi) {
        for (int r = bstart[bi]; r < bstart[bi] + bcnt[bi]; ++r) {
            int j = w[r].idx;
            if (bsumr[bi] == 0.0) {
                beta[j] = 0.0;
            } else {
                double a = fabs(u[j]);
                beta[j] = sgn(u[j]) * (a - bval[bi] / rho);
            }
        }
    }
    free(bstart); free(bcnt); free(bsumw); free(bsumr); free(bval);
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Primal and dual objectives (eqs. node_composite, prelim_fenchel_dual,     */
/* dual_candidate_vector_form, batched_primal/dual_value_component).         */
/* ------------------------------------------------------------------------ */

static void matvec(const orc_problem *P, const double *b, double *s)
{
    for (int i = 0; i < P->n; ++i) {
        const double *xi = P->X + (size_t)i * P->p;
        double acc = 0.0;
        for (int j = 0; j < P->p; ++j)
            acc += xi[j] * b[j];
        s[i] = acc;
    }
}

static void matvec_t(const orc_problem *P, const double *r, double *g)
{
    for (int j = 0; j < P->p; ++j)
        g[j] = 0.0;
    for (int i = 0; i < P->n; ++i) {
        const double *xi = P->X + (size_t)i * P->p;
        for (int j = 0; j < P->p; ++j)
            g[j] += xi[j] * r[i];
    }
}

double orc_primal(const orc_problem *P, const signed char *st, const double *beta)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)P->n);
    matvec(P, beta, s);
    double f = 0.0;
    for (int i = 0; i < P->n; ++i)
        f += orc_loss(P->loss, s[i], P->y[i]);
    free(s);
    return f + 2.0 * P->lambda2 * orc_g(P, st, beta);
}

void orc_dual_point(const orc_problem *P, const double *beta, double *zeta)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)P->n);
    matvec(P, beta, s);
    for (int i = 0; i < P->n; ++i)
        zeta[i] = -orc_dloss(P->loss, s[i], P->y[i]);
    free(s);
}

double orc_dual(const orc_problem *P, const signed char *st, const double *zeta)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)P->p);
    matvec_t(P, zeta, q);
    for (int j = 0; j < P->p; ++j)
        q[j] /= 2.0 * P->lambda2;
    double fc = 0.0;
    for (int i = 0; i < P->n; ++i)
        fc += orc_loss_conj(P->loss, -zeta[i], P->y[i]);
    double val = -fc - 2.0 * P->lambda2 * orc_gstar(P, st, q);
    free(q);
    return val;
}

/* ------------------------------------------------------------------------ */
/* Step size: L = c_l lambda_max(X^T X) by power iteration, times 1.01.      */
/* ------------------------------------------------------------------------ */

double orc_lipschitz(const orc_problem *P)
{
    const int p = P->p;
    double *v = (double *)malloc(sizeof(double) * (size_t)p);
    double *w = (double *)malloc(sizeof(double) * (size_t)p);
    double *s = (double *)malloc(sizeof(double) * (size_t)P->n);
    double nrm = 0.0;
    for (int j = 0; j < p; ++j) {
        v[j] = 1.0 + 0.5 * sin((double)j + 1.0);
        nrm += v[j] * v[j];
    }
    nrm = sqrt(nrm);
    for (int j = 0; j < p; ++j) v[j] /= nrm;
    double lam = 0.0;
    for (int it = 0; it < 20000; ++it) {
        matvec(P, v, s);
        matvec_t(P, s, w);
        double rq = 0.0, ww = 0.0;
        for (int j = 0; j < p; ++j) {
            rq += v[j] * w[j];
            ww += w[j] * w[j];
        }
        ww = sqrt(ww);
        if (ww == 0.0) break;
        for (int j = 0; j < p; ++j) v[j] = w[j] / ww;
        if (it > 10 && fabs(rq - lam) <= 1e-13 * rq) {
            lam = rq;
            break;
        }
        lam = rq;
    }
    free(v); free(w); free(s);
    double c = (P->loss == ORC_SQUARED) ? 2.0 : 0.25;
    return 1.01 * c * lam;
}

/* ------------------------------------------------------------------------ */
/* Node lower bound by accelerated proximal gradient (Sec. 3, eq.            */
/* pgd_step_vector_form with the acceleration and restart its footnote       */
/* allows) and the safe dual bound (eq. dual_candidate_vector_form, weak     */
/* duality): after every step zeta^t = -grad F(X beta^t) and                 */
/* LB = max_t Psi_N(zeta^t).                                                 */
/* ------------------------------------------------------------------------ */

int orc_node_bound(const orc_problem *P, const signed char *st, double L,
                   const double *warm, double tol, int max_iter, double ub,
                   double prune_rel, double *beta_out, double *info)
{
    const int n = P->n, p = P->p;
    int kbar = orc_kbar(P, st);
    if (kbar < 0) {
        if (info) { info[0] = NAN; info[1] = NAN; info[2] = NAN; info[3] = 0; info[4] = ORC_INVALID; }
        return ORC_INVALID;
    }
    const double eta = 1.0 / L;
    double *beta = (double *)calloc((size_t)p, sizeof(double));
    double *ymom = (double *)malloc(sizeof(double) * (size_t)p);
    double *bnew = (double *)malloc(sizeof(double) * (size_t)p);
    double *u = (double *)malloc(sizeof(double) * (size_t)p);
    double *grad = (double *)malloc(sizeof(double) * (size_t)p);
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    if (warm)
        for (int j = 0; j < p; ++j)
            beta[j] = (st[j] == ORC_OUT) ? 0.0 : warm[j];
    memcpy(ymom, beta, sizeof(double) * (size_t)p);
    double t = 1.0;
    double LB = -INFINITY, PHI = INFINITY, gap = INFINITY;
    int status = ORC_MAXITER, it = 0;
    for (it = 1; it <= max_iter; ++it) {
        /* gradient of F at the extrapolated point: X^T l'(X y) */
        matvec(P, ymom, s);
        for (int i = 0; i < n; ++i)
            r[i] = orc_dloss(P->loss, s[i], P->y[i]);
        matvec_t(P, r, grad);
        for (int j = 0; j < p; ++j)
            u[j] = ymom[j] - eta * grad[j];
        orc_prox(P, st, eta, u, bnew);
        /* restart test, then momentum */
        double dot = 0.0;
        for (int j = 0; j < p; ++j)
            dot += (ymom[j] - bnew[j]) * (bnew[j] - beta[j]);
        double tn, theta;
        if (dot > 0.0) {
            tn = 1.0;
            theta = 0.0;
        } else {
            tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            theta = (t - 1.0) / tn;
        }
        for (int j = 0; j < p; ++j) {
            ymom[j] = bnew[j] + theta * (bnew[j] - beta[j]);
            beta[j] = bnew[j];
        }
        t = tn;
        /* primal value and safe dual bound at beta^t */
        double phi = orc_primal(P, st, beta);
        orc_dual_point(P, beta, r);
        double psi = orc_dual(P, st, r);
        if (psi > LB) LB = psi;
        if (phi < PHI) PHI = phi;
        double den = fabs(PHI) > 1e-12 ? fabs(PHI) : 1e-12;
        gap = (PHI - LB) / den;
        if (LB >= ub - prune_rel * fabs(ub)) {
            status = ORC_PRUNED;
            break;
        }
        if (gap <= tol) {
            status = ORC_CONVERGED;
            break;
        }
    }
    if (it > max_iter) it = max_iter;
    if (beta_out) memcpy(beta_out, beta, sizeof(double) * (size_t)p);
    if (info) {
        info[0] = LB; info[1] = PHI; info[2] = gap; info[3] = it; info[4] = status;
    }
    free(beta); free(ymom); free(bnew); free(u); free(grad); free(s); free(r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Rounding and branching from beta (Sec. 4.3, after Thm. 4.1): the support  */
/* J1 plus the kbar largest free |beta_j|, and j* = argmax over free |beta_j|.*/
/* ------------------------------------------------------------------------ */

void orc_round_branch(const orc_problem *P, const signed char *st,
                      const double *beta, int *support, int *support_len,
                      int *branch)
{
    const int p = P->p;
    int kbar = orc_kbar(P, st);
    orc_kv *a = (orc_kv *)malloc(sizeof(orc_kv) * (size_t)(p > 0 ? p : 1));
    int pf = 0, len = 0;
    for (int j = 0; j < p; ++j) {
        if (st[j] == ORC_FREE) {
            a[pf].key = fabs(beta[j]);
            a[pf].idx = j;
            ++pf;
        }
    }
    qsort(a, (size_t)pf, sizeof(orc_kv), cmp_desc);
    char *in = (char *)calloc((size_t)(p > 0 ? p : 1), 1);
    for (int j = 0; j < p; ++j)
        if (st[j] == ORC_IN) in[j] = 1;
    for (int r = 0; r < pf && r < kbar; ++r)
        in[a[r].idx] = 1;
    for (int j = 0; j < p; ++j)
        if (in[j]) support[len++] = j;
    *support_len = len;
    *branch = (pf > 0) ? a[0].idx : -1;
    free(in);
    free(a);
}

/* ------------------------------------------------------------------------ */
/* v(S) (Sec. 4.5): the restricted problem with |beta| <= M on S is the node */
/* J1 = S, J0 = complement, Jf empty, whose relaxation is exact.  Its best    */
/* primal value (an attained objective) is returned.                          */
/* ------------------------------------------------------------------------ */

double orc_support_value(const orc_problem *P, const int *support, int len, double L,
                         double tol, int max_iter, double *beta_out)
{
    signed char *st = (signed char *)malloc((size_t)P->p);
    for (int j = 0; j < P->p; ++j) st[j] = ORC_OUT;
    for (int r = 0; r < len; ++r) st[support[r]] = ORC_IN;
    orc_problem Q = *P;
    if (Q.k < len) Q.k = len;
    double info[5];
    orc_node_bound(&Q, st, L, NULL, tol, max_iter, INFINITY, 0.0, beta_out, info);
    free(st);
    return info[1];
}

/* ------------------------------------------------------------------------ */
/* Best-bound branch and bound (Sec. 4.1, Fig. 1; Sec. 4.3).                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    signed char *st;
    double *warm;
    double lb;
    int depth;
    long seq;
} orc_node;

typedef struct {
    orc_node *a;
    long n, cap;
} orc_heap;

/* smaller lower bound first; then deeper; then first in */
static int node_before(const orc_node *x, const orc_node *y)
{
    if (x->lb != y->lb) return x->lb < y->lb;
    if (x->depth != y->depth) return x->depth > y->depth;
    return x->seq < y->seq;
}

static void heap_push(orc_heap *h, orc_node nd)
{
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 64;
        h->a = (orc_node *)realloc(h->a, sizeof(orc_node) * (size_t)h->cap);
    }
    long i = h->n++;
    h->a[i] = nd;
    while (i > 0) {
        long par = (i - 1) / 2;
        if (!node_before(&h->a[i], &h->a[par])) break;
        orc_node tmp = h->a[i]; h->a[i] = h->a[par]; h->a[par] = tmp;
        i = par;
    }
}

static orc_node heap_pop(orc_heap *h)
{
    orc_node top = h->a[0];
    h->a[0] = h->a[--h->n];
    long i = 0;
    for (;;) {
        long l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && node_before(&h->a[l], &h->a[m])) m = l;
        if (r < h->n && node_before(&h->a[r], &h->a[m])) m = r;
        if (m == i) break;
        orc_node tmp = h->a[i]; h->a[i] = h->a[m]; h->a[m] = tmp;
        i = m;
    }
    return top;
}

int orc_bnb(const orc_problem *P, double node_tol, int node_max_iter,
            double gap_tol, double prune_rel, long max_nodes,
            int *support_out, double *beta_out, double *info)
{
    const int p = P->p;
    const double L = orc_lipschitz(P);
    orc_heap H = {0};
    long seq = 0, processed = 0, updates = 0;
    double UB = INFINITY;
    double *beta = (double *)malloc(sizeof(double) * (size_t)p);
    double *bre = (double *)malloc(sizeof(double) * (size_t)p);
    int *supp = (int *)malloc(sizeof(int) * (size_t)(p + 1));
    int best_len = 0;
    for (int j = 0; j < P->k && j < p; ++j) support_out[j] = -1;
    if (beta_out) memset(beta_out, 0, sizeof(double) * (size_t)p);

    orc_node root;
    root.st = (signed char *)calloc((size_t)p, 1);
    root.warm = (double *)calloc((size_t)p, sizeof(double));
    root.lb = -INFINITY;
    root.depth = 0;
    root.seq = seq++;
    heap_push(&H, root);

    int status = 0;
    double LBg = -INFINITY;
    while (H.n > 0) {
        /* global lower bound: the smallest bound among open nodes */
        LBg = H.a[0].lb;
        if (UB < INFINITY && LBg >= UB - gap_tol * fabs(UB))
            break;
        if (processed >= max_nodes) {
            status = 1;
            break;
        }
        orc_node nd = heap_pop(&H);
        if (nd.lb >= UB - prune_rel * fabs(UB)) {
            free(nd.st); free(nd.warm);
            continue;
        }
        double ninfo[5];
        orc_node_bound(P, nd.st, L, nd.warm, node_tol, node_max_iter, UB, prune_rel, beta, ninfo);
        ++processed;
        double lb = ninfo[0] > nd.lb ? ninfo[0] : nd.lb;
        if (lb >= UB - prune_rel * fabs(UB)) {
            free(nd.st); free(nd.warm);
            continue;
        }
        /* rounding and re-optimisation: a feasible support and its value */
        int len = 0, jstar = -1;
        orc_round_branch(P, nd.st, beta, supp, &len, &jstar);
        double v = orc_support_value(P, supp, len, L, 1e-13, 20000, bre);
        if (v < UB) {
            UB = v;
            best_len = len;
            for (int r = 0; r < len; ++r) support_out[r] = supp[r];
            for (int r = len; r < P->k; ++r) support_out[r] = -1;
            if (beta_out) memcpy(beta_out, bre, sizeof(double) * (size_t)p);
            ++updates;
        }
        /* a node whose free budget is not binding is integral: its relaxation
           equals the value of J1 plus all free coordinates, already rounded */
        int kbar = orc_kbar(P, nd.st), pf = 0;
        for (int j = 0; j < p; ++j)
            if (nd.st[j] == ORC_FREE) ++pf;
        if (kbar == 0 || pf <= kbar || jstar < 0) {
            free(nd.st); free(nd.warm);
            continue;
        }
        /* branch on j*: child with z_j* = 0 and child with z_j* = 1 */
        orc_node c0, c1;
        c0.st = (signed char *)malloc((size_t)p);
        c1.st = (signed char *)malloc((size_t)p);
        memcpy(c0.st, nd.st, (size_t)p);
        memcpy(c1.st, nd.st, (size_t)p);
        c0.st[jstar] = ORC_OUT;
        c1.st[jstar] = ORC_IN;
        c0.warm = (double *)malloc(sizeof(double) * (size_t)p);
        c1.warm = (double *)malloc(sizeof(double) * (size_t)p);
        memcpy(c0.warm, beta, sizeof(double) * (size_t)p);
        memcpy(c1.warm, beta, sizeof(double) * (size_t)p);
        c0.warm[jstar] = 0.0;
        c0.lb = c1.lb = lb;
        c0.depth = c1.depth = nd.depth + 1;
        c0.seq = seq++;
        c1.seq = seq++;
        heap_push(&H, c0);
        heap_push(&H, c1);
        free(nd.st); free(nd.warm);
    }
    if (H.n == 0)
        LBg = UB;
    else if (LBg > UB)
        LBg = UB;
    while (H.n > 0) {
        orc_node nd = heap_pop(&H);
        free(nd.st); free(nd.warm);
    }
    free(H.a);
    free(beta); free(bre); free(supp);
    (void)best_len;
    if (info) {
        double den = fabs(UB) > 1e-12 ? fabs(UB) : 1e-12;
        info[0] = UB;
        info[1] = LBg;
        info[2] = (UB - LBg) / den;
        info[3] = (double)processed;
        info[4] = status;
        info[5] = (double)updates;
    }
    return status;
}


/* ------------------------------------------------------------------------ */
/* Rashomon-set collection (Sec. 4.5, "Rashomon-set collection").            */
/*                                                                           */
/* The same best-bound tree with two changes:                                */
/*  - a node is pruned only when its bound exceeds the threshold             */
/*    tau = min((1 + eps) UB, v_(cap)), v_(cap) the cap-th best value found  */
/*    (+inf before cap supports are known, or when cap = 0);                 */
/*  - a node is a leaf only when no indicator is left to decide: kbar = 0    */
/*    (the free coordinates are forced to zero) or no free coordinate.  Its  */
/*    support is J1, and v(J1) is computed directly.                         */
/* Every leaf and every re-optimised rounding support with value <= tau is   */
/* recorded.  Each support with |S| <= k is the J1 of exactly one leaf, and   */
/* a pruned node contains only supports with v(S) >= its bound > tau >=       */
/* (1 + eps) Phi*, so at the end the recorded supports with value at most    */
/* the final threshold are the set.                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int *supp;     /* n x k, ascending, -1 padded */
    double *val;
    long n, cap;
} orc_pool;

static int pool_find(const orc_pool *pl, const int *s, int k)
{
    for (long i = 0; i < pl->n; ++i)
        if (memcmp(pl->supp + i * k, s, sizeof(int) * (size_t)k) == 0) return 1;
    return 0;
}

static void pool_add(orc_pool *pl, const int *s, int len, int k, double v)
{
    int key[256];
    for (int r = 0; r < k; ++r) key[r] = r < len ? s[r] : -1;
    if (pool_find(pl, key, k)) return;
    if (pl->n == pl->cap) {
        pl->cap = pl->cap ? 2 * pl->cap : 64;
        pl->supp = (int *)realloc(pl->supp, sizeof(int) * (size_t)(pl->cap * k));
        pl->val = (double *)realloc(pl->val, sizeof(double) * (size_t)pl->cap);
    }
    memcpy(pl->supp + pl->n * k, key, sizeof(int) * (size_t)k);
    pl->val[pl->n] = v;
    ++pl->n;
}

/* the c-th smallest recorded value (1-based), +inf when fewer are recorded */
static double pool_kth(const orc_pool *pl, long c)
{
    if (c <= 0 || pl->n < c) return INFINITY;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)pl->n);
    memcpy(tmp, pl->val, sizeof(double) * (size_t)pl->n);
    /* selection by repeated minimum: plain and small */
    double v = INFINITY;
    for (long r = 0; r < c; ++r) {
        long bi = -1;
        for (long i = 0; i < pl->n; ++i)
            if (bi < 0 || tmp[i] < tmp[bi]) bi = i;
        v = tmp[bi];
        tmp[bi] = INFINITY;
    }
    free(tmp);
    return v;
}

static int g_pool_k;
static const orc_pool *g_pool_sort;
static int pool_cmp(const void *a, const void *b)
{
    const long i = *(const long *)a, j = *(const long *)b;
    const double vi = g_pool_sort->val[i], vj = g_pool_sort->val[j];
    if (vi < vj) return -1;
    if (vi > vj) return 1;
    return memcmp(g_pool_sort->supp + i * g_pool_k, g_pool_sort->supp + j * g_pool_k,
                  sizeof(int) * (size_t)g_pool_k);
}

long orc_rashomon(const orc_problem *P, double eps, long cap, double node_tol,
                  int node_max_iter, long max_nodes, long max_out,
                  int *out_supports, double *out_values, double *info)
{
    const int p = P->p, k = P->k;
    const double L = orc_lipschitz(P);
    orc_heap H = {0};
    orc_pool pl = {0};
    long seq = 0, processed = 0;
    double UB = INFINITY;
    double *beta = (double *)malloc(sizeof(double) * (size_t)p);
    double *bre = (double *)malloc(sizeof(double) * (size_t)p);
    int *supp = (int *)malloc(sizeof(int) * (size_t)(p + 1));
    int status = 0;

    orc_node root;
    root.st = (signed char *)calloc((size_t)p, 1);
    root.warm = (double *)calloc((size_t)p, sizeof(double));
    root.lb = -INFINITY;
    root.depth = 0;
    root.seq = seq++;
    heap_push(&H, root);

#define TAU() (fmin((1.0 + eps) * UB, pool_kth(&pl, cap)))
    while (H.n > 0) {
        if (processed >= max_nodes) {
            status = 1;
            break;
        }
        orc_node nd = heap_pop(&H);
        if (nd.lb > TAU()) {
            free(nd.st); free(nd.warm);
            continue;
        }
        const int kbar = orc_kbar(P, nd.st);
        int pf = 0, len = 0;
        for (int j = 0; j < p; ++j)
            if (nd.st[j] == ORC_FREE) ++pf;
        if (kbar == 0 || pf == 0) {
            /* leaf: the support is J1 */
            for (int j = 0; j < p; ++j)
                if (nd.st[j] == ORC_IN) supp[len++] = j;
            const double v = orc_support_value(P, supp, len, L, 1e-13, 50000, bre);
            ++processed;
            if (v < UB) UB = v;
            if (v <= TAU()) pool_add(&pl, supp, len, k, v);
            free(nd.st); free(nd.warm);
            continue;
        }
        double ninfo[5];
        orc_node_bound(P, nd.st, L, nd.warm, node_tol, node_max_iter, INFINITY, 0.0, beta, ninfo);
        ++processed;
        const double lb = ninfo[0] > nd.lb ? ninfo[0] : nd.lb;
        /* rounding and re-optimisation: a feasible support and its value */
        int jstar = -1;
        orc_round_branch(P, nd.st, beta, supp, &len, &jstar);
        const double v = orc_support_value(P, supp, len, L, 1e-13, 50000, bre);
        if (v < UB) UB = v;
        if (v <= TAU()) pool_add(&pl, supp, len, k, v);
        if (lb > TAU()) {
            free(nd.st); free(nd.warm);
            continue;
        }
        if (jstar < 0)  /* no free coordinate is nonzero: branch on the first free one */
            for (int j = 0; j < p && jstar < 0; ++j)
                if (nd.st[j] == ORC_FREE) jstar = j;
        orc_node c0, c1;
        c0.st = (signed char *)malloc((size_t)p);
        c1.st = (signed char *)malloc((size_t)p);
        memcpy(c0.st, nd.st, (size_t)p);
        memcpy(c1.st, nd.st, (size_t)p);
        c0.st[jstar] = ORC_OUT;
        c1.st[jstar] = ORC_IN;
        c0.warm = (double *)malloc(sizeof(double) * (size_t)p);
        c1.warm = (double *)malloc(sizeof(double) * (size_t)p);
        memcpy(c0.warm, beta, sizeof(double) * (size_t)p);
        memcpy(c1.warm, beta, sizeof(double) * (size_t)p);
        c0.warm[jstar] = 0.0;
        c0.lb = c1.lb = lb;
        c0.depth = c1.depth = nd.depth + 1;
        c0.seq = seq++;
        c1.seq = seq++;
        heap_push(&H, c0);
        heap_push(&H, c1);
        free(nd.st); free(nd.warm);
    }
    const double tau = TAU();
#undef TAU
    while (H.n > 0) {
        orc_node nd = heap_pop(&H);
        free(nd.st); free(nd.warm);
    }
    free(H.a);
    /* the set: recorded supports within the final threshold, by value */
    long *ord = (long *)malloc(sizeof(long) * (size_t)(pl.n + 1));
    long cnt = 0;
    for (long i = 0; i < pl.n; ++i)
        if (pl.val[i] <= tau) ord[cnt++] = i;
    g_pool_k = k;
    g_pool_sort = &pl;
    qsort(ord, (size_t)cnt, sizeof(long), pool_cmp);
    if (cap > 0 && cnt > cap) cnt = cap;
    for (long r = 0; r < cnt && r < max_out; ++r) {
        memcpy(out_supports + r * k, pl.supp + ord[r] * k, sizeof(int) * (size_t)k);
        out_values[r] = pl.val[ord[r]];
    }
    if (info) {
        info[0] = UB;
        info[1] = tau;
        info[2] = (double)processed;
        info[3] = status;
    }
    free(ord);
    free(pl.supp); free(pl.val);
    free(beta); free(bre); free(supp);
    return cnt;
}

/* Fixed-model reliance: drop feature j's fitted contribution from the linear
 * predictor, keep every other coefficient, and compare the mean losses. */
void orc_reliance(const orc_problem *P, const double *beta, double *R)
{
    double *eta = (double *)malloc(sizeof(double) * (size_t)P->n);
    matvec(P, beta, eta);
    double base = 0.0;
    for (int i = 0; i < P->n; ++i) base += orc_loss(P->loss, eta[i], P->y[i]);
    for (int j = 0; j < P->p; ++j) {
        if (beta[j] == 0.0) {
            R[j] = 0.0;
            continue;
        }
        double dropped = 0.0;
        for (int i = 0; i < P->n; ++i)
            dropped += orc_loss(P->loss, eta[i] - P->X[(size_t)i * P->p + j] * beta[j], P->y[i]);
        R[j] = (dropped - base) / (double)P->n;
    }
    free(eta);
}
