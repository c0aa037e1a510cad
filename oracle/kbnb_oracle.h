/*
 * kbnb_oracle.h -- plain, sequential float64 CPU reference for the node
 * relaxations and the branch-and-bound of cardinality-constrained GLMs.
 *
 * TEST INFRASTRUCTURE ONLY: this is the oracle that the GPU library is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline load it.  It shares no code, header, table or constant with the
 * GPU library, and the GPU library never calls it.
 *
 * Problem (paper, Sec. 1, eqs. intro_sparse_glm / intro_sparse_glm_mip):
 *   min_beta  f(X beta, y) + lambda2 ||beta||^2
 *   s.t.      ||beta||_0 <= k,  ||beta||_inf <= M
 * with f(s, y) = sum_i l(s_i, y_i) (Sec. 4.2), squared l = (y - s)^2 or
 * logistic l = log(1 + exp(-y s)), y in {-1, +1}.
 *
 * A node fixes some indicators: state[j] = 1 (z_j = 1, set J1),
 * state[j] = -1 (z_j = 0, set J0), state[j] = 0 (free, set Jf).
 */
#ifndef KBNB_ORACLE_H
#define KBNB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SQUARED = 0, ORC_LOGISTIC = 1 };
enum { ORC_FREE = 0, ORC_IN = 1, ORC_OUT = -1 };
enum { ORC_CONVERGED = 0, ORC_PRUNED = 1, ORC_MAXITER = 2, ORC_INVALID = -1 };

typedef struct {
    int n, p, k, loss;
    double lambda2, M;
    const double *X; /* row-major n x p, float64 */
    const double *y; /* n */
} orc_problem;

/* Scalar loss, its derivative in s, and its convex conjugate l*(v, y). */
double orc_loss(int loss, double s, double y);
double orc_dloss(int loss, double s, double y);
double orc_loss_conj(int loss, double v, double y);

/* Huber function with threshold M and the prox of c * H_M. */
double orc_huber(double q, double M);
double orc_prox_huber(double x, double c, double M);

/* Node functions. */
int orc_kbar(const orc_problem *P, const signed char *state);
double orc_g(const orc_problem *P, const signed char *state, const double *beta);
double orc_gstar(const orc_problem *P, const signed char *state, const double *q);
void orc_prox(const orc_problem *P, const signed char *state, double eta,
              const double *u, double *beta_out);
double orc_primal(const orc_problem *P, const signed char *state, const double *beta);
double orc_dual(const orc_problem *P, const signed char *state, const double *zeta);
void orc_dual_point(const orc_problem *P, const double *beta, double *zeta_out);

/* Smoothness constant of F(X beta): c_l * lambda_max(X^T X) (power iteration). */
double orc_lipschitz(const orc_problem *P);

/* FISTA node bound.  info[0..4] = LB, Phi_best, rel_gap, iterations, status. */
int orc_node_bound(const orc_problem *P, const signed char *state, double L,
                   const double *warm, double tol, int max_iter, double ub,
                   double prune_rel, double *beta_out, double *info);

/* Rounding support (J1 plus the kbar largest free |beta|) and branching index. */
void orc_round_branch(const orc_problem *P, const signed char *state,
                      const double *beta, int *support, int *support_len,
                      int *branch);

/* v(S): best objective on a support, with |beta| <= M (node with J1 = S, Jf empty). */
double orc_support_value(const orc_problem *P, const int *support, int len, double L,
                         double tol, int max_iter, double *beta_out);

/* Best-bound branch and bound.
 * info[0..5] = objective, lower_bound, rel_gap, nodes, status (0 optimal,
 *              1 node limit), incumbent updates. */
int orc_bnb(const orc_problem *P, double node_tol, int node_max_iter,
            double gap_tol, double prune_rel, long max_nodes,
            int *support_out, double *beta_out, double *info);

/* Support-level Rashomon set (Sec. 4.5): every support S with |S| <= k and
 * v(S) <= (1 + eps) Phi*, or the best `cap` of them when cap > 0.
 * out_supports: max_out x k entries (ascending, -1 padded); out_values:
 * max_out.  Entries are ordered by value, ties by the support sequence.
 * info[0..3] = Phi*, final threshold, nodes bounded, status (0 complete,
 * 1 node limit).  Returns the number of entries in the set (only the first
 * max_out are written). */
long orc_rashomon(const orc_problem *P, double eps, long cap, double node_tol,
                  int node_max_iter, long max_nodes, long max_out,
                  int *out_supports, double *out_values, double *info);

/* Fixed-model reliance (appendix on variable importance over the Rashomon
 * set) of one model beta (p entries): for every feature j,
 *   R[j] = (1/n) sum_i l(eta_i - x_ij beta_j, y_i) - (1/n) sum_i l(eta_i, y_i),
 * eta = X beta; R[j] = 0 where beta_j = 0. */
void orc_reliance(const orc_problem *P, const double *beta, double *R);

#ifdef __cplusplus
}
#endif
#endif
