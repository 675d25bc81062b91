/*
 * gm_oracle.h -- serial FP64 CPU oracle for adaptive Genz-Malik cubature.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * (the HIP library behind include/gm.h) never calls it and shares no code,
 * header, table or constant with it.
 *
 * What it computes (Tonarelli et al., "Adaptive Multidimensional Quadrature
 * on Multi-GPU Systems", arXiv 2511.01573):
 *   - the fully symmetric Genz-Malik rule and an embedded lower-degree rule
 *     on a hyper-rectangle (Sec. 2), with a local error estimate (Sec. 2,
 *     "heuristic estimator") and a fourth-difference split axis (Sec. 2);
 *   - the breadth-first adaptive loop of Sec. 3 (initial uniform partition,
 *     evaluate every region, global convergence test of Sec. 4, heuristic
 *     classifier, split along the chosen axis);
 *   - the test integrands of Sec. 4 and their seeded Genz-family
 *     generalisations;
 *   - the derivative of the fixed-tree quadrature with respect to the
 *     integrand parameters, and a lock-step batch of independent integrals;
 *   - the tensor-product Gauss-Kronrod rule the framework offers besides
 *     the Genz-Malik rule (Sec. 3), for d <= 6;
 *   - a degree-9 fully symmetric rule (the "9-order" reading of Sec. 2)
 *     with the degree-7 rule embedded, and a null-rule error heuristic.
 *
 * All floating point is IEEE binary64, built with -ffp-contract=off; every
 * fused multiply-add is written out as fma().
 */
#ifndef GM_ORACLE_H
#define GM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GMO_OSCILLATORY = 1,
  GMO_PRODUCT_PEAK = 2,
  GMO_CORNER_PEAK = 3,
  GMO_GAUSSIAN = 4,
  GMO_C0 = 5,
  GMO_DISCONTINUOUS = 6,
  GMO_POLY = 7,
  /* Oracle-only test family: prod_j (x_j - u_j)^k_j with k_j = (int)a_j.
     Used to pin the rule on monomials; not part of the product's API. */
  GMO_MONOMIAL = 99
};

enum {
  GMO_OK = 0,
  GMO_MAX_REGIONS = 1,
  GMO_MAX_ITERS = 2,
  GMO_PRECISION_LIMIT = 3,
  GMO_NONFINITE = 4,
  GMO_EINVAL = -1,
  GMO_ENOMEM = -2,
  GMO_RUNNING = 100
};

/* Stats layout (int64[8]). */
enum {
  GMO_ST_ITERS = 0,       /* evaluate steps executed                   */
  GMO_ST_REGIONS = 1,     /* sum of active-set sizes over iterations    */
  GMO_ST_EVALS = 2,       /* REGIONS * N(d)                             */
  GMO_ST_ACTIVE = 3,      /* size of the last evaluated active set      */
  GMO_ST_FINISHED = 4,    /* regions retired by the classifier          */
  GMO_ST_MAX_ACTIVE = 5,  /* largest active set                         */
  GMO_ST_GEOMETRY = 6,    /* regions retired by the geometry guard      */
  GMO_ST_ROUNDOFF = 7     /* regions retired by the round-off guard     */
};

int64_t gmo_num_nodes(int d);
/* lam[5] = {0, l2, l3, l4, l5}; w[5], v[5] and e[5] = w - v, classes 1..5. */
void gmo_constants(int d, double lam[5], double w[5], double v[5], double e[5]);
/* All N(d) nodes of the region (c, h) in visit order: x[N*d], cls[N] in 1..5. */
void gmo_nodes(int d, const double* c, const double* h, double* x, int* cls);
/* Tensor-product Gauss-Kronrod rule: the 15 Kronrod abscissae on [-1, 1]
   (ascending; the 7 Gauss abscissae are those at odd indices), the Kronrod
   weights and the Gauss weights (0 off the Gauss abscissae), mean measure. */
void gmo_gk_constants(double x[15], double wk[15], double wg[15]);
int64_t gmo_gk_num_nodes(int d);
/* One region with the Gauss-Kronrod rule; out layout as gmo_rule with
   S[0] = K-sum, S[1] = G-sum and D[i] = the one-axis estimates e_i. */
int gmo_rule_gk(int fam, int d, const double* params, const double* c, const double* h, int lvl,
                double vol_omega, double* out);
/* Degree-9 fully symmetric rule with the degree-7 and degree-5 rules
   embedded (classes 1..8, see gm_oracle.c).  lam[6] = {0, l2, l3, l4, l5, l6};
   w[8] the degree-9 weights, e[8] = w minus the degree-7 weights. */
int64_t gmo_num_nodes9(int d);
void gmo_constants9(int d, double lam[6], double w[8], double e[8]);
/* All N9(d) nodes in visit order: x[N*d], cls[N] in 1..8. */
void gmo_nodes9(int d, const double* c, const double* h, double* x, int* cls);
/* One region with the degree-9 rule.  out layout (double):
 *   [0] Q9  [1] err (model 0: vol |Q9 - Q7|; 1: null-rule ratio test)
 *   [2] axis  [3] geometry flag  [4] scaleQ  [5] scaleE
 *   [6] Q7  [7] n1 = vol |Q9 - Q7|  [8] n2 = vol |Q7 - Q5|  [9] n3 = vol |Q5 - Q3|
 *   [10..18) S_1..S_8  [18..26) Sabs_1..Sabs_8  [26..26+d) D_0..D_{d-1} */
int gmo_rule9(int fam, int d, const double* params, const double* c, const double* h, int lvl,
              double vol_omega, int err_model, double* out);
/* Integrand value at x; params = a[0..d), u[0..d). */
double gmo_f(int fam, int d, const double* params, const double* x);
/* Gradient of f at x with respect to params (out[2d]); returns f. */
double gmo_df(int fam, int d, const double* params, const double* x, double* out);

/*
 * One region.  out layout (double):
 *   [0] Q   [1] err   [2] axis   [3] geometry flag (0/1)
 *   [4] scaleQ = vol * sum_k |w_k| Sabs_k
 *   [5] scaleE = vol * sum_k |e_k| Sabs_k
 *   [6..11) S_1..S_5     [11..16) Sabs_1..Sabs_5
 *   [16..16+d) D_0..D_{d-1}
 * Returns 0, or GMO_NONFINITE if some f value or class sum is not finite.
 */
int gmo_rule(int fam, int d, const double* params, const double* c, const double* h,
             int lvl, double vol_omega, double* out);

/* Adaptive run (handle API). */
typedef struct gmo_run gmo_run;
gmo_run* gmo_create(int fam, int d, const double* params, const double* lo, const double* hi,
                    double rel_tol, double abs_tol, int64_t max_regions, int init_log2,
                    int max_iters, int keep_leaves, int* status);
/* One full iteration; returns GMO_RUNNING or the final status. */
/* Select the rule of a run before its first step: 0 Genz-Malik degree 7
   (default), 1 tensor-product Gauss-Kronrod (2 <= d <= 6), 2 degree-9 fully
   symmetric rule.  GMO_EINVAL otherwise. */
int gmo_set_rule(gmo_run* r, int rule);
/* Error model of the degree-9 rule (before the first step): 0 |Q9 - Q7|,
   1 null-rule ratio test. */
int gmo_set_err_model(gmo_run* r, int model);
/* Memory-pressure pruning (before the first step): when the kept regions would
   overflow the capacity, relax the classifier's budget by the smallest power
   of two that makes them fit and continue.  gmo_pruned: whether it happened. */
int gmo_set_prune(gmo_run* r, int on);
int gmo_pruned(const gmo_run* r);
int gmo_step(gmo_run* r);
int gmo_run_to_end(gmo_run* r);
void gmo_result(const gmo_run* r, double* I, double* E, int* status, int64_t* stats);
int64_t gmo_active_count(const gmo_run* r);
/* Test diagnostic: sum over the frozen tree of vol * sum_k |w_k - v_k| Sabs_k
   (the magnitude that the error estimates cancel), for parity bounds on E. */
double gmo_escale(const gmo_run* r);
/* Last evaluated active set (c, h: n*d row-major; lvl; Q; err; axis). */
void gmo_get_active(const gmo_run* r, double* c, double* h, int32_t* lvl, double* Q,
                    double* err, int32_t* axis);
int64_t gmo_leaf_count(const gmo_run* r);
/* Frozen tree: retired leaves followed by the last evaluated active set. */
void gmo_get_leaves(const gmo_run* r, double* c, double* h, int32_t* lvl);
/* Per-iteration trace, int64 [iters][2] = (n_active, n_finished) and
   double [iters][2] = (I, E). */
int64_t gmo_trace_len(const gmo_run* r);
void gmo_get_trace(const gmo_run* r, int64_t* counts, double* IE);
void gmo_free(gmo_run* r);

/* Fixed-tree quadrature and its parameter gradient over a leaf list. */
int gmo_quad_leaves(int fam, int d, const double* params, int64_t n, const double* c,
                    const double* h, const int32_t* lvl, double vol_omega, double* out_q);
int gmo_grad_leaves(int fam, int d, const double* params, int64_t n, const double* c,
                    const double* h, const int32_t* lvl, double vol_omega, double* out_grad);
/* The same with the rule chosen: 0 degree 7, 2 degree 9 (GMO_EINVAL otherwise). */
int gmo_quad_leaves_rule(int fam, int d, const double* params, int64_t n, const double* c,
                         const double* h, const int32_t* lvl, double vol_omega, int rule,
                         double* out_q);
int gmo_grad_leaves_rule(int fam, int d, const double* params, int64_t n, const double* c,
                         const double* h, const int32_t* lvl, double vol_omega, int rule,
                         double* out_grad);

/* Lock-step batch of independent integrals sharing one region capacity. */
int gmo_integrate_batch(int n, const int* fam, const double* params, const int* d,
                        const double* lo, const double* hi, const double* rel_tol,
                        const double* abs_tol, int64_t max_regions_total, int init_log2,
                        int max_iters, double* out_est, double* out_err, int* out_status,
                        int64_t* out_iters);
/* The same with the rule and error model of every item selected (rule as in
   gmo_set_rule, err_model as in gmo_set_err_model; an item that rejects them
   reports GMO_EINVAL). */
int gmo_integrate_batch_rule(int n, const int* fam, const double* params, const int* d,
                             const double* lo, const double* hi, const double* rel_tol,
                             const double* abs_tol, int64_t max_regions_total, int init_log2,
                             int max_iters, int rule, int err_model, double* out_est,
                             double* out_err, int* out_status, int64_t* out_iters);

/* Threads of the per-region evaluation loop: 1 unless built with OpenMP. */
int gmo_threads(void);

#ifdef __cplusplus
}
#endif
#endif
