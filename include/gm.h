/*
 * gm.h -- C ABI of libgm, adaptive Genz-Malik cubature on AMD Instinct MI355X
 * (gfx950), FP64.
 *
 * Method: Tonarelli, Riva, Benedusi, Ferrandi, Krause, "Adaptive
 * Multidimensional Quadrature on Multi-GPU Systems", arXiv 2511.01573.
 *   Sec. 2  - the fully symmetric Genz-Malik rule, its embedded lower-degree
 *             rule and the |Q7 - Q5| local error estimate; the split axis
 *             from per-axis fourth differences.
 *   Sec. 3  - breadth-first adaptivity: every region is evaluated each
 *             iteration, the global estimate is checked, regions with a
 *             negligible error share are retired by a classifier and the rest
 *             are halved along their axis; region data stays on the device
 *             in structure-of-arrays form; filtering and splitting are fused.
 *   Sec. 4  - the stopping rule  E <= max(abs_tol, rel_tol * |I|)  (the
 *             paper uses abs_tol = 1e-16) and the test integrands.
 *
 * Conventions shared by every entry point
 *   - All array arguments are HOST pointers unless stated otherwise.  The
 *     caller owns them; the library keeps no pointer after a call returns
 *     (except a workspace registered with gm_set_workspace).
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     of a call is enqueued on it and the call returns after its results are
 *     final (host-synchronous).
 *   - params layout for every integrand: double[2d] = a[0..d), u[0..d).
 *   - Return value: a status code below.  On a negative code the outputs are
 *     left untouched.
 *   - Calls on one process are serialised by an internal mutex; they are not
 *     reentrant from device callbacks.
 */
#ifndef GM_H
#define GM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Integrands on a box, parameters a, u (Sec. 4 and their Genz families):
 *   1 oscillatory   cos(2 pi u_0 + sum a_j x_j)               (paper f1: a_j = j, u = 0)
 *   2 product peak  prod 1 / (a_j^-2 + (x_j - u_j)^2)          (f2: a = 50, u = 1/2)
 *   3 corner peak   (1 + sum a_j x_j)^-(d+1)                   (f3: a_j = j)
 *   4 Gaussian      exp(-sum a_j^2 (x_j - u_j)^2)              (f4: a = 25, u = 1/2)
 *   5 C0            exp(-sum a_j |x_j - u_j|)                  (f5: a = 10, u = 1/2)
 *   6 discontinuous 0 if x_j > u_j for any j, else exp(sum a_j x_j)
 *                                                  (f6: a_j = j + 4, u_j = (3 + j)/10)
 *   7 polynomial    (sum x_j^2)^11                             (f7; params ignored) */
enum {
  GM_OSCILLATORY = 1,
  GM_PRODUCT_PEAK = 2,
  GM_CORNER_PEAK = 3,
  GM_GAUSSIAN = 4,
  GM_C0 = 5,
  GM_DISCONTINUOUS = 6,
  GM_POLY_F7 = 7
};

/* Status codes. */
enum {
  GM_OK = 0,              /* E <= max(abs_tol, rel_tol |I|)                               */
  GM_MAX_REGIONS = 1,     /* splitting would exceed the region capacity; best (I, E) out  */
  GM_MAX_ITERS = 2,       /* iteration budget (option max_iters) used up; (I, E) out      */
  GM_PRECISION_LIMIT = 3, /* every region retired by a guard while E > T; (I, E) out      */
  GM_NONFINITE = 4,       /* f (or a rule sum) was NaN/Inf somewhere; outputs are NaN     */
  GM_EINVAL = -1,         /* invalid argument; nothing ran                                */
  GM_ENOMEM = -2,         /* device memory (or the registered workspace) too small        */
  GM_EHIP = -3            /* HIP runtime error; see gm_status_string(GM_EHIP)              */
};

/*
 * gm_integrate -- integrate f over the box [lo, hi] (Sec. 3 loop).
 *   integrand_id  one of GM_OSCILLATORY .. GM_POLY_F7
 *   params        double[2d] (a, u), finite
 *   d             2 <= d <= 16
 *   lo, hi        double[d], finite, lo[j] < hi[j]
 *   rel_tol       >= 0, abs_tol >= 0, finite, not both 0
 *   max_regions   capacity of the active region set; must hold the initial
 *                 partition (2^(d*floor(L0/d)) regions, L0 = option
 *                 init_log2_regions, default 12)
 *   out_est, out_err  host double*: I and E
 * Returns GM_OK .. GM_NONFINITE, or a negative error.
 */
int gm_integrate(int integrand_id, const double* params, int d, const double* lo, const double* hi,
                 double rel_tol, double abs_tol, int64_t max_regions, double* out_est,
                 double* out_err, void* stream);

/*
 * gm_integrate_batch -- n independent integrals in one lock-stepped,
 * device-resident region store (thousands of small integrals at once).
 *   integrand_ids int[n]; d int[n] (2..16 for the packing; items with d > 10
 *                 are rejected with GM_EINVAL in out_status)
 *   params        packed: item i contributes 2*d[i] doubles (a then u)
 *   lo, hi        packed: item i contributes d[i] doubles each
 *   rel_tol, abs_tol double[n]
 *   max_regions_total  shared capacity of all items' active regions
 *   out_est, out_err double[n], out_status int[n]
 * Item i follows exactly the loop of gm_integrate with its own tolerance; all
 * items advance one iteration together.  If the kept regions of all still
 * running items would need more than max_regions_total rows, every still
 * running item stops with GM_MAX_REGIONS and its current (I, E).  An invalid
 * item gets GM_EINVAL in out_status and NaN outputs; the call returns the
 * largest non-negative item status, or a negative code for a call-level fault.
 */
int gm_integrate_batch(int n, const int* integrand_ids, const double* params, const int* d,
                       const double* lo, const double* hi, const double* rel_tol,
                       const double* abs_tol, int64_t max_regions_total, double* out_est,
                       double* out_err, int* out_status, void* stream);

/*
 * gm_integrate_grad -- gm_integrate plus the gradient of the estimate with
 * respect to params, out_grad double[2d] in the params layout.  The gradient
 * is the exact derivative of the fixed-tree quadrature: the region tree the
 * forward run ended with (retired leaves plus the last active set) is frozen
 * and sum_leaves vol * sum_nodes w * df/dtheta is evaluated by an adjoint
 * kernel.  Discontinuity locations (u of the discontinuous family) get 0.
 */
int gm_integrate_grad(int integrand_id, const double* params, int d, const double* lo,
                      const double* hi, double rel_tol, double abs_tol, int64_t max_regions,
                      double* out_est, double* out_err, double* out_grad, void* stream);

/*
 * gm_integrate_noalloc -- gm_integrate for callers that cannot allocate
 * device or pinned memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, options, results
 * and kernels as gm_integrate, but every device buffer of the run (region
 * store, per-region outputs, tile counts, status block) is laid out in a
 * fixed device array of 64 MiB that the library holds on each GPU it runs on
 * until the process ends; the call makes no hipMalloc, hipFree, hipHostMalloc
 * or other allocating call (the status block is read through a pinned host
 * copy only if an earlier gm_integrate made one; option "timing" is ignored).
 *   max_regions   as gm_integrate, and the run's buffers must fit the array:
 *                 gm_workspace_bytes(d, max_regions, 0) <= 64 MiB (about
 *                 2.3e5 regions at d = 8, 1.2e5 at d = 16), else GM_EINVAL
 *                 before anything runs.
 * The array is shared by every call on that GPU and keeps the last call's
 * contents (each run writes its initial partition and status block before
 * reading them).  Calls from one process are serialised by the library's
 * mutex; calls that overlap on one GPU from several processes race.
 */
int gm_integrate_noalloc(int integrand_id, const double* params, int d, const double* lo,
                         const double* hi, double rel_tol, double abs_tol, int64_t max_regions,
                         double* out_est, double* out_err, void* stream);

/*
 * gm_eval_regions -- the rule kernel alone on a caller-given region list
 * (Sec. 2: rule value, error estimate and split axis of each region), with
 * the rule and error model the options "rule" and "err_model" select.
 *   c, h        host double[n*d], row-major: region r is prod_j [c - h, c + h]
 *   lvl         host int32[n]: region volume = vol(box [lo, hi]) * 2^-lvl
 *   out_q, out_err  host double[n]; out_axis host int32[n] (bit 7 set when
 *               halving along the axis would not change the region)
 */
int gm_eval_regions(int integrand_id, const double* params, int d, const double* lo,
                    const double* hi, int64_t n, const double* c, const double* h,
                    const int32_t* lvl, double* out_q, double* out_err, int32_t* out_axis,
                    void* stream);

/*
 * gm_set_workspace -- register a caller-owned DEVICE buffer (e.g. a torch
 * uint8 tensor) used for the region store and every other per-call device
 * buffer of gm_integrate, gm_integrate_grad and gm_integrate_batch instead of
 * library allocations (gm_workspace_bytes gives the size; the gradient
 * mode's store of retired leaves, whose size is only known as the run goes,
 * stays library-owned).  device_ptr must be 256-byte aligned (GM_EINVAL
 * otherwise).  bytes == 0 (or ptr == NULL) returns to library-owned memory.
 * The caller keeps the buffer alive while registered; the library never frees
 * it and writes only its first `bytes` bytes.  A call needing more than
 * `bytes` returns GM_ENOMEM before any device work, outputs untouched.
 */
int gm_set_workspace(void* device_ptr, size_t bytes);

/* Bytes of device workspace one call needs: mode 0 integrate, 1 grad (without
   the leaf store, which grows on demand), 2 batch (d = max item dimension,
   max_regions = max_regions_total, up to 65536 items). */
size_t gm_workspace_bytes(int d, int64_t max_regions, int mode);

/*
 * gm_set_option -- process-wide knobs.  Returns GM_OK or GM_EINVAL.
 *   "init_log2_regions"  L0, initial partition 2^(d*floor(L0/d)) cells (default 12, 0..30)
 *   "max_iters"          iteration budget (default 10000, >= 1)
 *   "graph_iters"        iterations enqueued per host read of the device status
 *                        block.  gm_integrate: 0 (default) = automatic, 6 while
 *                        the active set is below 2^16 regions, 3 below 2^20, 2
 *                        above; k >= 1 = k iterations (at most 8); kernels are
 *                        launched directly (no graph) and those queued past the
 *                        end return at once.  gm_integrate_grad reads the status
 *                        after every iteration whatever the value.
 *                        gm_integrate_batch: k >= 1 = one iteration's kernels
 *                        are captured k times into a hipGraph (kernel nodes
 *                        only) that is replayed until every item has stopped;
 *                        0 = direct launches and a host read every iteration
 *   "lanes_per_region"   0 = automatic, else 1..64 power of two (rule kernel mapping)
 *   "timing"             1 = record the rule kernel's device time with hipEvents on
 *                        the call's stream, 2 = every phase (default 0 = off)
 *   "rule"               0 = the Genz-Malik rule (Sec. 2, default); 1 = the
 *                        tensor-product Gauss-Kronrod rule (Sec. 3: 7-point
 *                        Gauss / 15-point Kronrod per axis, 15^d nodes,
 *                        err = vol |Q_K - Q_G|), for gm_integrate and
 *                        gm_eval_regions with 2 <= d <= 6 (GM_EINVAL above),
 *                        and for gm_integrate_batch (items of d > 6 get
 *                        GM_EINVAL); gm_integrate_grad returns GM_EINVAL while
 *                        it is selected; 2 = the degree-9
 *                        fully symmetric rule (the "9-order" rule of Sec. 2,
 *                        read as degree 9 with the degree-7 and degree-5
 *                        Genz-Malik rules embedded: 1 + 6d + 6d(d-1) +
 *                        8 C(d,3) + 2^d nodes, error estimate per
 *                        "err_model"), for gm_integrate and gm_eval_regions
 *                        with 2 <= d <= 16, for gm_integrate_batch (every
 *                        item; d <= 10) and for gm_integrate_grad (forward
 *                        tree and adjoint with the degree-9 nodes and weights)
 *   "err_model"          error estimate of the degree-9 rule: 0 = vol |Q9 - Q7|
 *                        (default); 1 = the null-rule ratio test of Sec. 2's
 *                        heuristic-estimator reading: with n1 = |Q9 - Q7|,
 *                        n2 = |Q7 - Q5|, n3 = |Q5 - Q3| (Q3 the degree-3 rule
 *                        on the centre and the +-l3 e_i nodes),
 *                        err = vol n1 min(1, 2 max(n1/n2, n2/n3))
 *   "prune"              1 = memory-pressure pruning: when the kept regions would
 *                        overflow max_regions, relax the classifier's budget
 *                        (err <= T 2^-lvl) by the smallest power of two 2^k,
 *                        k = 1..64, that makes them fit and continue instead of
 *                        stopping; a run that pruned returns GM_OK if E <= T is
 *                        still reached, else GM_MAX_REGIONS with the refined
 *                        (I, E).  gm_integrate / gm_integrate_grad only
 *                        (gm_integrate_batch returns GM_EINVAL).  Default 0.
 *   "log"                1 = print one line per iteration to stderr (default 0)
 *   "check_selftest"     bounds-check builds (-DGM_CHECK) only: a kernel checks
 *                        index n = value against bound n without accessing
 *                        memory; returns GM_EHIP with the violation as
 *                        gm_status_string(GM_EHIP) (GM_EINVAL in normal builds)
 */
int gm_set_option(const char* key, int64_t value);

/* Human-readable text of a status code (the last HIP error text for GM_EHIP). */
const char* gm_status_string(int status);

/* Statistics of the last completed call. */
typedef struct {
  int64_t iterations;        /* evaluate steps executed                           */
  int64_t regions_evaluated; /* sum over iterations of the active-set size         */
  int64_t evals;             /* integrand evaluations (regions * N(d))              */
  int64_t max_active;        /* largest active set                                 */
  int64_t final_active;      /* active regions in the last evaluated set            */
  int64_t finished;          /* regions retired by the classifier                   */
  int64_t status;            /* status of the call                                 */
  int64_t lanes_per_region;  /* rule-kernel mapping used in the last iteration      */
  double rule_ms;            /* device time in the rule kernel (option timing)      */
  double reduce_ms;          /* global reduction + convergence test (timing 2)      */
  double classify_ms;        /* classify + block counts (timing 2)                  */
  double split_ms;           /* scan + split + compaction (timing 2)                */
  double total_ms;           /* wall time of the call                               */
  int64_t rule_launches;     /* number of rule-kernel launches timed                */
} gm_stats;

int gm_last_stats(gm_stats* out);

/*
 * gm_set_tile -- tile shape the batched rule kernels use for items of
 * dimension d (2..10) and family integrand_id: lanes_per_region 1 (one lane
 * per region) or 4/16/64 (lanes of one wavefront sharing a region's corner
 * sweep; needs d >= 6/8/10), grid_blocks = workgroups of 256 lanes launched
 * (grid-stride; 0 = default 2048).  lanes_per_region = 0 removes the entry.
 * Written by the project's autotuner (paper_2511_01573_amd/autotune.py).
 */
int gm_set_tile(int d, int integrand_id, int lanes_per_region, int grid_blocks);

/* Number of integrand nodes per region, 2^d + 2 d^2 + 2 d + 1. */
int64_t gm_num_nodes(int d);

/*
 * gm_last_active -- copy out the last evaluated active set of the most recent
 * gm_integrate / gm_integrate_grad call (introspection for parity checks).
 * Copies regions [offset, offset + n) clipped to the set: c, h host
 * double[n*d] row-major, lvl int32[n], q, err double[n], axis int32[n] (the
 * packed byte: bits 0-5 split axis, bit 6 non-finite, bit 7 geometry guard);
 * any pointer may be NULL.  Returns the count of the whole set (0 when no run
 * is recorded), GM_EINVAL for offset < 0, GM_EHIP if a copy fails.
 */
int64_t gm_last_active(int64_t offset, int64_t n, double* c, double* h, int32_t* lvl, double* q,
                       double* err, int32_t* axis);

#ifdef __cplusplus
}
#endif
#endif
