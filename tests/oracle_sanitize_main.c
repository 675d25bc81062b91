/*
 * Host sanitizer run of the CPU oracle (tests/test_oracle_sanitize.py builds
 * this file with the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer and runs it).  It walks every entry point of oracle/gm_oracle.h
 * on small inputs: the three rules region by region, adaptive runs with each
 * rule (and pruning), the lock-step batch, and the fixed-tree quadrature and
 * gradient.  Exit status 0 and no sanitizer report is the pass condition; the
 * numbers themselves are checked by the Python tests.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/gm_oracle.h"

static unsigned long long rng_state = 88172645463325252ull;
static double urand(void) {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int fail(const char* what) {
  fprintf(stderr, "oracle sanitize run: %s\n", what);
  return 1;
}

int main(void) {
  double out[64], p[32], c[16], h[16], lo[16], hi[16];
  int d, fam, k, rule;
  for (d = 2; d <= 8; ++d) {
    for (fam = 1; fam <= 7; ++fam) {
      for (k = 0; k < d; ++k) {
        p[k] = 0.5 + 3.0 * urand();
        p[d + k] = urand();
        c[k] = 0.2 + 0.6 * urand();
        h[k] = 0.01 + 0.1 * urand();
      }
      if (gmo_rule(fam, d, p, c, h, 3, 1.0, out) < 0) return fail("rule");
      if (gmo_rule9(fam, d, p, c, h, 3, 1.0, k & 1, out) < 0) return fail("rule9");
      if (d <= 4 && gmo_rule_gk(fam, d, p, c, h, 3, 1.0, out) < 0) return fail("rule_gk");
    }
    {
      int64_t n = gmo_num_nodes9(d);
      double* x = (double*)malloc(sizeof(double) * (size_t)(n * d));
      int* cls = (int*)malloc(sizeof(int) * (size_t)n);
      gmo_nodes9(d, c, h, x, cls);
      free(x);
      free(cls);
    }
  }
  for (rule = 0; rule <= 2; ++rule) {
    for (d = 2; d <= 4; ++d) {
      int st, prune;
      for (k = 0; k < d; ++k) {
        p[k] = 2.0 + urand();
        p[d + k] = urand();
        lo[k] = 0.0;
        hi[k] = 1.0;
      }
      for (prune = 0; prune <= 1; ++prune) {
        double I, E;
        int64_t stats[8], n, nl, nt;
        gmo_run* r = gmo_create(4, d, p, lo, hi, 1e-7, 1e-16, prune ? 400 : 1 << 16, 2, 100,
                                1, &st);
        if (!r) return fail("create");
        if (gmo_set_rule(r, rule) != GMO_OK) return fail("set_rule");
        if (rule == 2 && gmo_set_err_model(r, 1) != GMO_OK) return fail("set_err_model");
        if (gmo_set_prune(r, prune) != GMO_OK) return fail("set_prune");
        gmo_run_to_end(r);
        gmo_result(r, &I, &E, &st, stats);
        n = gmo_active_count(r);
        nl = gmo_leaf_count(r);
        nt = gmo_trace_len(r);
        {
          double* ac = (double*)malloc(sizeof(double) * (size_t)(n * d + 1));
          double* ah = (double*)malloc(sizeof(double) * (size_t)(n * d + 1));
          int32_t* al = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
          double* aq = (double*)malloc(sizeof(double) * (size_t)(n + 1));
          double* ae = (double*)malloc(sizeof(double) * (size_t)(n + 1));
          int32_t* ax = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
          double* lc = (double*)malloc(sizeof(double) * (size_t)(nl * d + 1));
          double* lh = (double*)malloc(sizeof(double) * (size_t)(nl * d + 1));
          int32_t* ll = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nl + 1));
          int64_t* tc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * nt + 1));
          double* tv = (double*)malloc(sizeof(double) * (size_t)(2 * nt + 1));
          double q, g[32];
          gmo_get_active(r, ac, ah, al, aq, ae, ax);
          gmo_get_leaves(r, lc, lh, ll);
          gmo_get_trace(r, tc, tv);
          if (rule != 1) {
            if (gmo_quad_leaves_rule(4, d, p, nl, lc, lh, ll, 1.0, rule, &q) < 0)
              return fail("quad_leaves");
            if (gmo_grad_leaves_rule(4, d, p, nl, lc, lh, ll, 1.0, rule, g) < 0)
              return fail("grad_leaves");
          }
          free(ac);
          free(ah);
          free(al);
          free(aq);
          free(ae);
          free(ax);
          free(lc);
          free(lh);
          free(ll);
          free(tc);
          free(tv);
        }
        (void)gmo_escale(r);
        (void)gmo_pruned(r);
        gmo_free(r);
      }
    }
  }
  {
    int fams[4] = {4, 1, 2, 3}, ds[4] = {2, 3, 3, 4}, st[4], i, j, po = 0, bo = 0;
    double params[32], blo[16], bhi[16], rt[4], at[4], est[4], err[4];
    int64_t its[4];
    for (i = 0; i < 4; ++i) {
      for (j = 0; j < ds[i]; ++j) {
        params[po + j] = 1.0 + urand();
        params[po + ds[i] + j] = urand();
        blo[bo + j] = 0.0;
        bhi[bo + j] = 1.0;
      }
      po += 2 * ds[i];
      bo += ds[i];
      rt[i] = 1e-6;
      at[i] = 1e-16;
    }
    for (rule = 0; rule <= 2; ++rule)
      if (gmo_integrate_batch_rule(4, fams, params, ds, blo, bhi, rt, at, 1 << 18, 2, 200, rule,
                                   0, est, err, st, its) < 0)
        return fail("batch");
  }
  {
    double x[15], wk[15], wg[15], lam[6], w[8], e[8], l7[5], w7[5], v7[5], e7[5];
    gmo_gk_constants(x, wk, wg);
    gmo_constants9(8, lam, w, e);
    gmo_constants(8, l7, w7, v7, e7);
  }
  printf("oracle sanitize run ok\n");
  return 0;
}
