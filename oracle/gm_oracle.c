/*
 * gm_oracle.c -- plain serial FP64 oracle for adaptive Genz-Malik cubature.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the
 * benchmark).  Shares no code with the HIP library.
 *
 * Paper: Tonarelli, Riva, Benedusi, Ferrandi, Krause, "Adaptive
 * Multidimensional Quadrature on Multi-GPU Systems", arXiv 2511.01573.
 * The paper names the rule (Sec. 2: a fully symmetric Genz-Malik rule with
 * O(2^d) nodes), the error estimator family (Sec. 2: the Genz-Berntsen style
 * heuristic built on the embedded rule), the split heuristic (Sec. 2: fourth
 * derivative along each axis), the breadth-first loop (Sec. 3) and the
 * stopping rule (Sec. 4).  It prints no constants; the ones below are the
 * unique solution of the moment equations of a degree-7 fully symmetric rule
 * with generators {0, l2 e_i, l3 e_i, l4(e_i+e_j), l5 (1,..,1)} and the
 * degree-5 rule embedded in the same nodes.  Where the paper is silent the
 * readings are stated at each function.
 *
 * Build: gcc -O3 -std=c11 -ffp-contract=off -fPIC -shared -lm (serial); the
 * all-cores CPU baseline adds -fopenmp (only the per-region evaluation loop of
 * an iteration runs in parallel; results are bitwise those of the serial build).
 */
#include "gm_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) summation.                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  double s, c;
} ksum;

static void ks_add(ksum* k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x))
    k->c += (k->s - t) + x;
  else
    k->c += (x - t) + k->s;
  k->s = t;
}
static double ks_val(const ksum* k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* Rule constants (Sec. 2, the Genz-Malik degree-7 rule and its embedded     */
/* degree-5 rule, mean measure on [-1,1]^d).  Each value is one correctly    */
/* rounded division of exact integers, or a square root of one.              */
/* ------------------------------------------------------------------------ */
int64_t gmo_num_nodes(int d) {
  return ((int64_t)1 << d) + 2 * (int64_t)d * d + 2 * (int64_t)d + 1;
}

void gmo_constants(int d, double lam[5], double w[5], double v[5], double e[5]) {
  int64_t D = d;
  lam[0] = 0.0;
  lam[1] = sqrt(9.0 / 70.0);
  lam[2] = sqrt(9.0 / 10.0);
  lam[3] = sqrt(9.0 / 10.0);
  lam[4] = sqrt(9.0 / 19.0);
  w[0] = (double)(400 * D * D - 9120 * D + 12824) / 19683.0;
  w[1] = 980.0 / 6561.0;
  w[2] = (double)(1820 - 400 * D) / 19683.0;
  w[3] = 200.0 / 19683.0;
  w[4] = ldexp(6859.0 / 19683.0, -d);
  v[0] = (double)(50 * D * D - 950 * D + 729) / 729.0;
  v[1] = 245.0 / 486.0;
  v[2] = (double)(265 - 100 * D) / 1458.0;
  v[3] = 25.0 / 729.0;
  v[4] = 0.0;
  /* e = w - v as exact rationals, then rounded once. */
  e[0] = (double)(-19 * (50 * D * D - 870 * D + 361)) / 19683.0;
  e[1] = -4655.0 / 13122.0;
  e[2] = (double)(95 * (20 * D - 37)) / 39366.0;
  e[3] = -475.0 / 19683.0;
  e[4] = w[4];
}

/* ------------------------------------------------------------------------ */
/* Integrands (Sec. 4 test functions and their seeded Genz families).        */
/* params = a[0..d), u[0..d).  Sums run left to right over j = 0..d-1.       */
/* ------------------------------------------------------------------------ */
static const double TWO_PI = 6.283185307179586476925286766559;

double gmo_f(int fam, int d, const double* p, const double* x) {
  const double* a = p;
  const double* u = p + d;
  double s = 0.0;
  int j;
  switch (fam) {
    case GMO_OSCILLATORY: /* cos(2 pi u_1 + sum a_j x_j); f1 has a_j = j, u = 0 */
      for (j = 0; j < d; ++j) s = s + a[j] * x[j];
      return cos(TWO_PI * u[0] + s);
    case GMO_PRODUCT_PEAK: { /* prod 1/(a_j^-2 + (x_j-u_j)^2); f2 has a = 50, u = 1/2 */
      double den = 1.0;
      for (j = 0; j < d; ++j) {
        double t = x[j] - u[j];
        den = den * (1.0 / (a[j] * a[j]) + t * t);
      }
      return 1.0 / den;
    }
    case GMO_CORNER_PEAK: /* (1 + sum a_j x_j)^-(d+1); f3 has a_j = j */
      for (j = 0; j < d; ++j) s = s + a[j] * x[j];
      return pow(1.0 + s, -(double)(d + 1));
    case GMO_GAUSSIAN: /* exp(-sum a_j^2 (x_j-u_j)^2); f4 has a = 25, u = 1/2 */
      for (j = 0; j < d; ++j) {
        double t = a[j] * (x[j] - u[j]);
        s = s + t * t;
      }
      return exp(-s);
    case GMO_C0: /* exp(-sum a_j |x_j-u_j|); f5 has a = 10, u = 1/2 */
      for (j = 0; j < d; ++j) s = s + a[j] * fabs(x[j] - u[j]);
      return exp(-s);
    case GMO_DISCONTINUOUS: /* 0 if x_j > u_j for any j, else exp(sum a_j x_j) */
      for (j = 0; j < d; ++j)
        if (x[j] > u[j]) return 0.0;
      for (j = 0; j < d; ++j) s = s + a[j] * x[j];
      return exp(s);
    case GMO_POLY: /* f7 = (sum x_j^2)^11 */
      for (j = 0; j < d; ++j) s = s + x[j] * x[j];
      return pow(s, 11.0);
    case GMO_MONOMIAL: { /* test family: prod (x_j - u_j)^k_j, k_j = (int)a_j */
      double m = 1.0;
      for (j = 0; j < d; ++j) {
        int k, kj = (int)a[j];
        double t = x[j] - u[j];
        for (k = 0; k < kj; ++k) m = m * t;
      }
      return m;
    }
    default:
      return NAN;
  }
}

/* Partial derivatives of f with respect to a_j (out[j]) and u_j (out[d+j]).
   The discontinuous family's jump location does not enter the fixed-tree
   quadrature (nodes do not move), so its u-derivatives are zero. */
double gmo_df(int fam, int d, const double* p, const double* x, double* out) {
  const double* a = p;
  const double* u = p + d;
  double f = gmo_f(fam, d, p, x);
  int j;
  for (j = 0; j < 2 * d; ++j) out[j] = 0.0;
  switch (fam) {
    case GMO_OSCILLATORY: {
      double s = 0.0;
      for (j = 0; j < d; ++j) s = s + a[j] * x[j];
      double sn = sin(TWO_PI * u[0] + s);
      for (j = 0; j < d; ++j) out[j] = -sn * x[j];
      out[d] = -sn * TWO_PI;
      break;
    }
    case GMO_PRODUCT_PEAK:
      for (j = 0; j < d; ++j) {
        double t = x[j] - u[j];
        double den = 1.0 / (a[j] * a[j]) + t * t;
        out[j] = 2.0 * f / (a[j] * a[j] * a[j] * den);
        out[d + j] = 2.0 * f * t / den;
      }
      break;
    case GMO_CORNER_PEAK: {
      double s = 0.0;
      for (j = 0; j < d; ++j) s = s + a[j] * x[j];
      double g = -(double)(d + 1) * f / (1.0 + s);
      for (j = 0; j < d; ++j) out[j] = g * x[j];
      break;
    }
    case GMO_GAUSSIAN:
      for (j = 0; j < d; ++j) {
        double t = x[j] - u[j];
        out[j] = -2.0 * a[j] * t * t * f;
        out[d + j] = 2.0 * a[j] * a[j] * t * f;
      }
      break;
    case GMO_C0:
      for (j = 0; j < d; ++j) {
        double t = x[j] - u[j];
        out[j] = -fabs(t) * f;
        out[d + j] = (t > 0.0 ? 1.0 : (t < 0.0 ? -1.0 : 0.0)) * a[j] * f;
      }
      break;
    case GMO_DISCONTINUOUS:
      for (j = 0; j < d; ++j) out[j] = x[j] * f;
      break;
    default:
      break;
  }
  return f;
}

/* ------------------------------------------------------------------------ */
/* Node generation (Sec. 2: fully symmetric rule).  x = c + h*g with        */
/* generators, in this visit order:                                          */
/*   class 1: the centre;                                                    */
/*   class 2: +l2 e_i, -l2 e_i for i = 0..d-1;                                */
/*   class 3: +l3 e_i, -l3 e_i;                                               */
/*   class 4: for i < j: (+,+), (+,-), (-,+), (-,-) times l4 on (i, j);       */
/*   class 5: b = 0..2^d-1, coordinate j takes -l5 when bit j of b is set.    */
/* Each perturbed coordinate is fma(sigma*lambda, h_j, c_j).                 */
/* ------------------------------------------------------------------------ */
typedef void (*node_visitor)(void* ctx, int cls, const double* x);

static void visit_nodes(int d, const double* c, const double* h, node_visitor fn, void* ctx) {
  double lam[5], w[5], v[5], e[5];
  double x[64];
  int i, j, k;
  gmo_constants(d, lam, w, v, e);
  for (k = 0; k < d; ++k) x[k] = c[k];
  fn(ctx, 1, x);
  for (k = 2; k <= 3; ++k) {
    double l = lam[k - 1];
    for (i = 0; i < d; ++i) {
      x[i] = fma(l, h[i], c[i]);
      fn(ctx, k, x);
      x[i] = fma(-l, h[i], c[i]);
      fn(ctx, k, x);
      x[i] = c[i];
    }
  }
  {
    double l = lam[3];
    for (i = 0; i < d; ++i)
      for (j = i + 1; j < d; ++j) {
        int si, sj;
        for (si = 0; si < 2; ++si)
          for (sj = 0; sj < 2; ++sj) {
            x[i] = fma(si ? -l : l, h[i], c[i]);
            x[j] = fma(sj ? -l : l, h[j], c[j]);
            fn(ctx, 4, x);
          }
        x[i] = c[i];
        x[j] = c[j];
      }
  }
  {
    double l = lam[4];
    int64_t b, nb = (int64_t)1 << d;
    for (b = 0; b < nb; ++b) {
      for (k = 0; k < d; ++k) x[k] = fma(((b >> k) & 1) ? -l : l, h[k], c[k]);
      fn(ctx, 5, x);
    }
  }
}

typedef struct {
  int d;
  int64_t n;
  double* x;
  int* cls;
} nodes_ctx;

static void nodes_cb(void* p, int cls, const double* x) {
  nodes_ctx* q = (nodes_ctx*)p;
  memcpy(q->x + q->n * q->d, x, sizeof(double) * q->d);
  q->cls[q->n] = cls;
  q->n++;
}

void gmo_nodes(int d, const double* c, const double* h, double* x, int* cls) {
  nodes_ctx q = {d, 0, x, cls};
  visit_nodes(d, c, h, nodes_cb, &q);
}

/* ------------------------------------------------------------------------ */
/* One region: rule value, error estimate, split axis (Sec. 2).             */
/*                                                                          */
/* Q   = vol * sum_k w_k S_k                       (degree-7 rule)          */
/* err = vol * |sum_k (w_k - v_k) S_k| = |Q7 - Q5| (embedded-rule estimate) */
/* D_i = |A_i - B_i/7|, A_i = f(c+l2 h_i e_i) + f(c-l2 h_i e_i) - 2 f(c),   */
/*       B_i the same with l3; 1/7 = l2^2/l3^2 cancels the second           */
/*       derivative, leaving a fourth-difference estimate.                   */
/* Split axis (reading; the paper only says "largest estimate"): every D_i  */
/* within a noise band of the largest is a candidate, band = 1e-10 times    */
/* the largest sum of the magnitudes that enter one D_i; among candidates   */
/* the widest h_i wins, then the lowest index.                              */
/* ------------------------------------------------------------------------ */
typedef struct {
  int fam, d;
  const double* p;
  ksum S[5];
  double Sabs[5];
  double f0;
  double f2[32], f3[32]; /* [2i] = +, [2i+1] = - */
  int n2, n3;
  int nonfinite;
} rule_ctx;

static void rule_cb(void* pp, int cls, const double* x) {
  rule_ctx* r = (rule_ctx*)pp;
  double f = gmo_f(r->fam, r->d, r->p, x);
  if (!isfinite(f)) r->nonfinite = 1;
  ks_add(&r->S[cls - 1], f);
  r->Sabs[cls - 1] += fabs(f);
  if (cls == 1) r->f0 = f;
  if (cls == 2) r->f2[r->n2++] = f;
  if (cls == 3) r->f3[r->n3++] = f;
}

static const double AXIS_BAND = 1e-10;

int gmo_rule(int fam, int d, const double* params, const double* c, const double* h, int lvl,
             double vol_omega, double* out) {
  double lam[5], w[5], v[5], e[5];
  rule_ctx r;
  int k, i;
  double S[5], vol, q, er, sq, se;
  gmo_constants(d, lam, w, v, e);
  memset(&r, 0, sizeof r);
  r.fam = fam;
  r.d = d;
  r.p = params;
  visit_nodes(d, c, h, rule_cb, &r);
  for (k = 0; k < 5; ++k) S[k] = ks_val(&r.S[k]);
  for (k = 0; k < 5; ++k)
    if (!isfinite(S[k])) r.nonfinite = 1;
  vol = ldexp(vol_omega, -lvl);
  q = w[0] * S[0] + w[1] * S[1];
  q = q + w[2] * S[2];
  q = q + w[3] * S[3];
  q = q + w[4] * S[4];
  er = e[0] * S[0] + e[1] * S[1];
  er = er + e[2] * S[2];
  er = er + e[3] * S[3];
  er = er + e[4] * S[4];
  sq = 0.0;
  se = 0.0;
  for (k = 0; k < 5; ++k) {
    sq += fabs(w[k]) * r.Sabs[k];
    se += fabs(e[k]) * r.Sabs[k];
  }
  out[0] = vol * q;
  out[1] = vol * fabs(er);
  out[4] = vol * sq;
  out[5] = vol * se;
  for (k = 0; k < 5; ++k) {
    out[6 + k] = S[k];
    out[11 + k] = r.Sabs[k];
  }
  {
    const double r7 = 1.0 / 7.0;
    double Dmax = -1.0, scale = 0.0, band;
    int axis = 0;
    double D[32];
    for (i = 0; i < d; ++i) {
      double A = (r.f2[2 * i] + r.f2[2 * i + 1]) - 2.0 * r.f0;
      double B = (r.f3[2 * i] + r.f3[2 * i + 1]) - 2.0 * r.f0;
      double m = (fabs(r.f2[2 * i]) + fabs(r.f2[2 * i + 1]) + 2.0 * fabs(r.f0)) +
                 r7 * (fabs(r.f3[2 * i]) + fabs(r.f3[2 * i + 1]) + 2.0 * fabs(r.f0));
      D[i] = fabs(A - B * r7);
      out[16 + i] = D[i];
      if (D[i] > Dmax) Dmax = D[i];
      if (m > scale) scale = m;
    }
    band = AXIS_BAND * scale;
    axis = -1;
    for (i = 0; i < d; ++i) {
      if (D[i] >= Dmax - band) {
        if (axis < 0 || h[i] > h[axis]) axis = i;
      }
    }
    out[2] = (double)axis;
    {
      double hp = h[axis] * 0.5;
      int geo = (c[axis] - hp == c[axis]) || (c[axis] + hp == c[axis]) || (hp == 0.0);
      out[3] = geo ? 1.0 : 0.0;
    }
  }
  return r.nonfinite ? GMO_NONFINITE : 0;
}


/* ------------------------------------------------------------------------ */
/* Degree-9 fully symmetric rule (the "9-order" Genz-Malik reading of        */
/* Sec. 2), with the degree-7 and degree-5 rules above embedded in its nodes. */
/*                                                                          */
/* Generators (mean measure on [-1,1]^d, lambda values squared):             */
/*   class 1: 0;                                                            */
/*   class 2: +-l2 e_i (9/70);  class 3: +-l3 e_i (9/10);                    */
/*   class 4: (+-l4, +-l4) on i < j (9/10);                                  */
/*   class 5: (+-l5, .., +-l5) (9/19);                                       */
/*   class 6: +-l6 e_i (759/1190);                                           */
/*   class 7: +-l2 on i, +-l3 on j, for every ordered pair i != j;           */
/*   class 8: (+-l4, +-l4, +-l4) on i < j < k.                               */
/* N9(d) = 1 + 6d + 6d(d-1) + 8 C(d,3) + 2^d nodes.                          */
/* Derivation: the even moments of degree <= 8 give 12 equations, which     */
/* separate by the number of coordinates a monomial involves.  x^2y^2z^2w^2  */
/* sees only the corners (fixes w5 for l5^2 = 9/19); x^2y^2z^2 and x^4y^2z^2 */
/* then fix the triple class (its lambda comes out as 9/10 = l4^2); the four */
/* two-coordinate moments x^2y^2, x^4y^2, x^6y^2, x^4y^4 need an asymmetric  */
/* pair (x^6y^2 and x^4y^4 agree on every symmetric one), and their solution */
/* puts it at (l2, l3); the one-coordinate moments x^2 .. x^8 with three     */
/* axis classes fix l6^2 = 759/1190 and the axis weights, and the constant   */
/* fixes w1.  The weights below are that unique solution; every monomial of */
/* degree <= 9 is integrated exactly, x^10 is not.                          */
/*                                                                          */
/* Error estimates (readings: the paper names the degree and a null-rule     */
/* heuristic but prints neither):                                           */
/*   model 0: err = vol |Q9 - Q7|, the embedded-rule difference;             */
/*   model 1: null-rule ratio test.  The differences of successive embedded */
/*     rules are null rules: n1 = |Q9 - Q7| vanishes on degree <= 7,         */
/*     n2 = |Q7 - Q5| on degree <= 5, n3 = |Q5 - Q3| on degree <= 3, with    */
/*     Q3 = (1 - 10d/27) f(c) + 5/27 sum_i (f(c + l3 h_i e_i) + f(c - ..)),  */
/*     the degree-3 rule on classes 1 and 3.  While they fall geometrically  */
/*     with the degree the ratio rho = max(n1/n2, n2/n3) (both steps must     */
/*     fall) measures the decay, and the error of Q9 is below n1 by about    */
/*     that factor: err = vol n1 min(1, 2 rho) -- the plain difference when   */
/*     rho >= 1/2, the difference scaled by twice the ratio below.            */
/* Split axis: the fourth differences of classes 2 and 3, as for degree 7.   */
/* ------------------------------------------------------------------------ */
int64_t gmo_num_nodes9(int d) {
  int64_t D = d;
  return 1 + 6 * D + 6 * D * (D - 1) + 4 * D * (D - 1) * (D - 2) / 3 + ((int64_t)1 << d);
}

void gmo_constants9(int d, double lam[6], double w[8], double e[8]) {
  int64_t D = d;
  lam[0] = 0.0;
  lam[1] = sqrt(9.0 / 70.0);
  lam[2] = sqrt(9.0 / 10.0);
  lam[3] = sqrt(9.0 / 10.0);
  lam[4] = sqrt(9.0 / 19.0);
  lam[5] = sqrt(759.0 / 1190.0);
  w[0] = (double)(-160 * (6325 * D * D * D - 345345 * D * D + 1801355 * D - 1902813)) /
         403363719.0;
  w[1] = (double)(-490 * (2020 * D - 8711)) / 17891847.0;
  w[2] = (double)(5 * (10400 * D * D - 236080 * D + 404019)) / 13817466.0;
  w[3] = (double)(-1000 * (2 * D - 9)) / 531441.0;
  w[4] = ldexp(130321.0 / 531441.0, -d);
  w[5] = 20462645.0 / 484331562.0;
  w[6] = 4900.0 / 177147.0;
  w[7] = 1000.0 / 531441.0;
  /* e = w - (degree-7 weights, 0 on classes 6..8), exact, rounded once */
  e[0] = (double)(-8 * (126500 * D * D * D - 5882250 * D * D + 12665080 * D - 5205981)) /
         403363719.0;
  e[1] = (double)(-490 * (2020 * D - 3257)) / 17891847.0;
  e[2] = (double)(5 * (10400 * D * D - 179920 * D + 148491)) / 13817466.0;
  e[3] = (double)(-400 * (5 * D - 9)) / 531441.0;
  e[4] = ldexp(-54872.0 / 531441.0, -d);
  e[5] = w[5];
  e[6] = w[6];
  e[7] = w[7];
}

/* Node order: classes 1-5 as for degree 7, then class 6 (i ascending, + then
   -), class 7 (i, then j != i ascending; signs (+,+), (+,-), (-,+), (-,-) on
   (i, j)), class 8 (i < j < k lexicographic; sign pattern s = 0..7, bit 0 on
   i, bit 1 on j, bit 2 on k, set = negative). */
static void visit_nodes9(int d, const double* c, const double* h, node_visitor fn, void* ctx) {
  double lam[6], w[8], e[8];
  double x[64];
  int i, j, k, s;
  gmo_constants9(d, lam, w, e);
  visit_nodes(d, c, h, fn, ctx);
  for (k = 0; k < d; ++k) x[k] = c[k];
  for (i = 0; i < d; ++i) {
    x[i] = fma(lam[5], h[i], c[i]);
    fn(ctx, 6, x);
    x[i] = fma(-lam[5], h[i], c[i]);
    fn(ctx, 6, x);
    x[i] = c[i];
  }
  for (i = 0; i < d; ++i)
    for (j = 0; j < d; ++j) {
      if (j == i) continue;
      for (s = 0; s < 4; ++s) {
        x[i] = fma((s & 2) ? -lam[1] : lam[1], h[i], c[i]);
        x[j] = fma((s & 1) ? -lam[2] : lam[2], h[j], c[j]);
        fn(ctx, 7, x);
      }
      x[i] = c[i];
      x[j] = c[j];
    }
  for (i = 0; i < d; ++i)
    for (j = i + 1; j < d; ++j)
      for (k = j + 1; k < d; ++k) {
        for (s = 0; s < 8; ++s) {
          x[i] = fma((s & 1) ? -lam[3] : lam[3], h[i], c[i]);
          x[j] = fma((s & 2) ? -lam[3] : lam[3], h[j], c[j]);
          x[k] = fma((s & 4) ? -lam[3] : lam[3], h[k], c[k]);
          fn(ctx, 8, x);
        }
        x[i] = c[i];
        x[j] = c[j];
        x[k] = c[k];
      }
}

void gmo_nodes9(int d, const double* c, const double* h, double* x, int* cls) {
  nodes_ctx q = {d, 0, x, cls};
  visit_nodes9(d, c, h, nodes_cb, &q);
}

typedef struct {
  int fam, d;
  const double* p;
  ksum S[8];
  double Sabs[8];
  double f0;
  double f2[32], f3[32];
  int n2, n3;
  int nonfinite;
} rule9_ctx;

static void rule9_cb(void* pp, int cls, const double* x) {
  rule9_ctx* r = (rule9_ctx*)pp;
  double f = gmo_f(r->fam, r->d, r->p, x);
  if (!isfinite(f)) r->nonfinite = 1;
  ks_add(&r->S[cls - 1], f);
  r->Sabs[cls - 1] += fabs(f);
  if (cls == 1) r->f0 = f;
  if (cls == 2) r->f2[r->n2++] = f;
  if (cls == 3) r->f3[r->n3++] = f;
}

int gmo_rule9(int fam, int d, const double* params, const double* c, const double* h, int lvl,
              double vol_omega, int err_model, double* out) {
  double lam[6], w[8], e[8], lam7[5], w7[5], v7[5], e7[5];
  rule9_ctx r;
  int k, i;
  double S[8], vol, q, q7, n1, n2, sq, se;
  gmo_constants9(d, lam, w, e);
  gmo_constants(d, lam7, w7, v7, e7);
  memset(&r, 0, sizeof r);
  r.fam = fam;
  r.d = d;
  r.p = params;
  visit_nodes9(d, c, h, rule9_cb, &r);
  for (k = 0; k < 8; ++k) S[k] = ks_val(&r.S[k]);
  for (k = 0; k < 8; ++k)
    if (!isfinite(S[k])) r.nonfinite = 1;
  vol = ldexp(vol_omega, -lvl);
  q = w[0] * S[0];
  for (k = 1; k < 8; ++k) q = q + w[k] * S[k];
  q7 = w7[0] * S[0];
  for (k = 1; k < 5; ++k) q7 = q7 + w7[k] * S[k];
  n1 = e[0] * S[0];
  for (k = 1; k < 8; ++k) n1 = n1 + e[k] * S[k];
  n1 = fabs(n1);
  n2 = e7[0] * S[0];
  for (k = 1; k < 5; ++k) n2 = n2 + e7[k] * S[k];
  n2 = fabs(n2);
  sq = 0.0;
  se = 0.0;
  for (k = 0; k < 8; ++k) {
    sq += fabs(w[k]) * r.Sabs[k];
    se += fabs(e[k]) * r.Sabs[k];
  }
  for (k = 0; k < 5; ++k) se += fabs(e7[k]) * r.Sabs[k];
  out[0] = vol * q;
  {
    /* degree-3 rule on classes 1 and 3: (1 - 10d/27) f(c) + 5/27 sum f(c +- l3 e_i) */
    double q3 = (double)(27 - 10 * d) / 27.0 * S[0] + (5.0 / 27.0) * S[2];
    double q5 = q7 - (e7[0] * S[0] + e7[1] * S[1] + e7[2] * S[2] + e7[3] * S[3] + e7[4] * S[4]);
    double n3 = fabs(q5 - q3);
    double rho = fmax(n1 / n2, n2 / n3);
    out[9] = vol * n3;
    out[1] = err_model ? vol * (n1 * fmin(1.0, 2.0 * rho)) : vol * n1;
  }
  out[4] = vol * sq;
  out[5] = vol * se;
  out[6] = vol * q7;
  out[7] = vol * n1;
  out[8] = vol * n2;
  for (k = 0; k < 8; ++k) {
    out[10 + k] = S[k];
    out[18 + k] = r.Sabs[k];
  }
  {
    const double r7 = 1.0 / 7.0;
    double Dmax = -1.0, scale = 0.0, band;
    int axis;
    double D[32];
    for (i = 0; i < d; ++i) {
      double A = (r.f2[2 * i] + r.f2[2 * i + 1]) - 2.0 * r.f0;
      double B = (r.f3[2 * i] + r.f3[2 * i + 1]) - 2.0 * r.f0;
      double m = (fabs(r.f2[2 * i]) + fabs(r.f2[2 * i + 1]) + 2.0 * fabs(r.f0)) +
                 r7 * (fabs(r.f3[2 * i]) + fabs(r.f3[2 * i + 1]) + 2.0 * fabs(r.f0));
      D[i] = fabs(A - B * r7);
      out[26 + i] = D[i];
      if (D[i] > Dmax) Dmax = D[i];
      if (m > scale) scale = m;
    }
    band = AXIS_BAND * scale;
    axis = -1;
    for (i = 0; i < d; ++i)
      if (D[i] >= Dmax - band && (axis < 0 || h[i] > h[axis])) axis = i;
    out[2] = (double)axis;
    {
      double hp = h[axis] * 0.5;
      int geo = (c[axis] - hp == c[axis]) || (c[axis] + hp == c[axis]) || (hp == 0.0);
      out[3] = geo ? 1.0 : 0.0;
    }
  }
  return r.nonfinite ? GMO_NONFINITE : 0;
}

/* ------------------------------------------------------------------------ */
/* Tensor-product Gauss-Kronrod rule (Sec. 3: the framework's second rule,  */
/* "a tensor-product Gauss-Kronrod rule [Kronrod 1965]").                    */
/*                                                                          */
/* Reading: the 1-D pair is the 7-point Gauss-Legendre rule and its 15-point */
/* Kronrod extension on [-1, 1]; the d-dimensional rule is their tensor      */
/* product (15^d nodes), the embedded estimate is the tensor Gauss rule      */
/* (7^d of the same nodes), err = vol |Q_K - Q_G|, and the split axis is the */
/* axis i whose one-axis estimate e_i = vol |Q_K - Q_{K, G on axis i}| is     */
/* largest (same tie band as the Genz-Malik rule, relative to the K-sum of   */
/* |f|).  Usable for 2 <= d <= 6 (its cost grows as 15^d).                  */
/*                                                                          */
/* Constants from their definitions, in __float128 (rounded once to double): */
/*   Gauss nodes: roots of P7 (Newton on the three-term recurrence);         */
/*   Kronrod extra nodes: roots of the Stieltjes polynomial E8, the monic    */
/*   even polynomial of degree 8 orthogonal to x^k P7 for k < 8 (coefficients */
/*   from exact moments); weights: exactness on x^0, x^2, ... (8 symmetric   */
/*   Kronrod unknowns, 4 Gauss unknowns).  Weights are for the mean measure. */
/* ------------------------------------------------------------------------ */
typedef __float128 qf;

static qf q_abs(qf x) { return x < 0 ? -x : x; }

/* P_n(x) and P_n'(x) by the recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static qf q_legendre(int n, qf x, qf* dp) {
  qf p0 = 1, p1 = x, p2;
  int k;
  if (n == 0) {
    *dp = 0;
    return 1;
  }
  for (k = 1; k < n; ++k) {
    p2 = ((qf)(2 * k + 1) * x * p1 - (qf)k * p0) / (qf)(k + 1);
    p0 = p1;
    p1 = p2;
  }
  *dp = (qf)n * (x * p1 - p0) / (x * x - 1);
  return p1;
}

/* Solve A x = b (n <= 8) by Gaussian elimination with partial pivoting. */
static void q_solve(int n, qf A[8][8], qf* b) {
  int i, j, k;
  for (k = 0; k < n; ++k) {
    int piv = k;
    for (i = k + 1; i < n; ++i)
      if (q_abs(A[i][k]) > q_abs(A[piv][k])) piv = i;
    if (piv != k) {
      qf t;
      for (j = 0; j < n; ++j) {
        t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
      t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    for (i = k + 1; i < n; ++i) {
      qf m = A[i][k] / A[k][k];
      for (j = k; j < n; ++j) A[i][j] -= m * A[k][j];
      b[i] -= m * b[k];
    }
  }
  for (i = n - 1; i >= 0; --i) {
    qf s = b[i];
    for (j = i + 1; j < n; ++j) s -= A[i][j] * b[j];
    b[i] = s / A[i][i];
  }
}

/* int_{-1}^{1} x^a dx */
static qf q_moment(int a) { return (a % 2) ? (qf)0 : (qf)2 / (qf)(a + 1); }

static int gk_ready = 0;
static double GK_X[15], GK_WK[15], GK_WG[15];

static void gk_build(void) {
  qf g[3], kx[4], P7[8], e[5];
  qf pa[9], pb[9], pc[9];
  int i, j, m, k;
  if (gk_ready) return;
  /* positive Gauss nodes, ascending */
  for (i = 0; i < 3; ++i) {
    /* i-th largest root estimate cos(pi (i + 0.75) / 7.5), refined by Newton */
    qf x = (qf)cos(3.14159265358979323846 * (2 - i + 0.75) / 7.5), dp;
    for (k = 0; k < 100; ++k) {
      qf p = q_legendre(7, x, &dp);
      qf dx = p / dp;
      x -= dx;
      if (q_abs(dx) < (qf)1e-33) break;
    }
    g[i] = x;
  }
  /* coefficients of P7 by the recurrence on coefficient arrays */
  for (j = 0; j < 9; ++j) pa[j] = pb[j] = 0;
  pa[0] = 1;       /* P0 */
  pb[1] = 1;       /* P1 */
  for (k = 1; k < 7; ++k) {
    for (j = 0; j < 9; ++j) pc[j] = -(qf)k * pa[j];
    for (j = 0; j < 8; ++j) pc[j + 1] += (qf)(2 * k + 1) * pb[j];
    for (j = 0; j < 9; ++j) {
      pc[j] /= (qf)(k + 1);
      pa[j] = pb[j];
      pb[j] = pc[j];
    }
  }
  for (j = 0; j < 8; ++j) P7[j] = pb[j];
  /* E8(y) = sum_m e_m x^(2m), e_4 = 1: int E8 P7 x^k = 0 for k = 1, 3, 5, 7 */
  {
    qf A[8][8], b[8];
    for (i = 0; i < 4; ++i) {
      int kk = 2 * i + 1;
      for (m = 0; m <= 4; ++m) {
        qf s = 0;
        for (j = 0; j < 8; ++j)
          if (P7[j] != 0) s += P7[j] * q_moment(2 * m + j + kk);
        if (m < 4) A[i][m] = s;
        else b[i] = -s;
      }
    }
    q_solve(4, A, b);
    for (m = 0; m < 4; ++m) e[m] = b[m];
    e[4] = 1;
  }
  /* roots of E8 in y = x^2 by bisection, one in each gap (0, g1^2), (g1^2, g2^2), ... , (g3^2, 1) */
  for (i = 0; i < 4; ++i) {
    qf lo = i == 0 ? (qf)0 : g[i - 1] * g[i - 1];
    qf hi = i == 3 ? (qf)1 : g[i] * g[i];
    qf flo = e[0] + lo * (e[1] + lo * (e[2] + lo * (e[3] + lo)));
    for (k = 0; k < 240; ++k) {
      qf mid = (lo + hi) / 2;
      qf fm = e[0] + mid * (e[1] + mid * (e[2] + mid * (e[3] + mid)));
      if ((fm < 0) == (flo < 0)) {
        lo = mid;
        flo = fm;
      } else {
        hi = mid;
      }
    }
    {
      /* sqrt of the root by Newton from the double estimate */
      qf y = (lo + hi) / 2, x = (qf)sqrt((double)y);
      for (k = 0; k < 8; ++k) x = (x + y / x) / 2;
      kx[i] = x;
    }
  }
  {
    /* ascending positive nodes: k1 < g1 < k2 < g2 < k3 < g3 < k4 */
    qf pos[7] = {kx[0], g[0], kx[1], g[1], kx[2], g[2], kx[3]};
    qf A[8][8], b[8], wk[8], wg[4];
    /* Kronrod weights: unknowns W0 (centre), W1..W7 (pos[0..6]) */
    for (m = 0; m < 8; ++m) {
      A[m][0] = (m == 0) ? (qf)1 : (qf)0;
      for (j = 0; j < 7; ++j) {
        qf xp = 1;
        for (k = 0; k < 2 * m; ++k) xp *= pos[j];
        A[m][j + 1] = 2 * xp;
      }
      b[m] = q_moment(2 * m);
    }
    q_solve(8, A, b);
    for (j = 0; j < 8; ++j) wk[j] = b[j];
    /* Gauss weights: unknowns V0, V1..V3 on g[0..2] */
    for (m = 0; m < 4; ++m) {
      A[m][0] = (m == 0) ? (qf)1 : (qf)0;
      for (j = 0; j < 3; ++j) {
        qf xp = 1;
        for (k = 0; k < 2 * m; ++k) xp *= g[j];
        A[m][j + 1] = 2 * xp;
      }
      b[m] = q_moment(2 * m);
    }
    q_solve(4, A, b);
    for (j = 0; j < 4; ++j) wg[j] = b[j];
    /* 15 nodes ascending; index 7 is the centre; Gauss nodes at odd indices */
    GK_X[7] = 0.0;
    GK_WK[7] = (double)(wk[0] / 2);
    GK_WG[7] = (double)(wg[0] / 2);
    for (j = 0; j < 7; ++j) {
      GK_X[8 + j] = (double)pos[j];
      GK_X[6 - j] = -(double)pos[j];
      GK_WK[8 + j] = GK_WK[6 - j] = (double)(wk[j + 1] / 2);
      GK_WG[8 + j] = GK_WG[6 - j] = (j % 2 == 1) ? (double)(wg[(j + 1) / 2] / 2) : 0.0;
    }
  }
  gk_ready = 1;
}

void gmo_gk_constants(double x[15], double wk[15], double wg[15]) {
  gk_build();
  memcpy(x, GK_X, sizeof GK_X);
  memcpy(wk, GK_WK, sizeof GK_WK);
  memcpy(wg, GK_WG, sizeof GK_WG);
}

int64_t gmo_gk_num_nodes(int d) {
  int64_t n = 1;
  int j;
  for (j = 0; j < d; ++j) n *= 15;
  return n;
}

int gmo_rule_gk(int fam, int d, const double* params, const double* c, const double* h, int lvl,
                double vol_omega, double* out) {
  ksum SK = {0, 0}, SG = {0, 0}, SM[6];
  double absK = 0, absE = 0, vol, x[6], e[6], emax = -1.0, band;
  int k[6], j, i, nonfinite = 0, axis;
  int64_t t, N;
  if (d < 2 || d > 6) return GMO_EINVAL;
  gk_build();
  memset(SM, 0, sizeof SM);
  N = gmo_gk_num_nodes(d);
  for (t = 0; t < N; ++t) {
    int64_t q = t;
    double f, WK, WG;
    /* node index tuple, axis d-1 fastest */
    for (j = d - 1; j >= 0; --j) {
      k[j] = (int)(q % 15);
      q /= 15;
    }
    for (j = 0; j < d; ++j) x[j] = fma(GK_X[k[j]], h[j], c[j]);
    f = gmo_f(fam, d, params, x);
    if (!isfinite(f)) nonfinite = 1;
    WK = GK_WK[k[0]];
    WG = GK_WG[k[0]];
    for (j = 1; j < d; ++j) {
      WK = WK * GK_WK[k[j]];
      WG = WG * GK_WG[k[j]];
    }
    ks_add(&SK, WK * f);
    ks_add(&SG, WG * f);
    for (i = 0; i < d; ++i) {
      double WM = (i == 0) ? GK_WG[k[0]] : GK_WK[k[0]];
      for (j = 1; j < d; ++j) WM = WM * ((j == i) ? GK_WG[k[j]] : GK_WK[k[j]]);
      ks_add(&SM[i], WM * f);
    }
    absK += WK * fabs(f);
    absE += fabs(WK - WG) * fabs(f);
  }
  vol = ldexp(vol_omega, -lvl);
  out[0] = vol * ks_val(&SK);
  out[1] = vol * fabs(ks_val(&SK) - ks_val(&SG));
  out[4] = vol * absK;
  out[5] = vol * absE;
  for (i = 0; i < 10; ++i) out[6 + i] = 0.0;
  out[6] = ks_val(&SK);
  out[7] = ks_val(&SG);
  for (i = 0; i < d; ++i) {
    e[i] = vol * fabs(ks_val(&SK) - ks_val(&SM[i]));
    out[16 + i] = e[i];
    if (e[i] > emax) emax = e[i];
  }
  band = AXIS_BAND * out[4];
  axis = -1;
  for (i = 0; i < d; ++i)
    if (e[i] >= emax - band && (axis < 0 || h[i] > h[axis])) axis = i;
  out[2] = (double)axis;
  {
    double hp = h[axis] * 0.5;
    int geo = (c[axis] - hp == c[axis]) || (c[axis] + hp == c[axis]) || (hp == 0.0);
    out[3] = geo ? 1.0 : 0.0;
  }
  if (!(isfinite(out[0]) && isfinite(out[1]))) nonfinite = 1;
  return nonfinite ? GMO_NONFINITE : 0;
}

/* ------------------------------------------------------------------------ */
/* Adaptive loop (Sec. 3 workflow, Sec. 4 stopping rule).                   */
/*                                                                          */
/* 1. Initial uniform partition: s = 2^floor(L0/d) cells per axis, cell     */
/*    t = sum_j k_j s^j (axis 0 fastest), h_j = ldexp(H_j, -m),             */
/*    c_j = fma(2 k_j + 1, h_j, lo_j), level m*d.                           */
/* 2. Evaluate every active region.                                         */
/* 3. I = I_fin + sum Q, E = E_fin + sum err (compensated, store order);     */
/*    T = max(abs_tol, rel_tol |I|); stop when E <= T.                       */
/* 4. Stop when the iteration budget is used up.                            */
/* 5. Classifier (reading of "discards subregions whose contribution to     */
/*    the error is negligible"): a region retires if                        */
/*      (a) err <= ldexp(T, -lvl)   (its error density is within budget),    */
/*      (b) fl(|I| + err) == |I|    (round-off guard), or                   */
/*      (c) halving along its axis changes nothing (geometry guard).         */
/* 6. Retired regions join I_fin, E_fin (and the leaf list).                 */
/* 7. No region left -> precision limit; 2*n_keep > capacity -> stop, or,   */
/*    with memory-pressure pruning on, relax the budget of step 5(a) by the  */
/*    smallest power of two 2^k (k = 1..64) that leaves at most capacity/2   */
/*    regions unretired, retire the rest and go on (a run that pruned and    */
/*    then runs out of regions ends with the capacity status).               */
/* 8. Split each kept region in half along its axis: child "-" at rank p,   */
/*    child "+" at n_keep + p (stable order).                               */
/* ------------------------------------------------------------------------ */
struct gmo_run {
  int fam, d, max_iters, keep_leaves;
  int rule; /* 0 Genz-Malik degree 7, 1 tensor-product Gauss-Kronrod, 2 degree 9 */
  int err_model; /* degree-9 rule: 0 |Q9 - Q7|, 1 null-rule ratio test */
  int prune, pruned; /* memory-pressure pruning: enabled, happened */
  double params[32];
  double rel_tol, abs_tol, vol_omega;
  int64_t max_regions;
  int status;
  int iter;
  int64_t n;   /* active count */
  int64_t cap; /* allocated rows */
  double *c, *h, *Q, *err, *escl;
  int32_t *lvl, *axis;
  unsigned char *geo, *fin;
  double I, E, T;
  ksum Ifin, Efin;
  /* test diagnostic: sum over the frozen tree of vol * sum_k |w_k - v_k| Sabs_k,
     the magnitude the error estimates cancel (sets parity tolerances on E) */
  ksum Sfin;
  double Escale;
  int64_t n_keep;
  int64_t stats[8];
  /* leaves */
  int64_t nleaf, leafcap;
  double *lc, *lh;
  int32_t* llvl;
  /* trace */
  int64_t ntr, trcap;
  int64_t* trc;
  double* trv;
};

static int grow(gmo_run* r, int64_t need) {
  int64_t nc;
  if (need <= r->cap) return 0;
  nc = r->cap ? r->cap : 1024;
  while (nc < need) nc *= 2;
  r->c = (double*)realloc(r->c, sizeof(double) * nc * r->d);
  r->h = (double*)realloc(r->h, sizeof(double) * nc * r->d);
  r->Q = (double*)realloc(r->Q, sizeof(double) * nc);
  r->err = (double*)realloc(r->err, sizeof(double) * nc);
  r->escl = (double*)realloc(r->escl, sizeof(double) * nc);
  r->lvl = (int32_t*)realloc(r->lvl, sizeof(int32_t) * nc);
  r->axis = (int32_t*)realloc(r->axis, sizeof(int32_t) * nc);
  r->geo = (unsigned char*)realloc(r->geo, nc);
  r->fin = (unsigned char*)realloc(r->fin, nc);
  if (!r->c || !r->h || !r->Q || !r->err || !r->escl || !r->lvl || !r->axis || !r->geo || !r->fin) return -1;
  r->cap = nc;
  return 0;
}

static int leaf_push(gmo_run* r, const double* c, const double* h, int32_t lvl) {
  int d = r->d;
  if (r->nleaf == r->leafcap) {
    int64_t nc = r->leafcap ? 2 * r->leafcap : 1024;
    r->lc = (double*)realloc(r->lc, sizeof(double) * nc * d);
    r->lh = (double*)realloc(r->lh, sizeof(double) * nc * d);
    r->llvl = (int32_t*)realloc(r->llvl, sizeof(int32_t) * nc);
    if (!r->lc || !r->lh || !r->llvl) return -1;
    r->leafcap = nc;
  }
  memcpy(r->lc + r->nleaf * d, c, sizeof(double) * d);
  memcpy(r->lh + r->nleaf * d, h, sizeof(double) * d);
  r->llvl[r->nleaf] = lvl;
  r->nleaf++;
  return 0;
}

static void trace_push(gmo_run* r, int64_t nact, int64_t nfin) {
  if (r->ntr == r->trcap) {
    int64_t nc = r->trcap ? 2 * r->trcap : 64;
    r->trc = (int64_t*)realloc(r->trc, sizeof(int64_t) * 2 * nc);
    r->trv = (double*)realloc(r->trv, sizeof(double) * 2 * nc);
    r->trcap = nc;
  }
  r->trc[2 * r->ntr] = nact;
  r->trc[2 * r->ntr + 1] = nfin;
  r->trv[2 * r->ntr] = r->I;
  r->trv[2 * r->ntr + 1] = r->E;
  r->ntr++;
}

gmo_run* gmo_create(int fam, int d, const double* params, const double* lo, const double* hi,
                    double rel_tol, double abs_tol, int64_t max_regions, int init_log2,
                    int max_iters, int keep_leaves, int* status) {
  gmo_run* r;
  int j, m;
  int64_t s, n0, t;
  double H[32];
  *status = GMO_EINVAL;
  if (d < 2 || d > 16 || ((fam < 1 || fam > 7) && fam != GMO_MONOMIAL) || init_log2 < 0 || init_log2 > 40 || max_iters < 1)
    return NULL;
  if (!(rel_tol >= 0.0) || !(abs_tol >= 0.0) || !isfinite(rel_tol) || !isfinite(abs_tol) ||
      (rel_tol == 0.0 && abs_tol == 0.0))
    return NULL;
  for (j = 0; j < d; ++j)
    if (!isfinite(lo[j]) || !isfinite(hi[j]) || !(lo[j] < hi[j])) return NULL;
  for (j = 0; j < 2 * d; ++j)
    if (!isfinite(params[j])) return NULL;
  m = init_log2 / d;
  s = (int64_t)1 << m;
  n0 = (int64_t)1 << (m * d);
  if (max_regions < n0) return NULL;
  r = (gmo_run*)calloc(1, sizeof(gmo_run));
  if (!r) {
    *status = GMO_ENOMEM;
    return NULL;
  }
  r->fam = fam;
  r->d = d;
  r->max_iters = max_iters;
  r->keep_leaves = keep_leaves;
  memcpy(r->params, params, sizeof(double) * 2 * d);
  r->rel_tol = rel_tol;
  r->abs_tol = abs_tol;
  r->max_regions = max_regions;
  r->vol_omega = 1.0;
  for (j = 0; j < d; ++j) r->vol_omega = r->vol_omega * (hi[j] - lo[j]);
  if (grow(r, n0)) {
    gmo_free(r);
    *status = GMO_ENOMEM;
    return NULL;
  }
  for (j = 0; j < d; ++j) H[j] = (hi[j] - lo[j]) * 0.5;
  for (t = 0; t < n0; ++t) {
    for (j = 0; j < d; ++j) {
      int64_t kj = (t >> (m * j)) & (s - 1);
      double hj = ldexp(H[j], -m);
      r->h[t * d + j] = hj;
      r->c[t * d + j] = fma((double)(2 * kj + 1), hj, lo[j]);
    }
    r->lvl[t] = m * d;
  }
  r->n = n0;
  r->status = GMO_RUNNING;
  *status = GMO_RUNNING;
  return r;
}

/* Phase A: evaluate, global test, classify (nothing committed yet). */
static int phase_eval(gmo_run* r) {
  int64_t i;
  int d = r->d;
  ksum Is = r->Ifin, Es = r->Efin;
  r->iter++;
  r->stats[GMO_ST_ITERS] = r->iter;
  r->stats[GMO_ST_REGIONS] += r->n;
  r->stats[GMO_ST_EVALS] += r->n * (r->rule == 1   ? gmo_gk_num_nodes(d)
                                     : r->rule == 2 ? gmo_num_nodes9(d)
                                                    : gmo_num_nodes(d));
  r->stats[GMO_ST_ACTIVE] = r->n;
  if (r->n > r->stats[GMO_ST_MAX_ACTIVE]) r->stats[GMO_ST_MAX_ACTIVE] = r->n;
  /* Every region is evaluated on its own; the OpenMP build (the CPU
     baseline's all-cores variant) spreads this loop over threads, and every
     sum below stays serial in store order, so both builds give the same bits. */
  {
    int nonfinite = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) reduction(| : nonfinite)
#endif
    for (i = 0; i < r->n; ++i) {
      int rc;
      double o[16 + 32];
      if (r->rule == 1)
        rc = gmo_rule_gk(r->fam, d, r->params, r->c + i * d, r->h + i * d, r->lvl[i],
                         r->vol_omega, o);
      else if (r->rule == 2)
        rc = gmo_rule9(r->fam, d, r->params, r->c + i * d, r->h + i * d, r->lvl[i], r->vol_omega,
                       r->err_model, o);
      else
        rc = gmo_rule(r->fam, d, r->params, r->c + i * d, r->h + i * d, r->lvl[i], r->vol_omega,
                      o);
      if (rc == GMO_NONFINITE) {
        nonfinite = 1;
        continue;
      }
      r->Q[i] = o[0];
      r->err[i] = o[1];
      r->escl[i] = o[5];
      r->axis[i] = (int32_t)o[2];
      r->geo[i] = (unsigned char)o[3];
    }
    if (nonfinite) {
      r->I = NAN;
      r->E = NAN;
      r->status = GMO_NONFINITE;
      trace_push(r, r->n, 0);
      return r->status;
    }
  }
  for (i = 0; i < r->n; ++i) ks_add(&Is, r->Q[i]);
  for (i = 0; i < r->n; ++i) ks_add(&Es, r->err[i]);
  {
    ksum Ss = r->Sfin;
    for (i = 0; i < r->n; ++i) ks_add(&Ss, r->escl[i]);
    r->Escale = ks_val(&Ss);
  }
  r->I = ks_val(&Is);
  r->E = ks_val(&Es);
  r->T = fmax(r->abs_tol, r->rel_tol * fabs(r->I));
  if (r->E <= r->T) {
    r->status = GMO_OK;
    trace_push(r, r->n, 0);
    return r->status;
  }
  if (r->iter >= r->max_iters) {
    r->status = GMO_MAX_ITERS;
    trace_push(r, r->n, 0);
    return r->status;
  }
  {
    double aI = fabs(r->I);
    int64_t keep = 0, nfin = 0;
    for (i = 0; i < r->n; ++i) {
      int a = r->err[i] <= ldexp(r->T, -r->lvl[i]);
      int b = (aI + r->err[i] == aI);
      int g = r->geo[i];
      r->fin[i] = (unsigned char)(a || b || g);
      if (r->fin[i]) nfin++;
      else keep++;
    }
    r->n_keep = keep;
    trace_push(r, r->n, nfin);
  }
  if (r->n_keep == 0) {
    r->status = r->pruned ? GMO_MAX_REGIONS : GMO_PRECISION_LIMIT;
    return r->status;
  }
  return GMO_RUNNING;
}

/* Smallest k in 1..64 with err <= T 2^(k - lvl) (65: none). */
static int prune_level(double err, double T, int lvl) {
  int k;
  for (k = 1; k <= 64; ++k)
    if (err <= ldexp(T, k - lvl)) return k;
  return 65;
}

/* Memory-pressure pruning (step 7): returns 1 when the kept set was cut down
   to at most capacity/2 regions, 0 when no budget factor up to 2^64 does it. */
static int prune(gmo_run* r) {
  int64_t hist[66], i, above = r->n_keep, half = r->max_regions / 2, nfin;
  int k, ks = -1;
  for (k = 0; k < 66; ++k) hist[k] = 0;
  for (i = 0; i < r->n; ++i)
    if (!r->fin[i]) hist[prune_level(r->err[i], r->T, r->lvl[i])]++;
  for (k = 1; k <= 64; ++k) {
    above -= hist[k];
    if (above <= half) {
      ks = k;
      break;
    }
  }
  if (ks < 0) return 0;
  for (i = 0; i < r->n; ++i)
    if (!r->fin[i] && r->err[i] <= ldexp(r->T, ks - r->lvl[i])) {
      r->fin[i] = 1;
      r->n_keep--;
    }
  r->pruned = 1;
  nfin = r->n - r->n_keep;
  r->trc[2 * (r->ntr - 1) + 1] = nfin; /* this iteration's trace entry */
  return 1;
}

/* Phase C: commit retired regions and split the kept ones. */
static int phase_split(gmo_run* r) {
  int d = r->d;
  int64_t i, p = 0, nk = r->n_keep, n2 = 2 * r->n_keep;
  double *nc_, *nh_;
  int32_t* nl_;
  double aI = fabs(r->I);
  for (i = 0; i < r->n; ++i) {
    if (r->fin[i]) {
      ks_add(&r->Ifin, r->Q[i]);
      ks_add(&r->Efin, r->err[i]);
      ks_add(&r->Sfin, r->escl[i]);
      r->stats[GMO_ST_FINISHED]++;
      if (r->geo[i]) r->stats[GMO_ST_GEOMETRY]++;
      else if (!(r->err[i] <= ldexp(r->T, -r->lvl[i])) && (aI + r->err[i] == aI))
        r->stats[GMO_ST_ROUNDOFF]++;
      if (r->keep_leaves && leaf_push(r, r->c + i * d, r->h + i * d, r->lvl[i])) return GMO_ENOMEM;
    }
  }
  nc_ = (double*)malloc(sizeof(double) * n2 * d);
  nh_ = (double*)malloc(sizeof(double) * n2 * d);
  nl_ = (int32_t*)malloc(sizeof(int32_t) * n2);
  if (!nc_ || !nh_ || !nl_) {
    free(nc_);
    free(nh_);
    free(nl_);
    return GMO_ENOMEM;
  }
  for (i = 0; i < r->n; ++i) {
    if (r->fin[i]) continue;
    {
      int k = r->axis[i];
      double hp = r->h[i * d + k] * 0.5;
      memcpy(nc_ + p * d, r->c + i * d, sizeof(double) * d);
      memcpy(nh_ + p * d, r->h + i * d, sizeof(double) * d);
      memcpy(nc_ + (nk + p) * d, r->c + i * d, sizeof(double) * d);
      memcpy(nh_ + (nk + p) * d, r->h + i * d, sizeof(double) * d);
      nc_[p * d + k] = r->c[i * d + k] - hp;
      nc_[(nk + p) * d + k] = r->c[i * d + k] + hp;
      nh_[p * d + k] = hp;
      nh_[(nk + p) * d + k] = hp;
      nl_[p] = r->lvl[i] + 1;
      nl_[nk + p] = r->lvl[i] + 1;
      p++;
    }
  }
  if (grow(r, n2)) {
    free(nc_);
    free(nh_);
    free(nl_);
    return GMO_ENOMEM;
  }
  memcpy(r->c, nc_, sizeof(double) * n2 * d);
  memcpy(r->h, nh_, sizeof(double) * n2 * d);
  memcpy(r->lvl, nl_, sizeof(int32_t) * n2);
  free(nc_);
  free(nh_);
  free(nl_);
  r->n = n2;
  return GMO_RUNNING;
}

int gmo_set_rule(gmo_run* r, int rule) {
  if (rule < 0 || rule > 2 || (rule == 1 && r->d > 6) || r->iter > 0) return GMO_EINVAL;
  r->rule = rule;
  return GMO_OK;
}

int gmo_set_err_model(gmo_run* r, int model) {
  if (model < 0 || model > 1 || r->iter > 0) return GMO_EINVAL;
  r->err_model = model;
  return GMO_OK;
}

int gmo_set_prune(gmo_run* r, int on) {
  if (on < 0 || on > 1 || r->iter > 0) return GMO_EINVAL;
  r->prune = on;
  return GMO_OK;
}

int gmo_pruned(const gmo_run* r) { return r->pruned; }

int gmo_step(gmo_run* r) {
  int st;
  if (r->status != GMO_RUNNING) return r->status;
  st = phase_eval(r);
  if (st != GMO_RUNNING) return st;
  if (2 * r->n_keep > r->max_regions) {
    if (!r->prune || !prune(r) || r->n_keep == 0) {
      r->status = GMO_MAX_REGIONS;
      return r->status;
    }
  }
  st = phase_split(r);
  if (st != GMO_RUNNING) r->status = st;
  return r->status;
}

int gmo_run_to_end(gmo_run* r) {
  while (r->status == GMO_RUNNING) gmo_step(r);
  return r->status;
}

void gmo_result(const gmo_run* r, double* I, double* E, int* status, int64_t* stats) {
  *I = r->I;
  *E = r->E;
  *status = r->status;
  memcpy(stats, r->stats, sizeof r->stats);
}

int64_t gmo_active_count(const gmo_run* r) { return r->n; }

double gmo_escale(const gmo_run* r) { return r->Escale; }

void gmo_get_active(const gmo_run* r, double* c, double* h, int32_t* lvl, double* Q, double* err,
                    int32_t* axis) {
  int64_t n = r->n;
  int d = r->d;
  if (c) memcpy(c, r->c, sizeof(double) * n * d);
  if (h) memcpy(h, r->h, sizeof(double) * n * d);
  if (lvl) memcpy(lvl, r->lvl, sizeof(int32_t) * n);
  if (Q) memcpy(Q, r->Q, sizeof(double) * n);
  if (err) memcpy(err, r->err, sizeof(double) * n);
  if (axis) memcpy(axis, r->axis, sizeof(int32_t) * n);
}

int64_t gmo_leaf_count(const gmo_run* r) { return r->nleaf + r->n; }

void gmo_get_leaves(const gmo_run* r, double* c, double* h, int32_t* lvl) {
  int d = r->d;
  if (r->nleaf > 0) { /* no leaf list is allocated before the first retirement */
    memcpy(c, r->lc, sizeof(double) * r->nleaf * d);
    memcpy(h, r->lh, sizeof(double) * r->nleaf * d);
    memcpy(lvl, r->llvl, sizeof(int32_t) * r->nleaf);
  }
  memcpy(c + r->nleaf * d, r->c, sizeof(double) * r->n * d);
  memcpy(h + r->nleaf * d, r->h, sizeof(double) * r->n * d);
  memcpy(lvl + r->nleaf, r->lvl, sizeof(int32_t) * r->n);
}

int64_t gmo_trace_len(const gmo_run* r) { return r->ntr; }

void gmo_get_trace(const gmo_run* r, int64_t* counts, double* IE) {
  memcpy(counts, r->trc, sizeof(int64_t) * 2 * r->ntr);
  memcpy(IE, r->trv, sizeof(double) * 2 * r->ntr);
}

void gmo_free(gmo_run* r) {
  if (!r) return;
  free(r->c);
  free(r->h);
  free(r->Q);
  free(r->err);
  free(r->escl);
  free(r->lvl);
  free(r->axis);
  free(r->geo);
  free(r->fin);
  free(r->lc);
  free(r->lh);
  free(r->llvl);
  free(r->trc);
  free(r->trv);
  free(r);
}

/* ------------------------------------------------------------------------ */
/* Fixed-tree quadrature and its gradient.                                   */
/* The gradient is the exact derivative of sum_leaves vol * sum_n w_n f(x_n) */
/* with the tree held fixed: sum_leaves vol * sum_n w_n df/dtheta(x_n).      */
/* ------------------------------------------------------------------------ */
int gmo_quad_leaves(int fam, int d, const double* params, int64_t n, const double* c,
                    const double* h, const int32_t* lvl, double vol_omega, double* out_q) {
  return gmo_quad_leaves_rule(fam, d, params, n, c, h, lvl, vol_omega, 0, out_q);
}

int gmo_quad_leaves_rule(int fam, int d, const double* params, int64_t n, const double* c,
                         const double* h, const int32_t* lvl, double vol_omega, int rule,
                         double* out_q) {
  ksum s = {0.0, 0.0};
  double out[16 + 32];
  int64_t i;
  int st = 0;
  if (rule != 0 && rule != 2) return GMO_EINVAL;
  for (i = 0; i < n; ++i) {
    int rc = rule == 2 ? gmo_rule9(fam, d, params, c + i * d, h + i * d, lvl[i], vol_omega, 0, out)
                       : gmo_rule(fam, d, params, c + i * d, h + i * d, lvl[i], vol_omega, out);
    if (rc) st = GMO_NONFINITE;
    ks_add(&s, out[0]);
  }
  *out_q = ks_val(&s);
  return st;
}

typedef struct {
  int fam, d;
  const double* p;
  double w[8];
  ksum g[32];
} grad_ctx;

static void grad_cb(void* pp, int cls, const double* x) {
  grad_ctx* q = (grad_ctx*)pp;
  double df[32];
  int j;
  gmo_df(q->fam, q->d, q->p, x, df);
  for (j = 0; j < 2 * q->d; ++j) ks_add(&q->g[j], q->w[cls - 1] * df[j]);
}

int gmo_grad_leaves(int fam, int d, const double* params, int64_t n, const double* c,
                    const double* h, const int32_t* lvl, double vol_omega, double* out_grad) {
  return gmo_grad_leaves_rule(fam, d, params, n, c, h, lvl, vol_omega, 0, out_grad);
}

/* The gradient of the fixed-tree quadrature with the degree-7 (rule 0) or
   the degree-9 (rule 2) rule: the same nodes and weights as the rule. */
int gmo_grad_leaves_rule(int fam, int d, const double* params, int64_t n, const double* c,
                         const double* h, const int32_t* lvl, double vol_omega, int rule,
                         double* out_grad) {
  double lam[6], v[5], e[8];
  ksum tot[32];
  int64_t i;
  int j;
  grad_ctx q;
  if (rule != 0 && rule != 2) return GMO_EINVAL;
  memset(tot, 0, sizeof tot);
  memset(&q, 0, sizeof q);
  q.fam = fam;
  q.d = d;
  q.p = params;
  if (rule == 2)
    gmo_constants9(d, lam, q.w, e);
  else
    gmo_constants(d, lam, q.w, v, e);
  for (i = 0; i < n; ++i) {
    double vol = ldexp(vol_omega, -lvl[i]);
    memset(q.g, 0, sizeof q.g);
    if (rule == 2)
      visit_nodes9(d, c + i * d, h + i * d, grad_cb, &q);
    else
      visit_nodes(d, c + i * d, h + i * d, grad_cb, &q);
    for (j = 0; j < 2 * d; ++j) ks_add(&tot[j], vol * ks_val(&q.g[j]));
  }
  for (j = 0; j < 2 * d; ++j) out_grad[j] = ks_val(&tot[j]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Lock-step batch.  Every item runs the loop above with its own tolerance; */
/* all items step together.  Reading of a shared region budget: when the    */
/* kept regions of all still-running items would need more than             */
/* max_regions_total rows after splitting, every still-running item stops    */
/* with the max-regions status and its current (I, E).  Below that budget    */
/* each item's result is that of an independent run.                         */
/* ------------------------------------------------------------------------ */
int gmo_integrate_batch(int n, const int* fam, const double* params, const int* d,
                        const double* lo, const double* hi, const double* rel_tol,
                        const double* abs_tol, int64_t max_regions_total, int init_log2,
                        int max_iters, double* out_est, double* out_err, int* out_status,
                        int64_t* out_iters) {
  return gmo_integrate_batch_rule(n, fam, params, d, lo, hi, rel_tol, abs_tol, max_regions_total,
                                  init_log2, max_iters, 0, 0, out_est, out_err, out_status,
                                  out_iters);
}

int gmo_integrate_batch_rule(int n, const int* fam, const double* params, const int* d,
                             const double* lo, const double* hi, const double* rel_tol,
                             const double* abs_tol, int64_t max_regions_total, int init_log2,
                             int max_iters, int rule, int err_model, double* out_est,
                             double* out_err, int* out_status, int64_t* out_iters) {
  gmo_run** runs;
  int i, worst = 0, running;
  int64_t po = 0, bo = 0;
  if (n < 1) return GMO_EINVAL;
  runs = (gmo_run**)calloc((size_t)n, sizeof(gmo_run*));
  if (!runs) return GMO_ENOMEM;
  for (i = 0; i < n; ++i) {
    int st;
    runs[i] = gmo_create(fam[i], d[i], params + po, lo + bo, hi + bo, rel_tol[i], abs_tol[i],
                         max_regions_total, init_log2, max_iters, 0, &st);
    po += 2 * d[i];
    bo += d[i];
    if (!runs[i]) {
      out_status[i] = st;
    } else if (gmo_set_rule(runs[i], rule) != GMO_OK ||
               gmo_set_err_model(runs[i], err_model) != GMO_OK) {
      gmo_free(runs[i]);
      runs[i] = NULL;
      out_status[i] = GMO_EINVAL;
    }
  }
  /* The initial partitions must fit together. */
  {
    int64_t tot = 0;
    for (i = 0; i < n; ++i)
      if (runs[i]) tot += runs[i]->n;
    if (tot > max_regions_total) {
      for (i = 0; i < n; ++i) gmo_free(runs[i]);
      free(runs);
      return GMO_EINVAL;
    }
  }
  do {
    int64_t need = 0;
    running = 0;
    for (i = 0; i < n; ++i) {
      if (!runs[i] || runs[i]->status != GMO_RUNNING) continue;
      if (phase_eval(runs[i]) == GMO_RUNNING) {
        need += 2 * runs[i]->n_keep;
        running++;
      }
    }
    if (running && need > max_regions_total) {
      for (i = 0; i < n; ++i)
        if (runs[i] && runs[i]->status == GMO_RUNNING) runs[i]->status = GMO_MAX_REGIONS;
      running = 0;
    }
    for (i = 0; i < n; ++i) {
      if (!runs[i] || runs[i]->status != GMO_RUNNING) continue;
      if (phase_split(runs[i]) != GMO_RUNNING) runs[i]->status = GMO_ENOMEM;
    }
  } while (running);
  for (i = 0; i < n; ++i) {
    if (!runs[i]) {
      out_est[i] = NAN;
      out_err[i] = NAN;
      if (out_iters) out_iters[i] = 0;
      continue;
    }
    out_est[i] = runs[i]->I;
    out_err[i] = runs[i]->E;
    out_status[i] = runs[i]->status;
    if (out_iters) out_iters[i] = runs[i]->iter;
    if (runs[i]->status > worst) worst = runs[i]->status;
    gmo_free(runs[i]);
  }
  free(runs);
  return worst;
}

/* Threads the evaluation loop uses (1 in the serial build). */
int gmo_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
