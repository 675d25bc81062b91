// gm_gk.hip -- the tensor-product Gauss-Kronrod rule kernel: the second rule
// of the framework (arXiv 2511.01573, Sec. 3: "a tensor-product Gauss-Kronrod
// rule"), for 2 <= d <= 6 (its cost grows as 15^d, prohibitive from d = 7 on,
// as the paper reports).
//
// Rule.  On each axis the 15-point Kronrod extension of the 7-point
// Gauss-Legendre rule; the tensor product over the d axes gives Q = Q_K
// (15^d nodes).  err = vol |Q_K - Q_G|, Q_G the tensor Gauss rule on the 7^d
// Gauss nodes among them.  Split axis: the i with the largest one-axis
// estimate vol |Q_K - Q_{K, Gauss on axis i}|, with the Genz-Malik rule's tie
// band (relative to vol times the Kronrod sum of |f|), widest half-width, then
// lowest index; geometry guard as for that rule.
//
// Mapping: one wavefront per region, four regions per workgroup.  Lane l takes
// the index pairs (k_0, k_1) = l, l + 64, ... of the first two axes' 225 pairs;
// the remaining axes are contracted inside the lane one axis at a time (sum
// factorisation): a level returns its all-Kronrod sum, all-Gauss sum, Kronrod
// sum of |f| and, for each deeper axis i, the sum with Gauss weights on axis i
// alone.  The per-axis terms T_j(c_j + x_k h_j) are tabulated once per region
// in LDS; every node argument is the left-to-right chain of the terms, as in
// the Genz-Malik kernel.  Lane sums are combined with double-double shuffles.
#include "gm_family.hpp"
#include "gm_gk_table.hpp"

namespace gm {

constexpr int kGkRegionsPerBlock = kRuleBlock / 64;

template <int D>
struct GkSums {
  double a;      // Kronrod weights on every contracted axis
  double b;      // Gauss weights on every contracted axis
  double abs_a;  // Kronrod weights, |f|
  double m[D];   // m[i]: Gauss weights on axis i, Kronrod on the other contracted axes
};

// Contraction of axes J .. D-1 below the argument prefix s.
template <int D, int FAM, int J>
__device__ __forceinline__ void gk_contract(const DevParams& P, const double (*tt)[15], double s,
                                            GkSums<D>& out) {
  using F = Fam<FAM>;
  if constexpr (J == D - 1) {
    // innermost axis: 15 nodes, outer functions in three interleaved groups of 5
    double a = 0.0, b = 0.0, ab = 0.0;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      double arg[5], f[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) arg[q] = F::comb(s, tt[J][5 * g + q]);
      F::template outer_n<D, 5>(P, arg, f);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const int k = 5 * g + q;
        a = fma(gk::kWK[k], f[q], a);
        if (gk::kWG[k] != 0.0) b = fma(gk::kWG[k], f[q], b);
        ab = fma(gk::kWK[k], fabs(f[q]), ab);
      }
    }
    out.a = a;
    out.b = b;
    out.abs_a = ab;
    out.m[J] = b;
  } else {
    GkSums<D> acc;
    acc.a = acc.b = acc.abs_a = 0.0;
#pragma unroll
    for (int i = J; i < D; ++i) acc.m[i] = 0.0;
    for (int k = 0; k < 15; ++k) {
      GkSums<D> ch;
      gk_contract<D, FAM, J + 1>(P, tt, F::comb(s, tt[J][k]), ch);
      const double wk = gk::kWK[k], wg = gk::kWG[k];
      acc.a = fma(wk, ch.a, acc.a);
      acc.b = fma(wg, ch.b, acc.b);
      acc.abs_a = fma(wk, ch.abs_a, acc.abs_a);
      acc.m[J] = fma(wg, ch.a, acc.m[J]);
#pragma unroll
      for (int i = J + 1; i < D; ++i) acc.m[i] = fma(wk, ch.m[i], acc.m[i]);
    }
    out = acc;
  }
}

template <int D, int FAM, bool BATCH>
__global__ __launch_bounds__(kRuleBlock) void rule_gk_kernel(RuleArgs A) {
  using F = Fam<FAM>;
  int64_t start, end;
  int buf;
  if (!active_range<BATCH>(A, start, end, buf)) return;
  const RegionSrc R = region_src<BATCH>(A, buf);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ double tt[kGkRegionsPerBlock][D][15];
  dd qs = {0.0, 0.0}, es = {0.0, 0.0};
  int nonfin = 0;
  // The trip count depends on the workgroup only, so the barriers are uniform.
  for (int64_t base = start + (int64_t)blockIdx.x * kGkRegionsPerBlock; base < end;
       base += (int64_t)gridDim.x * kGkRegionsPerBlock) {
    const int64_t r = base + wv;
    const bool ok = r < end;
    double volo;
    const DevParams& P = region_params<BATCH>(A, buf, ok ? r : start, volo);
    double c[D], h[D];
    int lvl = 0;
    if (ok) {
      lvl = load_region<D>(R, r, c, h);
    } else {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        c[j] = 0.0;
        h[j] = 0.0;
      }
    }
    if (ok && lane < 15) {
      const double xk = gk::kX[lane];
#pragma unroll
      for (int j = 0; j < D; ++j) tt[wv][j][lane] = F::term(P, j, fma(xk, h[j], c[j]));
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0, sab = 0.0, sm[D];
#pragma unroll
    for (int i = 0; i < D; ++i) sm[i] = 0.0;
    if (ok) {
      for (int o = lane; o < 225; o += 64) {
        const int k0 = o / 15, k1 = o - 15 * k0;
        const double s = F::comb(tt[wv][0][k0], tt[wv][1][k1]);
        GkSums<D> g;
        if constexpr (D == 2) {
          const double f = F::template outer<D>(P, s);
          g.a = f;
          g.b = f;
          g.abs_a = fabs(f);
        } else {
          gk_contract<D, FAM, 2>(P, tt[wv], s, g);
        }
        const double wk0 = gk::kWK[k0], wk1 = gk::kWK[k1];
        const double wg0 = gk::kWG[k0], wg1 = gk::kWG[k1];
        const double wkk = wk0 * wk1;
        sa = fma(wkk, g.a, sa);
        sb = fma(wg0 * wg1, g.b, sb);
        sab = fma(wkk, g.abs_a, sab);
        sm[0] = fma(wg0 * wk1, g.a, sm[0]);
        sm[1] = fma(wk0 * wg1, g.a, sm[1]);
#pragma unroll
        for (int i = 2; i < D; ++i) sm[i] = fma(wkk, g.m[i], sm[i]);
      }
    }
    const dd ta = wave_sum_dd(dd{sa, 0.0});
    const dd tb = wave_sum_dd(dd{sb, 0.0});
    const dd tab = wave_sum_dd(dd{sab, 0.0});
    double tm[D];
#pragma unroll
    for (int i = 0; i < D; ++i) tm[i] = dd_val(wave_sum_dd(dd{sm[i], 0.0}));
    if (ok && lane == 0) {
      const double vol = ldexp(volo, -lvl);
      const double QK = dd_val(ta), QG = dd_val(tb);
      RegionResult o;
      o.q = vol * QK;
      o.err = vol * fabs(QK - QG);
      double e[D], emax = -1.0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        e[i] = vol * fabs(QK - tm[i]);
        emax = e[i] > emax ? e[i] : emax;
      }
      const double thr = emax - A.K.axis_band * (vol * dd_val(tab));
      int axis = -1;
      double hb = 0.0, cb = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        if (e[i] >= thr && (axis < 0 || h[i] > hb)) {
          axis = i;
          hb = h[i];
          cb = c[i];
        }
      }
      if (axis < 0) {
        axis = 0;
        hb = h[0];
        cb = c[0];
      }
      const double hp = hb * 0.5;
      o.axis = axis;
      o.geo = (cb - hp == cb) || (cb + hp == cb) || (hp == 0.0);
      o.nonfinite = !(isfinite(QK) && isfinite(QG)) || !F::in_range(P, c, h);
      store_result(A, r, o);
      dd_add(qs, o.q);
      dd_add(es, o.err);
      nonfin |= o.nonfinite;
    }
    __syncthreads();
  }
  if constexpr (!BATCH) block_partials(A, qs, es, nonfin);
}

#ifndef GM_RULE_FAMILY
#error "gm_gk.hip is compiled once per integrand family (-DGM_RULE_FAMILY=k)"
#endif

#define GM_GK_CAT2(a, b) a##b
#define GM_GK_CAT(a, b) GM_GK_CAT2(a, b)

RuleKernelFn GM_GK_CAT(gk_kernel_f, GM_RULE_FAMILY)(int d, bool batch) {
  constexpr int F = GM_RULE_FAMILY;
  switch (d) {
    case 2: return batch ? rule_gk_kernel<2, F, true> : rule_gk_kernel<2, F, false>;
    case 3: return batch ? rule_gk_kernel<3, F, true> : rule_gk_kernel<3, F, false>;
    case 4: return batch ? rule_gk_kernel<4, F, true> : rule_gk_kernel<4, F, false>;
    case 5: return batch ? rule_gk_kernel<5, F, true> : rule_gk_kernel<5, F, false>;
    case 6: return batch ? rule_gk_kernel<6, F, true> : rule_gk_kernel<6, F, false>;
    default: return nullptr;
  }
}

}  // namespace gm
