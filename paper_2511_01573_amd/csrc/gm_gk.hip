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
// Mapping: up to d = 3 one wavefront per region (four regions per workgroup),
// lane l taking the index pairs (k_0, k_1) = l, l + 64, ... of the first two
// axes' 225 pairs; from d = 4 on a whole workgroup per region, thread t taking
// the triples t, t + 256, ... of the first three axes' 3375.  The remaining
// axes are contracted inside the thread one axis at a time (sum
// factorisation): a level returns its all-Kronrod sum, all-Gauss sum, Kronrod
// sum of |f| and, for each deeper axis i, the sum with Gauss weights on axis i
// alone.  The per-axis terms T_j(c_j + x_k h_j) are tabulated once per region
// in LDS; every node argument is the left-to-right chain of the terms, as in
// the Genz-Malik kernel.  Thread sums are combined with double-double
// shuffles within a wavefront and through LDS across wavefronts.
#include "gm_family.hpp"
#include "gm_gk_table.hpp"

namespace gm {

// Leading axes whose index tuples are spread over a region's gk_threads(d)
// threads: the 225 pairs of axes 0, 1 for one wavefront, the 3375 triples of
// axes 0, 1, 2 for a whole workgroup.
template <int D>
constexpr int gk_spread_axes() { return gk_threads(D) > 64 ? 3 : 2; }

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
  constexpr int NT = gk_threads(D);  // threads per region
  constexpr int RPB = kRuleBlock / NT;  // regions per block step
  constexpr int SPREAD = gk_spread_axes<D>();
  constexpr int NTUPLE = SPREAD == 3 ? 3375 : 225;
  constexpr int NW = NT / 64;  // wavefronts per region
  int64_t start, end;
  int buf;
  if (!active_range<BATCH>(A, start, end, buf)) return;
  const RegionSrc R = region_src<BATCH>(A, buf);
  const int slot = threadIdx.x / NT, t = threadIdx.x % NT;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ double tt[RPB][D][15];
  __shared__ dd red[kRuleBlock / 64][3 + D];  // per-wavefront partial sums
  dd qs = {0.0, 0.0}, es = {0.0, 0.0};
  int nonfin = 0;
  // The trip count depends on the workgroup only, so the barriers are uniform.
  for (int64_t base = start + (int64_t)blockIdx.x * RPB; base < end;
       base += (int64_t)gridDim.x * RPB) {
    const int64_t r = base + slot;
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
    if (ok && t < 15) {
      const double xk = gk::kX[t];
#pragma unroll
      for (int j = 0; j < D; ++j) tt[slot][j][t] = F::term(P, j, fma(xk, h[j], c[j]));
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0, sab = 0.0, sm[D];
#pragma unroll
    for (int i = 0; i < D; ++i) sm[i] = 0.0;
    if (ok) {
      for (int o = t; o < NTUPLE; o += NT) {
        if constexpr (SPREAD == 2) {
          const int k0 = o / 15, k1 = o - 15 * k0;
          const double s = F::comb(tt[slot][0][k0], tt[slot][1][k1]);
          GkSums<D> g;
          if constexpr (D == 2) {
            const double f = F::template outer<D>(P, s);
            g.a = f;
            g.b = f;
            g.abs_a = fabs(f);
          } else {
            gk_contract<D, FAM, 2>(P, tt[slot], s, g);
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
        } else {
          const int k0 = o / 225, k12 = o - 225 * k0;
          const int k1 = k12 / 15, k2 = k12 - 15 * k1;
          const double s =
              F::comb(F::comb(tt[slot][0][k0], tt[slot][1][k1]), tt[slot][2][k2]);
          GkSums<D> g;
          gk_contract<D, FAM, 3>(P, tt[slot], s, g);
          const double wk0 = gk::kWK[k0], wk1 = gk::kWK[k1], wk2 = gk::kWK[k2];
          const double wg0 = gk::kWG[k0], wg1 = gk::kWG[k1], wg2 = gk::kWG[k2];
          const double wkkk = (wk0 * wk1) * wk2;
          sa = fma(wkkk, g.a, sa);
          sb = fma((wg0 * wg1) * wg2, g.b, sb);
          sab = fma(wkkk, g.abs_a, sab);
          sm[0] = fma((wg0 * wk1) * wk2, g.a, sm[0]);
          sm[1] = fma((wk0 * wg1) * wk2, g.a, sm[1]);
          sm[2] = fma((wk0 * wk1) * wg2, g.a, sm[2]);
#pragma unroll
          for (int i = 3; i < D; ++i) sm[i] = fma(wkkk, g.m[i], sm[i]);
        }
      }
    }
    // Sums over the region's threads: double-double within each wavefront,
    // then across the region's wavefronts through LDS.
    dd tot[3 + D];
    tot[0] = wave_sum_dd(dd{sa, 0.0});
    tot[1] = wave_sum_dd(dd{sb, 0.0});
    tot[2] = wave_sum_dd(dd{sab, 0.0});
#pragma unroll
    for (int i = 0; i < D; ++i) tot[3 + i] = wave_sum_dd(dd{sm[i], 0.0});
    if constexpr (NW > 1) {
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 3 + D; ++q) red[wv][q] = tot[q];
      }
      __syncthreads();
      if (t == 0) {
#pragma unroll
        for (int q = 0; q < 3 + D; ++q) {
          dd v = red[slot * NW][q];
          for (int w = 1; w < NW; ++w) v = dd_sum(v, red[slot * NW + w][q]);
          tot[q] = v;
        }
      }
    }
    if (ok && t == 0) {
      const double vol = ldexp(volo, -lvl);
      const double QK = dd_val(tot[0]), QG = dd_val(tot[1]);
      RegionResult o;
      o.q = vol * QK;
      o.err = vol * fabs(QK - QG);
      double e[D], emax = -1.0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        e[i] = vol * fabs(QK - dd_val(tot[3 + i]));
        emax = e[i] > emax ? e[i] : emax;
      }
      const double thr = emax - A.K.axis_band * (vol * dd_val(tot[2]));
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

GM_CHECK_UNIT_F(gk, GM_RULE_FAMILY)

}  // namespace gm
