// gm_rule.hip -- the rule kernel: Genz-Malik rule, embedded-rule error
// estimate and fourth-difference split axis on every active region
// (arXiv 2511.01573, Sec. 2; the "evaluate subregions" step of Sec. 3).
//
// Node arithmetic.  Every integrand family is f(x) = G(T_0(x_0) (+) T_1(x_1)
// (+) ... (+) T_{d-1}(x_{d-1})) with a per-coordinate term T_j, a left-to-
// right combination (+) (a sum, or a product for the product peak) and an
// outer function G.  A region's nodes take only seven values per coordinate
// (c, c +- l2 h, c +- l3 h = c +- l4 h, c +- l5 h), so the terms are formed
// once per region and every node's argument is a chain of (+) over those
// terms in the same left-to-right order as the defining formula.  Common
// prefixes of the chain are shared:
//   - classes 1-4 (the centre, +-l2 e_i, +-l3 e_i, +-l4 (e_i +- e_j)) reuse
//     the prefix of centre terms up to the first perturbed coordinate;
//   - class 5 (the 2^d corners) is swept as a binary tree over the last four
//     coordinates below an outer loop over the leading ones, so a corner
//     costs about two (+) plus one G.
//
// Mappings.
//   TPR (d <= 10): one lane per region, fully unrolled classes 1-4.
//   WPR: L = 2^l lanes per region inside one wavefront.  Lane s fixes the
//        signs of the first l coordinates of the corners it sweeps; the
//        O(d^2) class 1-4 nodes are dealt out to the L lanes as work items
//        (one axis: 4 nodes and its fourth difference; one axis pair: 4
//        nodes) using per-region term tables in LDS.  Class sums are combined
//        across the L lanes with shuffles.
// Class sums are compensated per small group of nodes (TwoSum per 16 corners,
// per +- pair, per class 4 row).
#include "gm_corner.hpp"

namespace gm {

// Unrolling of the class 2/3 and class 4 loops of the one-lane-per-region
// kernel (full unrolling keeps every index compile-time; a count of 1 keeps
// the loops and indexes the term arrays with wavefront-uniform counters,
// which lowers register use).
#ifndef GM_UNROLL_A23
#define GM_UNROLL_A23 64
#endif
#ifndef GM_UNROLL_A4
#define GM_UNROLL_A4 64
#endif

__device__ __forceinline__ void rule_combine(const RuleConsts& K, double s1, double s2, double s3,
                                             double s4, double s5, double vol, RegionResult& r) {
  r.nonfinite = !(isfinite(s1) && isfinite(s2) && isfinite(s3) && isfinite(s4) && isfinite(s5));
  double q = K.w[0] * s1 + K.w[1] * s2;
  q = q + K.w[2] * s3;
  q = q + K.w[3] * s4;
  q = q + K.w[4] * s5;
  double er = K.e[0] * s1 + K.e[1] * s2;
  er = er + K.e[2] * s3;
  er = er + K.e[3] * s4;
  er = er + K.e[4] * s5;
  r.q = vol * q;
  r.err = vol * fabs(er);
}

// ---------------------------------------------------------------------------
// TPR: one lane per region (d <= 10).
// ---------------------------------------------------------------------------
template <int D, int FAM>
__device__ __forceinline__ RegionResult rule_region_tpr(const DevParams& P, const RuleConsts& K,
                                                        const double (&c)[D], const double (&h)[D],
                                                        double vol) {
  using F = Fam<FAM>;
  // Terms at the centre and at +-l3 (= +-l4) per coordinate; the +-l2 terms
  // are formed where they are used to keep the live register set small.
  double tc[D], t3p[D], t3m[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    tc[j] = F::term(P, j, c[j]);
    t3p[j] = F::term(P, j, fma(K.lam3, h[j], c[j]));
    t3m[j] = F::term(P, j, fma(-K.lam3, h[j], c[j]));
  }
  // pc[k] = tc[0] (+) ... (+) tc[k-1]
  double pc[D + 1];
  pc[0] = 0.0;
  pc[1] = tc[0];
#pragma unroll
  for (int k = 2; k <= D; ++k) pc[k] = F::comb(pc[k - 1], tc[k - 1]);
  const double f0 = F::template outer<D>(P, pc[D]);
  KSum S2 = {0.0, 0.0}, S3 = {0.0, 0.0}, S4 = {0.0, 0.0}, S5 = {0.0, 0.0};
  double Dv[D];
  double scale = 0.0;
#pragma unroll GM_UNROLL_A23
  for (int i = 0; i < D; ++i) {
    const double v[4] = {F::term(P, i, fma(K.lam2, h[i], c[i])),
                         F::term(P, i, fma(-K.lam2, h[i], c[i])), t3p[i], t3m[i]};
    double a[4], f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double s = (i == 0) ? v[q] : F::comb(pc[i], v[q]);
#pragma unroll GM_UNROLL_A23
      for (int k = i + 1; k < D; ++k) s = F::comb(s, tc[k]);
      a[q] = s;
    }
    F::template outer_n<D, 4>(P, a, f);
    ks_add(S2, f[0] + f[1]);
    ks_add(S3, f[2] + f[3]);
    double sc;
    fourth_diff(K, f0, f[0], f[1], f[2], f[3], Dv[i], sc);
    scale = sc > scale ? sc : scale;
  }
  // Class 4 walks (i, j) with loop counters that are the same in every lane
  // of the wavefront, so the term arrays are indexed uniformly.  Class sums
  // are compensated at the level of small groups: the +-pair of each class 2/3
  // axis and the (at most 2(d-1)) nodes of one (i, sign_i) row of class 4 are
  // added plainly and each group sum enters the compensated total.
#pragma unroll GM_UNROLL_A4
  for (int i = 0; i < D - 1; ++i) {
#pragma unroll
    for (int si = 0; si < 2; ++si) {
      const double ti = si ? t3m[i] : t3p[i];
      double m = (i == 0) ? ti : F::comb(pc[i], ti);
      double g = 0.0;
#pragma unroll GM_UNROLL_A4
      for (int j = i + 1; j < D; ++j) {
        double a[2], fv[2];
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          double s = F::comb(m, sj ? t3m[j] : t3p[j]);
#pragma unroll GM_UNROLL_A4
          for (int k = j + 1; k < D; ++k) s = F::comb(s, tc[k]);
          a[sj] = s;
        }
        F::template outer_n<D, 2>(P, a, fv);
        g = (j == i + 1) ? fv[0] : g + fv[0];
        g = g + fv[1];
        m = F::comb(m, tc[j]);
      }
      ks_add(S4, g);
    }
  }
  {
    double t5p[D], t5m[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      t5p[j] = F::term(P, j, fma(K.lam5, h[j], c[j]));
      t5m[j] = F::term(P, j, fma(-K.lam5, h[j], c[j]));
    }
    corner_sweep<D, FAM, 0>(P, t5p, t5m, 0u, S5);
  }

  RegionResult r;
  rule_combine(K, f0, ks_val(S2), ks_val(S3), ks_val(S4), ks_val(S5), vol, r);
  double dmax = -1.0;
#pragma unroll
  for (int i = 0; i < D; ++i) dmax = Dv[i] > dmax ? Dv[i] : dmax;
  const double thr = dmax - K.axis_band * scale;
  int axis = -1;
  double hb = 0.0, cb = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    if (Dv[i] >= thr && (axis < 0 || h[i] > hb)) {
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
  r.axis = axis;
  r.geo = (cb - hp == cb) || (cb + hp == cb) || (hp == 0.0);
  r.nonfinite |= !F::in_range(P, c, h);
  return r;
}

// Two wavefronts per SIMD: the compiler keeps the register file at 256 per
// lane (a few phase-A values spill to scratch, none inside the corner loop) so
// a second wavefront hides the latency of the first one's dependent FP64
// chains and loads.
#ifndef GM_TPR_WAVES
#define GM_TPR_WAVES 2
#endif
template <int D, int FAM, bool BATCH>
__global__ __launch_bounds__(kRuleBlock) __attribute__((amdgpu_waves_per_eu(GM_TPR_WAVES)))
void rule_tpr_kernel(RuleArgs A) {
  int64_t start, end;
  int buf;
  if (!active_range<BATCH>(A, start, end, buf)) return;
  const RegionSrc R = region_src<BATCH>(A, buf);
  const int64_t stride = (int64_t)gridDim.x * kRuleBlock;
  dd qs = {0.0, 0.0}, es = {0.0, 0.0};
  int nonfin = 0;
  // A split set holds the two children of parent q at q and q + n_par; lane
  // v takes child v & 1 of parent v >> 1, so siblings sit in neighbouring
  // lanes and a wavefront reads each parent record once.
  const bool pairs = R.split && end == 2 * R.npar;
  int64_t v = start + (int64_t)blockIdx.x * kRuleBlock + threadIdx.x;
  for (; v < end; v += stride) {
    const int64_t r = pairs ? ((v & 1) ? R.npar + (v >> 1) : (v >> 1)) : v;
    double c[D], h[D];
    const int lvl = load_region<D>(R, r, c, h);
    double volo;
    const DevParams& P = region_params<BATCH>(A, buf, r, volo);
    const double vol = ldexp(volo, -lvl);
    const RegionResult o = rule_region_tpr<D, FAM>(P, A.K, c, h, vol);
    store_result(A, r, o);
    dd_add(qs, o.q);
    dd_add(es, o.err);
    nonfin |= o.nonfinite;
  }
  if constexpr (!BATCH) block_partials(A, qs, es, nonfin);
}

// ---------------------------------------------------------------------------
// WPR: L = 2^LOG2L lanes per region.
// ---------------------------------------------------------------------------
// LDS per region: c[D], h[D], tc[D], pc[D] (pc[k] = tc[0] (+) .. (+) tc[k-1]),
// D_i[D], scale_i[D].
template <int D>
struct WprSlot {
  double c[D], h[D], tc[D], pc[D], dv[D], sc[D];
};

template <int D, int FAM, int LOG2L, bool BATCH>
__global__ __launch_bounds__(kRuleBlock) void rule_wpr_kernel(RuleArgs A) {
  using F = Fam<FAM>;
  constexpr int L = 1 << LOG2L;
  constexpr int RPB = kRuleBlock / L;  // regions per block step
  constexpr int NPAIR = D * (D - 1) / 2;
  constexpr int NITEM = D + NPAIR;
  __shared__ WprSlot<D> slots[RPB];
  int64_t start, n;
  int buf;
  if (!active_range<BATCH>(A, start, n, buf)) return;
  const RegionSrc R = region_src<BATCH>(A, buf);
  const RuleConsts& K = A.K;
  const int g = threadIdx.x >> LOG2L;  // region slot in the block
  const int s = threadIdx.x & (L - 1);
  WprSlot<D>& sl = slots[g];
  dd qs = {0.0, 0.0}, es = {0.0, 0.0};
  int nonfin = 0;
  for (int64_t base = start + (int64_t)blockIdx.x * RPB; base < n;
       base += (int64_t)gridDim.x * RPB) {
    const int64_t r = base + g;
    const bool valid = r < n;
    double volo;
    const DevParams& P = region_params<BATCH>(A, buf, valid ? r : start, volo);
    double c[D], h[D];
    int lvl = 0;
    if (valid) {
      lvl = load_region<D>(R, r, c, h);
    } else {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        c[j] = 0.5;
        h[j] = 0.25;
      }
    }
    // Per-region tables (each lane of the group writes the coordinates j = s mod L).
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if ((j & (L - 1)) == s) {
        sl.c[j] = c[j];
        sl.h[j] = h[j];
      }
    }
    double tc[D];
#pragma unroll
    for (int j = 0; j < D; ++j) tc[j] = F::term(P, j, c[j]);
    double pc = 0.0, full = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if ((k & (L - 1)) == s) {
        sl.tc[k] = tc[k];
        sl.pc[k] = pc;
      }
      pc = (k == 0) ? tc[0] : F::comb(pc, tc[k]);
    }
    full = pc;
    __syncthreads();
    const double f0 = F::template outer<D>(P, full);
    KSum S2 = {0.0, 0.0}, S3 = {0.0, 0.0}, S4 = {0.0, 0.0}, S5 = {0.0, 0.0};
    // Classes 2-4 as work items.  The chains run over the lane's own centre
    // terms (registers) with the runtime bounds as predicates, so an item's
    // nodes advance together instead of waiting on one LDS load per step.
    for (int it = s; it < NITEM; it += L) {
      if (it < D) {
        const int i = it;
        const double ci = sl.c[i], hi = sl.h[i];
        const double v[4] = {F::term(P, i, fma(K.lam2, hi, ci)), F::term(P, i, fma(-K.lam2, hi, ci)),
                             F::term(P, i, fma(K.lam3, hi, ci)), F::term(P, i, fma(-K.lam3, hi, ci))};
        double a[4], f[4];
        const double pci = sl.pc[i];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = (i == 0) ? v[q] : F::comb(pci, v[q]);
        chain_from<D, FAM, 4>(a, tc, i + 1, D);
        F::template outer_n<D, 4>(P, a, f);
        ks_add(S2, f[0]);
        ks_add(S2, f[1]);
        ks_add(S3, f[2]);
        ks_add(S3, f[3]);
        double dv, scv;
        fourth_diff(K, f0, f[0], f[1], f[2], f[3], dv, scv);
        sl.dv[i] = dv;
        sl.sc[i] = scv;
      } else {
        int i, j;
        pair_of<D>(it - D, i, j);
        const double ci = sl.c[i], hi = sl.h[i], cj = sl.c[j], hj = sl.h[j];
        const double tj[2] = {F::term(P, j, fma(K.lam4, hj, cj)), F::term(P, j, fma(-K.lam4, hj, cj))};
        const double pci = sl.pc[i];
        double m[2];
#pragma unroll
        for (int si = 0; si < 2; ++si) {
          const double ti = F::term(P, i, fma(si ? -K.lam4 : K.lam4, hi, ci));
          m[si] = (i == 0) ? ti : F::comb(pci, ti);
        }
        chain_from<D, FAM, 2>(m, tc, i + 1, j);
        double a[4] = {F::comb(m[0], tj[0]), F::comb(m[0], tj[1]), F::comb(m[1], tj[0]),
                       F::comb(m[1], tj[1])};
        chain_from<D, FAM, 4>(a, tc, j + 1, D);
        double f[4];
        F::template outer_n<D, 4>(P, a, f);
#pragma unroll
        for (int q = 0; q < 4; ++q) ks_add(S4, f[q]);
      }
    }
    // Class 5: this lane's 2^(D - LOG2L) corners.
    {
      double t5p[D], t5m[D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        t5p[j] = F::term(P, j, fma(K.lam5, h[j], c[j]));
        t5m[j] = F::term(P, j, fma(-K.lam5, h[j], c[j]));
      }
      corner_sweep<D, FAM, LOG2L>(P, t5p, t5m, (uint32_t)s, S5);
    }
    // Combine the L lanes of the group.
#pragma unroll
    for (int m = L / 2; m >= 1; m >>= 1) {
      S2 = ks_merge(S2, shfl_xor_ks(S2, m));
      S3 = ks_merge(S3, shfl_xor_ks(S3, m));
      S4 = ks_merge(S4, shfl_xor_ks(S4, m));
      S5 = ks_merge(S5, shfl_xor_ks(S5, m));
    }
    __syncthreads();
    RegionResult o;
    o.q = 0.0;
    o.err = 0.0;
    o.nonfinite = 0;
    if (s == 0 && valid) {
      const double vol = ldexp(volo, -lvl);
      rule_combine(K, f0, ks_val(S2), ks_val(S3), ks_val(S4), ks_val(S5), vol, o);
      double dmax = -1.0, scale = 0.0;
      for (int i = 0; i < D; ++i) {
        dmax = sl.dv[i] > dmax ? sl.dv[i] : dmax;
        scale = sl.sc[i] > scale ? sl.sc[i] : scale;
      }
      const double thr = dmax - K.axis_band * scale;
      int axis = -1;
      double hb = 0.0, cb = 0.0;
      for (int i = 0; i < D; ++i) {
        if (sl.dv[i] >= thr && (axis < 0 || sl.h[i] > hb)) {
          axis = i;
          hb = sl.h[i];
          cb = sl.c[i];
        }
      }
      if (axis < 0) {
        axis = 0;
        hb = sl.h[0];
        cb = sl.c[0];
      }
      const double hp = hb * 0.5;
      o.axis = axis;
      o.geo = (cb - hp == cb) || (cb + hp == cb) || (hp == 0.0);
      o.nonfinite |= !F::in_range_rt(P, D, sl.c, sl.h);
      store_result(A, r, o);
      dd_add(qs, o.q);
      dd_add(es, o.err);
      nonfin |= o.nonfinite;
    }
    __syncthreads();
  }
  if constexpr (!BATCH) block_partials(A, qs, es, nonfin);
}

// ---------------------------------------------------------------------------
// Dispatch over (d, mapping) for the family this translation unit is built
// for (-DGM_RULE_FAMILY=k; the build compiles one object per family).
// ---------------------------------------------------------------------------
#ifndef GM_RULE_FAMILY
#error "compile with -DGM_RULE_FAMILY=<1..7>"
#endif

template <int D, bool B>
static RuleKernelFn pick(int log2l) {
  constexpr int F = GM_RULE_FAMILY;
  if (log2l < 0) {
    if constexpr (D <= kTprMaxDim) return rule_tpr_kernel<D, F, B>;
    return nullptr;
  }
  if constexpr (D >= 6) {
    if (log2l == 2) return rule_wpr_kernel<D, F, 2, B>;
    if constexpr (D >= 8) {
      if (log2l == 4) return rule_wpr_kernel<D, F, 4, B>;
    }
    if constexpr (D >= 10) {
      if (log2l == 6) return rule_wpr_kernel<D, F, 6, B>;
    }
  }
  return nullptr;
}

template <bool B>
static RuleKernelFn rule_fn(int d, int log2l) {
  switch (d) {
    case 2: return pick<2, B>(log2l);
    case 3: return pick<3, B>(log2l);
    case 4: return pick<4, B>(log2l);
    case 5: return pick<5, B>(log2l);
    case 6: return pick<6, B>(log2l);
    case 7: return pick<7, B>(log2l);
    case 8: return pick<8, B>(log2l);
    case 9: return pick<9, B>(log2l);
    case 10: return pick<10, B>(log2l);
    case 11: return B ? nullptr : pick<11, false>(log2l);
    case 12: return B ? nullptr : pick<12, false>(log2l);
    case 13: return B ? nullptr : pick<13, false>(log2l);
    case 14: return B ? nullptr : pick<14, false>(log2l);
    case 15: return B ? nullptr : pick<15, false>(log2l);
    case 16: return B ? nullptr : pick<16, false>(log2l);
    default: return nullptr;
  }
}

#define GM_CAT2(a, b) a##b
#define GM_CAT(a, b) GM_CAT2(a, b)

RuleKernelFn GM_CAT(rule_kernel_f, GM_RULE_FAMILY)(int d, int log2l, bool batch) {
  return batch ? rule_fn<true>(d, log2l) : rule_fn<false>(d, log2l);
}

GM_CHECK_UNIT_F(rule, GM_RULE_FAMILY)

}  // namespace gm
