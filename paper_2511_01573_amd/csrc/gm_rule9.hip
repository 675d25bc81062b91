// gm_rule9.hip -- the degree-9 rule kernel: the fully symmetric rule of degree
// 9 (the "9-order" reading of arXiv 2511.01573, Sec. 2) with the degree-7 and
// degree-5 Genz-Malik rules embedded in its nodes, its error estimate and the
// fourth-difference split axis, on every active region (Sec. 3 evaluate step).
//
// Rule (mean measure on [-1,1]^d, lambda^2 in brackets):
//   class 1  centre                                weight w9_1(d)
//   class 2  +-l2 e_i                 (9/70)       w9_2(d)
//   class 3  +-l3 e_i                 (9/10)       w9_3(d)
//   class 4  +-l4 e_i +- l4 e_j, i<j  (9/10)       w9_4(d)
//   class 5  (+-l5, .., +-l5)         (9/19)       w9_5 2^-d
//   class 6  +-l6 e_i                 (759/1190)   w9_6
//   class 7  +-l2 e_i +- l3 e_j, i != j            w9_7
//   class 8  +-l4 (e_i +- e_j +- e_k), i<j<k       w9_8
// (the weights are the unique solution of the even-moment equations of degree
// <= 8 for these generators).  Classes 1-5 with the degree-7 weights give Q7;
// with the degree-5 weights Q5; classes 1 and 3 with (1 - 10d/27, 5/27) give a
// degree-3 rule Q3.  err = vol |Q9 - Q7| (model 0), or the null-rule ratio
// test vol n1 min(1, 2 max(n1/n2, n2/n3)) with n1 = |Q9 - Q7|, n2 = |Q7 - Q5|,
// n3 = |Q5 - Q3| (model 1).  Split axis: the degree-7 rule's fourth
// differences of classes 2 and 3.
//
// Mapping: L = 2^rule9_log2l(d) lanes of one wavefront per region.  Lane s
// fixes the signs of the first log2 L corner coordinates and sweeps its
// 2^(d - log2 L) corners as a binary tree; the O(d^3) nodes of the other
// classes are dealt out as work items (an axis: its 6 nodes and its fourth
// difference; an axis pair: 4 class-4 and 8 class-7 nodes; an axis triple: 8
// class-8 nodes).  An item's nodes of one class are summed plainly and the
// sum enters the class's compensated total.  Every node argument is the
// left-to-right chain of the per-coordinate terms, as in the degree-7 kernel,
// so node values match the defining formula's evaluation order bitwise.
#include "gm_corner.hpp"

namespace gm {

template <int D>
struct R9Slot {
  double c[D], h[D], tc[D], pc[D], dv[D], sc[D];
  // per-coordinate terms at the perturbed positions: [0] +l2, [1] -l2,
  // [2] +l3 (= +l4), [3] -l3, [4] +l6, [5] -l6
  double tp[6][D];
};

// Work-item tables: the axis pairs (i, j) and triples (i, j, k), packed 4
// bits per index, ordered by their last index so that the lanes of a round
// run tail chains of about the same length.
template <int D>
struct ItemTable {
  uint16_t pair[D * (D - 1) / 2 + 1];
  uint16_t tri[D * (D - 1) * (D - 2) / 6 + 1];
};

template <int D>
constexpr ItemTable<D> make_items() {
  ItemTable<D> t{};
  int n = 0;
  for (int j = 1; j < D; ++j)
    for (int i = 0; i < j; ++i) t.pair[n++] = (uint16_t)(i | (j << 4));
  n = 0;
  for (int k = 2; k < D; ++k)
    for (int j = 1; j < k; ++j)
      for (int i = 0; i < j; ++i) t.tri[n++] = (uint16_t)(i | (j << 4) | (k << 8));
  return t;
}

template <int D>
__device__ constexpr ItemTable<D> kItems = make_items<D>();

// Extend N node arguments by the centre terms of coordinates k0 .. k1-1, in
// order (one loop for all N chains: each step is one LDS read and N (+)).
template <int FAM, int N>
__device__ __forceinline__ void chain_n(double (&x)[N], const double* tc, int k0, int k1) {
  for (int k = k0; k < k1; ++k) {
    const double t = tc[k];
#pragma unroll
    for (int q = 0; q < N; ++q) x[q] = Fam<FAM>::comb(x[q], t);
  }
}

// Three wavefronts per SIMD up to d = 10 (at most a few values spill to
// scratch, and the extra wavefront hides more latency); two above, where the
// spill would grow.
template <int D, int FAM, int LOG2L, bool BATCH>
__global__ __launch_bounds__(kRuleBlock) __attribute__((amdgpu_waves_per_eu(D <= 10 ? 3 : 2)))
void rule9_kernel(RuleArgs A) {
  using F = Fam<FAM>;
  constexpr int L = 1 << LOG2L;
  constexpr int RPB = kRuleBlock / L;  // regions per block step
  constexpr int NPAIR = D * (D - 1) / 2;
  constexpr int NTRI = D * (D - 1) * (D - 2) / 6;
  static_assert(LOG2L <= D && LOG2L <= 6, "at least one corner and one wavefront per region");
  __shared__ R9Slot<D> slots[RPB];
  int64_t start, n;
  int buf;
  if (!active_range<BATCH>(A, start, n, buf)) return;
  const RegionSrc R = region_src<BATCH>(A, buf);
  const RuleConsts& K = A.K;
  const int g = threadIdx.x >> LOG2L;  // region slot in the block
  const int s = threadIdx.x & (L - 1);
  R9Slot<D>& sl = slots[g];
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
    double pc = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if ((k & (L - 1)) == s) {
        sl.tc[k] = tc[k];
        sl.pc[k] = pc;
        sl.tp[0][k] = F::term(P, k, fma(K.lam2, h[k], c[k]));
        sl.tp[1][k] = F::term(P, k, fma(-K.lam2, h[k], c[k]));
        sl.tp[2][k] = F::term(P, k, fma(K.lam3, h[k], c[k]));
        sl.tp[3][k] = F::term(P, k, fma(-K.lam3, h[k], c[k]));
        sl.tp[4][k] = F::term(P, k, fma(K.lam6, h[k], c[k]));
        sl.tp[5][k] = F::term(P, k, fma(-K.lam6, h[k], c[k]));
      }
      pc = (k == 0) ? tc[0] : F::comb(pc, tc[k]);
    }
    __syncthreads();
    const double f0 = F::template outer<D>(P, pc);
    KSum S2 = {0.0, 0.0}, S3 = {0.0, 0.0}, S4 = {0.0, 0.0}, S5 = {0.0, 0.0};
    KSum S6 = {0.0, 0.0}, S7 = {0.0, 0.0}, S8 = {0.0, 0.0};
    // The three node groups run one after the other, so the lanes of a
    // wavefront stay on the same code path.
    // Axes: +-l2, +-l3, +-l6 along axis i and its fourth difference.
    for (int i = s; i < D; i += L) {
      const double v[6] = {sl.tp[0][i], sl.tp[1][i], sl.tp[2][i],
                           sl.tp[3][i], sl.tp[4][i], sl.tp[5][i]};
      const double pci = sl.pc[i];
      double x[6], f[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) x[q] = (i == 0) ? v[q] : F::comb(pci, v[q]);
      chain_n<FAM, 6>(x, sl.tc, i + 1, D);
      F::template outer_n<D, 6>(P, x, f);
      ks_add(S2, f[0] + f[1]);
      ks_add(S3, f[2] + f[3]);
      ks_add(S6, f[4] + f[5]);
      double dv, scv;
      fourth_diff(K, f0, f[0], f[1], f[2], f[3], dv, scv);
      sl.dv[i] = dv;
      sl.sc[i] = scv;
    }
    // Axis pairs i < j: class 4 (+-l4, +-l4) and class 7 in both orders.
    for (int it = s; it < NPAIR; it += L) {
      const int pk = kItems<D>.pair[it];
      const int i = pk & 15, j = pk >> 4;
      // x_i at +l3, -l3 (= +-l4), +l2, -l2
      const double ti[4] = {sl.tp[2][i], sl.tp[3][i], sl.tp[0][i], sl.tp[1][i]};
      const double tj3[2] = {sl.tp[2][j], sl.tp[3][j]};
      const double tj2[2] = {sl.tp[0][j], sl.tp[1][j]};
      const double pci = sl.pc[i];
      double m[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) m[a] = (i == 0) ? ti[a] : F::comb(pci, ti[a]);
      chain_n<FAM, 4>(m, sl.tc, i + 1, j);
      // x[0..4): (+-l4 on i, +-l4 on j), class 4; x[4..12): (+-l3 on i, +-l2 on
      // j) and (+-l2 on i, +-l3 on j), class 7
      double x[12], f[12];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          x[2 * a + sj] = F::comb(m[a], tj3[sj]);
          x[4 + 2 * a + sj] = F::comb(m[a], tj2[sj]);
          x[8 + 2 * a + sj] = F::comb(m[2 + a], tj3[sj]);
        }
      }
      chain_n<FAM, 12>(x, sl.tc, j + 1, D);
      F::template outer_n<D, 12>(P, x, f);
      ks_add(S4, (f[0] + f[1]) + (f[2] + f[3]));
      ks_add(S7, ((f[4] + f[5]) + (f[6] + f[7])) + ((f[8] + f[9]) + (f[10] + f[11])));
    }
    // Axis triples i < j < k: class 8.
    for (int it = s; it < NTRI; it += L) {
      const int tk3 = kItems<D>.tri[it];
      const int i = tk3 & 15, j = (tk3 >> 4) & 15, k = tk3 >> 8;
      const double ti[2] = {sl.tp[2][i], sl.tp[3][i]};
      const double tj[2] = {sl.tp[2][j], sl.tp[3][j]};
      const double tk[2] = {sl.tp[2][k], sl.tp[3][k]};
      const double pci = sl.pc[i];
      double m1[2], m2[4], x8[8], f8[8];
#pragma unroll
      for (int a = 0; a < 2; ++a) m1[a] = (i == 0) ? ti[a] : F::comb(pci, ti[a]);
      chain_n<FAM, 2>(m1, sl.tc, i + 1, j);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) m2[2 * a + b] = F::comb(m1[a], tj[b]);
      }
      chain_n<FAM, 4>(m2, sl.tc, j + 1, k);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int e = 0; e < 2; ++e) x8[2 * q + e] = F::comb(m2[q], tk[e]);
      }
      chain_n<FAM, 8>(x8, sl.tc, k + 1, D);
      F::template outer_n<D, 8>(P, x8, f8);
      ks_add(S8, ((f8[0] + f8[1]) + (f8[2] + f8[3])) + ((f8[4] + f8[5]) + (f8[6] + f8[7])));
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
    // Combine the L lanes of the region: each lane's compensated class sums
    // are rounded once and added across the lanes in a butterfly (a + b and
    // b + a round alike, so every lane ends with the same totals).
    double T[7] = {ks_val(S2), ks_val(S3), ks_val(S4), ks_val(S5),
                   ks_val(S6), ks_val(S7), ks_val(S8)};
#pragma unroll
    for (int m = L / 2; m >= 1; m >>= 1) {
#pragma unroll
      for (int q = 0; q < 7; ++q) T[q] = T[q] + __shfl_xor(T[q], m, 64);
    }
    __syncthreads();
    if (s == 0 && valid) {
      const double vol = ldexp(volo, -lvl);
      const double S[8] = {f0, T[0], T[1], T[2], T[3], T[4], T[5], T[6]};
      RegionResult o;
      o.nonfinite = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) o.nonfinite |= !isfinite(S[q]);
      double q9 = K.w9[0] * S[0];
      double n1 = K.e9[0] * S[0];
#pragma unroll
      for (int q = 1; q < 8; ++q) {
        q9 = q9 + K.w9[q] * S[q];
        n1 = n1 + K.e9[q] * S[q];
      }
      n1 = fabs(n1);
      double q7 = K.w[0] * S[0];
      double d75 = K.e[0] * S[0];
#pragma unroll
      for (int q = 1; q < 5; ++q) {
        q7 = q7 + K.w[q] * S[q];
        d75 = d75 + K.e[q] * S[q];
      }
      const double n2 = fabs(d75);
      const double q5 = q7 - d75;
      const double q3 = K.q3[0] * S[0] + K.q3[1] * S[2];
      const double n3 = fabs(q5 - q3);
      o.q = vol * q9;
      o.err = K.err_model ? vol * (n1 * fmin(1.0, 2.0 * fmax(n1 / n2, n2 / n3))) : vol * n1;
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

#ifndef GM_RULE_FAMILY
#error "gm_rule9.hip is compiled once per integrand family (-DGM_RULE_FAMILY=k)"
#endif

#define GM_R9_CAT2(a, b) a##b
#define GM_R9_CAT(a, b) GM_R9_CAT2(a, b)

template <int D>
static RuleKernelFn r9_pick(bool batch, bool wide) {
  if constexpr (D <= kBatchMaxDim) {
    if (batch) return rule9_kernel<D, GM_RULE_FAMILY, rule9_log2l(D), true>;
  } else {
    if (batch) return nullptr;
  }
  if (wide) return rule9_kernel<D, GM_RULE_FAMILY, rule9_log2l_wide(D), false>;
  return rule9_kernel<D, GM_RULE_FAMILY, rule9_log2l(D), false>;
}

RuleKernelFn GM_R9_CAT(rule9_kernel_f, GM_RULE_FAMILY)(int d, bool batch, bool wide) {
  switch (d) {
    case 2: return r9_pick<2>(batch, wide);
    case 3: return r9_pick<3>(batch, wide);
    case 4: return r9_pick<4>(batch, wide);
    case 5: return r9_pick<5>(batch, wide);
    case 6: return r9_pick<6>(batch, wide);
    case 7: return r9_pick<7>(batch, wide);
    case 8: return r9_pick<8>(batch, wide);
    case 9: return r9_pick<9>(batch, wide);
    case 10: return r9_pick<10>(batch, wide);
    case 11: return r9_pick<11>(batch, wide);
    case 12: return r9_pick<12>(batch, wide);
    case 13: return r9_pick<13>(batch, wide);
    case 14: return r9_pick<14>(batch, wide);
    case 15: return r9_pick<15>(batch, wide);
    case 16: return r9_pick<16>(batch, wide);
    default: return nullptr;
  }
}

GM_CHECK_UNIT_F(rule9, GM_RULE_FAMILY)

}  // namespace gm
