// gm_corner.hpp -- node-sweep pieces shared by the fully symmetric rule
// kernels (degree 7, gm_rule.hip; degree 9, gm_rule9.hip): the binary-tree
// sweep of the 2^d corners (+-l5, .., +-l5) below a per-lane sign prefix, the
// lexicographic (i, j) pair index, the chain of centre terms that ends a node
// argument, and the fourth difference that picks the split axis (Sec. 2).
#pragma once

#include "gm_family.hpp"

namespace gm {

// ---------------------------------------------------------------------------
// Corner sweep: binary tree over coordinates D-U .. D-1 below a prefix.
// ---------------------------------------------------------------------------
// Arguments of the 2^M corners below prefix s over coordinates J .. J+M-1, in
// the tree's order (sign + before sign -); a chain that starts here (no
// prefix) starts with the family's corner bias.
template <int D, int FAM, int J, int M, bool HAS_PREFIX>
__device__ __forceinline__ void leaf_args(double s, const double (&t5p)[D], const double (&t5m)[D],
                                          double* out) {
  if constexpr (M == 0) {
    out[0] = s;
  } else {
    const double a = HAS_PREFIX ? Fam<FAM>::comb(s, t5p[J]) : Fam<FAM>::corner_first(t5p[J]);
    const double b = HAS_PREFIX ? Fam<FAM>::comb(s, t5m[J]) : Fam<FAM>::corner_first(t5m[J]);
    leaf_args<D, FAM, J + 1, M - 1, true>(a, t5p, t5m, out);
    leaf_args<D, FAM, J + 1, M - 1, true>(b, t5p, t5m, out + (1 << (M - 1)));
  }
}

// The last kLeafLog2 levels of the tree are evaluated together: their
// 2^kLeafLog2 outer functions run interleaved.
#ifndef GM_LEAF_LOG2
#define GM_LEAF_LOG2 2
#endif
constexpr int kLeafLog2 = GM_LEAF_LOG2;

template <int D, int FAM, int U, int K, bool HAS_PREFIX>
__device__ __forceinline__ void corner_tree(const DevParams& P, double s, const double (&t5p)[D],
                                            const double (&t5m)[D], double& local) {
  constexpr int LW = U < kLeafLog2 ? U : kLeafLog2;
  if constexpr (K == U - LW) {
    double a[1 << LW];
    leaf_args<D, FAM, D - U + K, LW, HAS_PREFIX>(s, t5p, t5m, a);
    Fam<FAM>::template accumulate_n<D, (1 << LW)>(P, a, local);
  } else {
    constexpr int j = D - U + K;
    if constexpr (!HAS_PREFIX && K == 0) {
      corner_tree<D, FAM, U, K + 1, true>(P, Fam<FAM>::corner_first(t5p[j]), t5p, t5m, local);
      corner_tree<D, FAM, U, K + 1, true>(P, Fam<FAM>::corner_first(t5m[j]), t5p, t5m, local);
    } else {
      corner_tree<D, FAM, U, K + 1, true>(P, Fam<FAM>::comb(s, t5p[j]), t5p, t5m, local);
      corner_tree<D, FAM, U, K + 1, true>(P, Fam<FAM>::comb(s, t5m[j]), t5p, t5m, local);
    }
  }
}

// Sweep the corners whose first LB coordinates have the signs given by
// `lane_bits` (bit j set -> -l5), i.e. 2^(D - LB) corners, into S5.
template <int D, int FAM, int LB>
__device__ __forceinline__ void corner_sweep(const DevParams& P, const double (&t5p)[D],
                                             const double (&t5m)[D], uint32_t lane_bits, KSum& S5) {
  constexpr int U = (D - LB) < 4 ? (D - LB) : 4;  // inner tree depth
  constexpr int NOUT = D - LB - U;                 // looped coordinates
  // lane prefix over coordinates 0 .. LB-1
  double pl = 0.0;
#pragma unroll
  for (int j = 0; j < LB; ++j) {
    const double t = ((lane_bits >> j) & 1u) ? t5m[j] : t5p[j];
    pl = (j == 0) ? Fam<FAM>::corner_first(t) : Fam<FAM>::comb(pl, t);
  }
  for (uint32_t m = 0; m < (1u << NOUT); ++m) {
    double pre = pl;
#pragma unroll
    for (int q = 0; q < NOUT; ++q) {
      constexpr int dummy = 0;
      (void)dummy;
      const int j = LB + q;
      const double t = ((m >> q) & 1u) ? t5m[j] : t5p[j];
      pre = (LB == 0 && q == 0) ? Fam<FAM>::corner_first(t) : Fam<FAM>::comb(pre, t);
    }
    double local = 0.0;
    corner_tree<D, FAM, U, 0, (LB + NOUT) != 0>(P, pre, t5p, t5m, local);
    ks_add(S5, local);
  }
}


// Fourth difference of axis i and the magnitude of the terms it cancels.
__device__ __forceinline__ void fourth_diff(const RuleConsts& K, double f0, double fp2, double fm2,
                                            double fp3, double fm3, double& Dv, double& sc) {
  const double A = (fp2 + fm2) - 2.0 * f0;
  const double B = (fp3 + fm3) - 2.0 * f0;
  Dv = fabs(A - B * K.r7);
  sc = (fabs(fp2) + fabs(fm2) + 2.0 * fabs(f0)) + K.r7 * (fabs(fp3) + fabs(fm3) + 2.0 * fabs(f0));
}

// The (i, j) pair with lexicographic index p, i < j < D.
template <int D>
__device__ __forceinline__ void pair_of(int p, int& i, int& j) {
  i = 0;
  int row = D - 1;
  while (p >= row) {
    p -= row;
    ++i;
    --row;
  }
  j = i + 1 + p;
}

template <int D, int FAM>
__device__ __forceinline__ double chain_tail(double s, const double* tc, int k0) {
  for (int k = k0; k < D; ++k) s = Fam<FAM>::comb(s, tc[k]);
  return s;
}

// s[q] (+) tc[k] for k = k0 .. k1 - 1 in order, for N chains at once, with the
// terms in registers: every index stays compile-time and the runtime bounds
// select which steps apply.
template <int D, int FAM, int N>
__device__ __forceinline__ void chain_from(double (&s)[N], const double (&tc)[D], int k0, int k1) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const bool on = k >= k0 && k < k1;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const double t = Fam<FAM>::comb(s[q], tc[k]);
      s[q] = on ? t : s[q];
    }
  }
}

}  // namespace gm
