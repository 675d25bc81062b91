// gm_family.hpp -- device pieces shared by the rule kernels (Genz-Malik,
// gm_rule.hip; tensor-product Gauss-Kronrod, gm_gk.hip): the integrand families
// of Sec. 4 split as f(x) = G(T_0(x_0) (+) ... (+) T_{d-1}(x_{d-1})), compensated
// accumulation, and the per-region result / per-block partial plumbing.
#pragma once

#include "gm_common.hpp"
#include "gm_math.hpp"

namespace gm {

constexpr int kRuleBlock = kRuleBlockSize;

// ---------------------------------------------------------------------------
// Family traits: term, combination and outer function (Sec. 4 integrands).
// ---------------------------------------------------------------------------
template <int FAM>
struct Fam {
  static constexpr bool kProduct = (FAM == kProductPeak);
  __device__ static __forceinline__ double term(const DevParams& P, int j, double x) {
    if constexpr (FAM == kOsc || FAM == kCornerPeak) {
      return P.a[j] * x;
    } else if constexpr (FAM == kProductPeak) {
      // the per-axis factor itself, so a node costs only the chain of products
      const double t = x - P.u[j];
      return fm::rcp(P.inv_a2[j] + t * t);
    } else if constexpr (FAM == kGaussian) {
      const double t = P.a[j] * (x - P.u[j]);
      return t * t;
    } else if constexpr (FAM == kC0) {
      return P.a[j] * fabs(x - P.u[j]);
    } else if constexpr (FAM == kDiscontinuous) {
      // outside the box x_j <= u_j the sum becomes -inf and G gives 0
      return (x > P.u[j]) ? -__builtin_inf() : P.a[j] * x;
    } else {
      return x * x;
    }
  }
  __device__ static __forceinline__ double comb(double s, double t) {
    if constexpr (kProduct) return s * t;
    else return s + t;
  }
  // The oscillatory family's cos is reduced by pi/2 in double-double steps that
  // stay accurate while |argument| < 2^48; a region whose nodes could exceed that
  // bound is reported as non-finite instead of evaluated inaccurately.
  template <int D>
  __device__ static __forceinline__ bool in_range(const DevParams& P, const double (&c)[D],
                                                  const double (&h)[D]) {
    if constexpr (FAM == kOsc) {
      double b = fabs(P.c0);
#pragma unroll
      for (int j = 0; j < D; ++j) b += fabs(P.a[j]) * (fabs(c[j]) + h[j]);
      return b < 0x1p48;
    } else {
      return true;
    }
  }
  __device__ static __forceinline__ bool in_range_rt(const DevParams& P, int d, const double* c,
                                                     const double* h) {
    if constexpr (FAM == kOsc) {
      double b = fabs(P.c0);
      for (int j = 0; j < d; ++j) b += fabs(P.a[j]) * (fabs(c[j]) + h[j]);
      return b < 0x1p48;
    } else {
      return true;
    }
  }
  // (1 + s)^-(d+1) needs (1 + s)^(d+1): binary powering
  template <int D>
  __device__ static __forceinline__ double cpk_power(double s) {
    return cpk_power_of_base<D>(1.0 + s);
  }
  template <int D>
  __device__ static __forceinline__ double cpk_power_of_base(double b) {
    double y = 1.0, p = b;
    int e = D + 1;
    bool first = true;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      if (e & 1) {
        y = first ? p : y * p;
        first = false;
      }
      e >>= 1;
      if (e) p = p * p;
    }
    return y;
  }
  // The outer function G of f = G(s) on N independent arguments at once.
  template <int D, int N>
  __device__ static __forceinline__ void outer_n(const DevParams& P, const double (&s)[N],
                                                 double (&f)[N]) {
    double a[N];
    if constexpr (FAM == kOsc) {
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = P.c0 + s[i];
      fm::cos_n<N>(a, f);
    } else if constexpr (FAM == kProductPeak) {
#pragma unroll
      for (int i = 0; i < N; ++i) f[i] = s[i];
    } else if constexpr (FAM == kCornerPeak) {
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = cpk_power<D>(s[i]);
      fm::rcp_n<N>(a, f);
    } else if constexpr (FAM == kGaussian || FAM == kC0) {
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = -s[i];
      fm::exp_n<N>(a, f);
    } else if constexpr (FAM == kDiscontinuous) {
      fm::exp_n<N>(s, f);
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double s2 = s[i] * s[i];
        const double s4 = s2 * s2;
        const double s8 = s4 * s4;
        f[i] = (s8 * s2) * s[i];
      }
    }
  }
  // Constant the corner sweep folds into the first term of each corner
  // argument (once per subtree instead of once per corner): the corner peak's
  // 1 of 1 + sum a_j x_j.
  static constexpr bool kCornerBias = (FAM == kCornerPeak);
  __device__ static __forceinline__ double corner_first(double t) {
    if constexpr (kCornerBias) return 1.0 + t;
    else return t;
  }
  // local + G(s[0]) + ... + G(s[N-1]), added in that order (the corner sweep's
  // sum; s[i] carries the corner bias, so the corner peak's base 1 + sum a_j x_j
  // arrives formed).
  template <int D, int N>
  __device__ static __forceinline__ void accumulate_n(const DevParams& P, const double (&s)[N],
                                                     double& local) {
    if constexpr (FAM == kCornerPeak) {
      double a[N], f[N];
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = cpk_power_of_base<D>(s[i]);
      fm::rcp_n<N>(a, f);
#pragma unroll
      for (int i = 0; i < N; ++i) local += f[i];
    } else {
      double f[N];
      outer_n<D, N>(P, s, f);
#pragma unroll
      for (int i = 0; i < N; ++i) local += f[i];
    }
  }
  template <int D>
  __device__ static __forceinline__ double outer(const DevParams& P, double s) {
    const double a[1] = {s};
    double f[1];
    outer_n<D, 1>(P, a, f);
    return f[0];
  }
};

struct KSum {
  double s, c;
};
__device__ __forceinline__ void ks_add(KSum& k, double x) {
  double t, e;
  two_sum(k.s, x, t, e);
  k.s = t;
  k.c += e;
}
__device__ __forceinline__ double ks_val(const KSum& k) { return k.s + k.c; }
__device__ __forceinline__ KSum ks_merge(KSum a, KSum b) {
  double t, e;
  two_sum(a.s, b.s, t, e);
  a.s = t;
  a.c += e + b.c;
  return a;
}
__device__ __forceinline__ KSum shfl_xor_ks(KSum v, int m) {
  KSum r;
  r.s = __shfl_xor(v.s, m, 64);
  r.c = __shfl_xor(v.c, m, 64);
  return r;
}

struct RegionResult {
  double q, err;
  int axis;
  int geo;
  int nonfinite;
};

__device__ __forceinline__ void store_result(const RuleArgs& A, int64_t r, const RegionResult& o) {
  if (!GM_INB(r, A.cap)) return;
  A.Q[r] = o.q;
  A.ERR[r] = o.err;
  A.AXIS[r] = (uint8_t)(o.axis | (o.nonfinite ? kNonfiniteBit : 0) | (o.geo ? kGeoBit : 0));
}

__device__ __forceinline__ void block_partials(const RuleArgs& A, dd qs, dd es, int nonfin) {
  __shared__ dd sq[kRuleBlock / 64], se[kRuleBlock / 64];
  __shared__ int snf[kRuleBlock / 64];
  qs = wave_sum_dd(qs);
  es = wave_sum_dd(es);
  const int anynf = __any(nonfin);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sq[w] = qs;
    se[w] = es;
    snf[w] = anynf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    dd tq = sq[0], te = se[0];
    int nf = snf[0];
    for (int k = 1; k < kRuleBlock / 64; ++k) {
      tq = dd_sum(tq, sq[k]);
      te = dd_sum(te, se[k]);
      nf |= snf[k];
    }
    double* p = A.partials + 4 * (int64_t)blockIdx.x;
    p[0] = tq.hi;
    p[1] = tq.lo;
    p[2] = te.hi;
    p[3] = te.lo;
    if (nf && A.n_fixed < 0) atomicOr(&A.st->nonfinite, 1);
  }
}

// Regions [start, end) of the store buffer `buf` this launch evaluates.
template <bool BATCH>
__device__ __forceinline__ bool active_range(const RuleArgs& A, int64_t& start, int64_t& end,
                                             int& buf) {
  if constexpr (BATCH) {
    start = A.grp[0];
    end = A.grp[1];
    buf = *A.bbuf;
    return end > start;
  }
  start = 0;
  if (A.n_fixed >= 0) {
    end = A.n_fixed;
    buf = 0;
    return true;
  }
  if (A.st->done) return false;
  end = A.st->n_active;
  buf = A.st->buf;
  return true;
}

// How the launch's regions are stored (batch stores and region lists hold
// the regions themselves).
template <bool BATCH>
__device__ __forceinline__ RegionSrc region_src(const RuleArgs& A, int buf) {
  RegionSrc R{A.C[buf], A.H[buf], A.L[buf], nullptr, A.cap, 0, 0};
  if constexpr (!BATCH) {
    if (A.n_fixed < 0 && A.st->split) {
      R.split = 1;
      R.npar = A.st->n_par;
      R.PAX = A.PAX[buf];
    }
  }
  return R;
}

template <bool BATCH>
__device__ __forceinline__ const DevParams& region_params(const RuleArgs& A, int buf, int64_t r,
                                                         double& vol_omega) {
  if constexpr (BATCH) {
    const uint32_t item = A.IT[buf][r];
    vol_omega = A.VOL[item];
    return A.PARAMS[item];
  } else {
    vol_omega = A.vol_omega;
    return A.P;
  }
}

}  // namespace gm
