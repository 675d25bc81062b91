// gm_adjoint.hip -- adjoint kernel of the gradient mode: the derivative of
// the fixed-tree quadrature with respect to (a, u), for the degree-7
// Genz-Malik rule or the degree-9 rule (its classes 6-8 added to the visit).
//
// The forward run (Sec. 3 loop) retains every retired region; together with
// the last evaluated active set they form the frozen tree whose rule values
// sum to the estimate.  The adjoint kernel evaluates
//     dI/dtheta = sum_leaves vol * sum_nodes w_class * df/dtheta(x_node)
// with the nodes and weights of the rule kernel (Sec. 2).  Per family the
// node derivative is accumulated in factored form (e.g. the Gaussian keeps
// sum w f (x_j - u_j)^2 and sum w f (x_j - u_j) per axis) and scaled once.
//
// Corner class.  Every family's node contribution is phi(s(x)) psi_j(x_j):
// phi a function of the node's argument s (a left-to-right chain of
// per-coordinate terms, as in the rule kernel) and psi_j a function of x_j
// alone.  A corner's x_j is c_j + l5 h_j or c_j - l5 h_j, so the corner sum
// of phi psi_j is psi_j(+) Phi_j^+ + psi_j(-) Phi_j^-, with Phi_j^+- the sums
// of phi over the corners on either side of axis j.  The corners are swept
// as a binary prefix tree over the per-coordinate terms (the last levels
// unrolled, the leading axes' sign patterns looped over), and each tree node
// adds its subtree's phi sum to Phi of its axis and side.
#include "gm_adjoint.hpp"

namespace gm {


// Per-node accumulation: acc[0..D) and acc[D..2D) are the family's factored
// sums; finish() turns them into dI/da_j and dI/du_j.
template <int D, int FAM>
__device__ __forceinline__ void adj_node(const DevParams& P, const double (&x)[D], double w,
                                         double (&acc)[2 * D]) {
  if constexpr (FAM == kOsc) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s = s + P.a[j] * x[j];
    const double ws = w * sin(P.c0 + s);
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = fma(ws, x[j], acc[j]);
    acc[D] += ws;
  } else if constexpr (FAM == kProductPeak) {
    double den[D];
    double prod = 1.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double t = x[j] - P.u[j];
      den[j] = P.inv_a2[j] + t * t;
      prod = prod * den[j];
    }
    const double wf = w / prod;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double r = wf / den[j];
      acc[j] += r;
      acc[D + j] = fma(r, x[j] - P.u[j], acc[D + j]);
    }
  } else if constexpr (FAM == kCornerPeak) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s = s + P.a[j] * x[j];
    const double b = 1.0 + s;
    const double g = w * pow(b, -(double)(D + 2));
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = fma(g, x[j], acc[j]);
  } else if constexpr (FAM == kGaussian) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double t = P.a[j] * (x[j] - P.u[j]);
      s = s + t * t;
    }
    const double wf = w * exp(-s);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double t = x[j] - P.u[j];
      const double wft = wf * t;
      acc[j] = fma(wft, t, acc[j]);
      acc[D + j] += wft;
    }
  } else if constexpr (FAM == kC0) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s = s + P.a[j] * fabs(x[j] - P.u[j]);
    const double wf = w * exp(-s);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double t = x[j] - P.u[j];
      acc[j] = fma(wf, fabs(t), acc[j]);
      acc[D + j] += (t > 0.0) ? wf : ((t < 0.0) ? -wf : 0.0);
    }
  } else if constexpr (FAM == kDiscontinuous) {
    bool out = false;
#pragma unroll
    for (int j = 0; j < D; ++j) out = out || (x[j] > P.u[j]);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s = s + P.a[j] * x[j];
    const double wf = out ? 0.0 : w * exp(s);
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = fma(wf, x[j], acc[j]);
  }
}

// Scale the factored sums of one region into (dI/da, dI/du) contributions.
template <int D, int FAM>
__device__ __forceinline__ void adj_finish(const DevParams& P, double vol, const double (&acc)[2 * D],
                                           double (&g)[2 * D]) {
#pragma unroll
  for (int j = 0; j < 2 * D; ++j) g[j] = 0.0;
  if constexpr (FAM == kOsc) {
#pragma unroll
    for (int j = 0; j < D; ++j) g[j] = -vol * acc[j];
    g[D] = -vol * (6.283185307179586476925286766559 * acc[D]);
  } else if constexpr (FAM == kProductPeak) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      g[j] = vol * (2.0 * acc[j] / (P.a[j] * P.a[j] * P.a[j]));
      g[D + j] = vol * (2.0 * acc[D + j]);
    }
  } else if constexpr (FAM == kCornerPeak) {
#pragma unroll
    for (int j = 0; j < D; ++j) g[j] = -vol * ((double)(D + 1) * acc[j]);
  } else if constexpr (FAM == kGaussian) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      g[j] = -vol * (2.0 * P.a[j] * acc[j]);
      g[D + j] = vol * (2.0 * P.a[j] * P.a[j] * acc[D + j]);
    }
  } else if constexpr (FAM == kC0) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      g[j] = -vol * acc[j];
      g[D + j] = vol * (P.a[j] * acc[D + j]);
    }
  } else if constexpr (FAM == kDiscontinuous) {
#pragma unroll
    for (int j = 0; j < D; ++j) g[j] = vol * acc[j];
  }
}

// Visit every node of region (c, h) in the rule's class order, calling
// fn(class_weight_index, x).
template <int D, bool CORNERS = true, typename Fn>
__device__ __forceinline__ void visit_nodes(const RuleConsts& K, const double (&c)[D],
                                            const double (&h)[D], Fn&& fn) {
  double x[D];
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = c[k];
  fn(0, x);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    x[i] = fma(K.lam2, h[i], c[i]);
    fn(1, x);
    x[i] = fma(-K.lam2, h[i], c[i]);
    fn(1, x);
    x[i] = fma(K.lam3, h[i], c[i]);
    fn(2, x);
    x[i] = fma(-K.lam3, h[i], c[i]);
    fn(2, x);
    x[i] = c[i];
  }
  for (int i = 0; i < D - 1; ++i) {
    for (int j = i + 1; j < D; ++j) {
      for (int sg = 0; sg < 4; ++sg) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const double si = (sg & 2) ? -K.lam4 : K.lam4;
          const double sj = (sg & 1) ? -K.lam4 : K.lam4;
          x[k] = (k == i) ? fma(si, h[k], c[k]) : ((k == j) ? fma(sj, h[k], c[k]) : c[k]);
        }
        fn(3, x);
      }
    }
  }
  if constexpr (!CORNERS) return;
  double xp[D], xm[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    xp[k] = fma(K.lam5, h[k], c[k]);
    xm[k] = fma(-K.lam5, h[k], c[k]);
  }
  for (uint32_t b = 0; b < (1u << D); ++b) {
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = ((b >> k) & 1u) ? xm[k] : xp[k];
    fn(4, x);
  }
}

// The degree-9 rule's further classes, in its order: +-l6 e_i (weight index
// 5), +-l2 e_i +- l3 e_j for ordered pairs i != j (6), +-l4 (e_i +- e_j +- e_k)
// for i < j < k (7).
template <int D, typename Fn>
__device__ __forceinline__ void visit_nodes9_extra(const RuleConsts& K, const double (&c)[D],
                                                   const double (&h)[D], Fn&& fn) {
  double x[D];
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = c[k];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    x[i] = fma(K.lam6, h[i], c[i]);
    fn(5, x);
    x[i] = fma(-K.lam6, h[i], c[i]);
    fn(5, x);
    x[i] = c[i];
  }
  for (int i = 0; i < D; ++i) {
    for (int j = 0; j < D; ++j) {
      if (j == i) continue;
      for (int sg = 0; sg < 4; ++sg) {
        const double si = (sg & 2) ? -K.lam2 : K.lam2;
        const double sj = (sg & 1) ? -K.lam3 : K.lam3;
#pragma unroll
        for (int k = 0; k < D; ++k)
          x[k] = (k == i) ? fma(si, h[k], c[k]) : ((k == j) ? fma(sj, h[k], c[k]) : c[k]);
        fn(6, x);
      }
    }
  }
  for (int i = 0; i < D - 2; ++i) {
    for (int j = i + 1; j < D - 1; ++j) {
      for (int l = j + 1; l < D; ++l) {
        for (int sg = 0; sg < 8; ++sg) {
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const double sk = (k == i)   ? ((sg & 1) ? -K.lam4 : K.lam4)
                              : (k == j) ? ((sg & 2) ? -K.lam4 : K.lam4)
                                         : ((sg & 4) ? -K.lam4 : K.lam4);
            x[k] = (k == i || k == j || k == l) ? fma(sk, h[k], c[k]) : c[k];
          }
          fn(7, x);
        }
      }
    }
  }
}

// b^E for a compile-time E >= 1 by binary powering (E <= 18 here: at most
// five multiplications, a few ulp).
template <int E>
__device__ __forceinline__ double ipow(double b) {
  double y = 1.0, p = b;
  bool first = true;
#pragma unroll
  for (int e = E; e > 0; e >>= 1) {
    if (e & 1) {
      y = first ? p : y * p;
      first = false;
    }
    if (e > 1) p = p * p;
  }
  return y;
}

// Per-family split of a node's contribution into phi(s) and psi_j(x_j)
// (the same quantities adj_node accumulates, without the class weight).
template <int FAM>
struct AdjSplit {
  // the empty chain: comb(kEmpty, t) == t exactly
  static constexpr double kEmpty = (FAM == kProductPeak) ? 1.0 : 0.0;
  // per-coordinate term of the argument and its combination
  __device__ static __forceinline__ double term(const DevParams& P, int j, double x) {
    if constexpr (FAM == kOsc || FAM == kCornerPeak) {
      return P.a[j] * x;
    } else if constexpr (FAM == kProductPeak) {
      const double t = x - P.u[j];
      return 1.0 / (P.inv_a2[j] + t * t);
    } else if constexpr (FAM == kGaussian) {
      const double t = P.a[j] * (x - P.u[j]);
      return t * t;
    } else if constexpr (FAM == kC0) {
      return P.a[j] * fabs(x - P.u[j]);
    } else {
      return (x > P.u[j]) ? -__builtin_inf() : P.a[j] * x;
    }
  }
  __device__ static __forceinline__ double comb(double s, double t) {
    if constexpr (FAM == kProductPeak) return s * t;
    else return s + t;
  }
  template <int D>
  __device__ static __forceinline__ double phi(const DevParams& P, double s) {
    if constexpr (FAM == kOsc) return sin(P.c0 + s);
    else if constexpr (FAM == kProductPeak) return s;
    else if constexpr (FAM == kCornerPeak) return 1.0 / ipow<D + 2>(1.0 + s);
    else if constexpr (FAM == kGaussian || FAM == kC0) return exp(-s);
    else return exp(s);  // the discontinuous family: exp(-inf) = 0 outside its box
  }
  // add w (psi(+) Phi^+ + psi(-) Phi^-) for axis j into the factored sums
  template <int D>
  __device__ static __forceinline__ void add_axis(const DevParams& P, int j, double xp, double xm,
                                                  double wp, double wm, double (&acc)[2 * D]) {
    if constexpr (FAM == kOsc || FAM == kCornerPeak || FAM == kDiscontinuous) {
      acc[j] = fma(wp, xp, fma(wm, xm, acc[j]));
    } else if constexpr (FAM == kProductPeak) {
      const double tp = xp - P.u[j], tm = xm - P.u[j];
      const double rp = wp / (P.inv_a2[j] + tp * tp), rm = wm / (P.inv_a2[j] + tm * tm);
      acc[j] += rp + rm;
      acc[D + j] = fma(rp, tp, fma(rm, tm, acc[D + j]));
    } else if constexpr (FAM == kGaussian) {
      const double tp = xp - P.u[j], tm = xm - P.u[j];
      acc[j] = fma(wp * tp, tp, fma(wm * tm, tm, acc[j]));
      acc[D + j] = fma(wp, tp, fma(wm, tm, acc[D + j]));
    } else {
      const double tp = xp - P.u[j], tm = xm - P.u[j];
      acc[j] = fma(wp, fabs(tp), fma(wm, fabs(tm), acc[j]));
      const double sp = (tp > 0.0) ? wp : ((tp < 0.0) ? -wp : 0.0);
      const double sm = (tm > 0.0) ? wm : ((tm < 0.0) ? -wm : 0.0);
      acc[D + j] += sp + sm;
    }
  }
};

// Unrolled subtree over axes J .. D-1 below the prefix s: returns its phi
// sum and adds each level's two halves to Phi^+ / Phi^- of that axis.
template <int D, int FAM, int J>
__device__ __forceinline__ double adj_corner_tree(const DevParams& P, double s,
                                                  const double (&tp)[D], const double (&tm)[D],
                                                  double (&fp)[D], double (&fm_)[D]) {
  using S = AdjSplit<FAM>;
  if constexpr (J == D) {
    return S::template phi<D>(P, s);
  } else {
    const double a = adj_corner_tree<D, FAM, J + 1>(P, S::comb(s, tp[J]), tp, tm, fp, fm_);
    const double b = adj_corner_tree<D, FAM, J + 1>(P, S::comb(s, tm[J]), tp, tm, fp, fm_);
    fp[J] += a;
    fm_[J] += b;
    return a + b;
  }
}

// The corner class (weight w) of region (c, h) added into acc.
template <int D, int FAM>
__device__ __forceinline__ void adj_corners(const DevParams& P, const RuleConsts& K, double w,
                                            const double (&c)[D], const double (&h)[D],
                                            double (&acc)[2 * D]) {
  using S = AdjSplit<FAM>;
  constexpr int U = D < 4 ? D : 4;  // unrolled levels
  constexpr int H = D - U;          // looped leading axes
  double xp[D], xm[D], tp[D], tm[D], fp[D], fm_[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    xp[j] = fma(K.lam5, h[j], c[j]);
    xm[j] = fma(-K.lam5, h[j], c[j]);
    tp[j] = S::term(P, j, xp[j]);
    tm[j] = S::term(P, j, xm[j]);
    fp[j] = 0.0;
    fm_[j] = 0.0;
  }
  for (uint32_t hb = 0; hb < (1u << H); ++hb) {
    double sum;
    if constexpr (H == 0) {
      sum = adj_corner_tree<D, FAM, 0>(P, S::kEmpty, tp, tm, fp, fm_);
    } else {
      // bit k of hb: the minus side on axis k (the corner order of the rule)
      double s = ((hb & 1u) ? tm[0] : tp[0]);
#pragma unroll
      for (int k = 1; k < H; ++k) s = S::comb(s, ((hb >> k) & 1u) ? tm[k] : tp[k]);
      sum = adj_corner_tree<D, FAM, H>(P, s, tp, tm, fp, fm_);
#pragma unroll
      for (int k = 0; k < H; ++k) {
        if ((hb >> k) & 1u) fm_[k] += sum;
        else fp[k] += sum;
      }
    }
    if constexpr (FAM == kOsc) acc[D] = fma(w, sum, acc[D]);
  }
#pragma unroll
  for (int j = 0; j < D; ++j) S::template add_axis<D>(P, j, xp[j], xm[j], w * fp[j], w * fm_[j], acc);
}

template <int D, int FAM, bool R9>
__global__ __launch_bounds__(kAdjBlock) void adjoint_kernel(AdjArgs A) {
  dd tot[2 * D];
#pragma unroll
  for (int j = 0; j < 2 * D; ++j) tot[j] = dd{0.0, 0.0};
  for (int64_t r = (int64_t)blockIdx.x * kAdjBlock + threadIdx.x; r < A.n;
       r += (int64_t)gridDim.x * kAdjBlock) {
    double c[D], h[D];
    const int lvl = load_region<D>(A.R, r, c, h);
    const double vol = ldexp(A.vol_omega, -lvl);
    double acc[2 * D];
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) acc[j] = 0.0;
    if constexpr (R9) {
      visit_nodes<D, false>(A.K, c, h, [&](int cls, const double (&x)[D]) {
        adj_node<D, FAM>(A.P, x, A.K.w9[cls], acc);
      });
      adj_corners<D, FAM>(A.P, A.K, A.K.w9[4], c, h, acc);
      visit_nodes9_extra<D>(A.K, c, h, [&](int cls, const double (&x)[D]) {
        adj_node<D, FAM>(A.P, x, A.K.w9[cls], acc);
      });
    } else {
      visit_nodes<D, false>(A.K, c, h, [&](int cls, const double (&x)[D]) {
        adj_node<D, FAM>(A.P, x, A.K.w[cls], acc);
      });
      adj_corners<D, FAM>(A.P, A.K, A.K.w[4], c, h, acc);
    }
    double g[2 * D];
    adj_finish<D, FAM>(A.P, vol, acc, g);
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) dd_add(tot[j], g[j]);
  }
  __shared__ dd sh[kAdjBlock / 64][2 * D];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 2 * D; ++j) {
    const dd v = wave_sum_dd(tot[j]);
    if ((threadIdx.x & 63) == 0) sh[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < 2 * D) {
    dd v = sh[0][threadIdx.x];
    for (int k = 1; k < kAdjBlock / 64; ++k) v = dd_sum(v, sh[k][threadIdx.x]);
    double* p = A.partials + ((int64_t)blockIdx.x * 2 * kMaxDim + threadIdx.x) * 2;
    p[0] = v.hi;
    p[1] = v.lo;
  }
}

#ifndef GM_FAMILY
#error "compile with -DGM_FAMILY=<1..7>"
#endif

template <int D>
static AdjFn adj_d(bool r9) {
  constexpr int F = GM_FAMILY;
  if constexpr (F >= 1 && F <= 6) return r9 ? adjoint_kernel<D, F, true> : adjoint_kernel<D, F, false>;
  return nullptr;
}

#define GM_CAT2(a, b) a##b
#define GM_CAT(a, b) GM_CAT2(a, b)

AdjFn GM_CAT(adjoint_kernel_f, GM_FAMILY)(int d, bool r9) {
  switch (d) {
    case 2: return adj_d<2>(r9);
    case 3: return adj_d<3>(r9);
    case 4: return adj_d<4>(r9);
    case 5: return adj_d<5>(r9);
    case 6: return adj_d<6>(r9);
    case 7: return adj_d<7>(r9);
    case 8: return adj_d<8>(r9);
    case 9: return adj_d<9>(r9);
    case 10: return adj_d<10>(r9);
    case 11: return adj_d<11>(r9);
    case 12: return adj_d<12>(r9);
    case 13: return adj_d<13>(r9);
    case 14: return adj_d<14>(r9);
    case 15: return adj_d<15>(r9);
    case 16: return adj_d<16>(r9);
    default: return nullptr;
  }
}

}  // namespace gm
