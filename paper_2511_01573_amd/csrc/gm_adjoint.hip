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
#include "gm_math.hpp"

namespace gm {

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

// Per-node accumulation: acc[0..D) and acc[D..2D) are the family's factored
// sums; finish() turns them into dI/da_j and dI/du_j.
template <int D, int FAM>
__device__ __forceinline__ void adj_node(const DevParams& P, const double (&x)[D], double w,
                                         double (&acc)[2 * D]) {
  if constexpr (FAM == kOsc) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s = s + P.a[j] * x[j];
    const double ws = w * fm::sin(P.c0 + s);
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
    const double wf = w * fm::rcp(prod);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double r = wf * fm::rcp(den[j]);
      acc[j] += r;
      acc[D + j] = fma(r, x[j] - P.u[j], acc[D + j]);
    }
  } else if constexpr (FAM == kCornerPeak) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) s = s + P.a[j] * x[j];
    const double b = 1.0 + s;
    const double g = w * fm::rcp(ipow<D + 2>(b));
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = fma(g, x[j], acc[j]);
  } else if constexpr (FAM == kGaussian) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double t = P.a[j] * (x[j] - P.u[j]);
      s = s + t * t;
    }
    const double wf = w * fm::exp(-s);
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
    const double wf = w * fm::exp(-s);
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
    const double wf = out ? 0.0 : w * fm::exp(s);
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = fma(wf, x[j], acc[j]);
  }
}

// The factor that turns the factored sums (times the region volume, summed
// over the regions) into dI/da_j (component j < D) and dI/du_j (D + j).  It
// depends on the parameters only, so it is applied once per block.
template <int D, int FAM>
__device__ __forceinline__ double adj_scale(const DevParams& P, int k) {
  const int j = k < D ? k : k - D;
  if constexpr (FAM == kOsc) {
    return k < D ? -1.0 : (k == D ? -6.283185307179586476925286766559 : 0.0);
  } else if constexpr (FAM == kProductPeak) {
    return k < D ? 2.0 / (P.a[j] * P.a[j] * P.a[j]) : 2.0;
  } else if constexpr (FAM == kCornerPeak) {
    return k < D ? -(double)(D + 1) : 0.0;
  } else if constexpr (FAM == kGaussian) {
    return k < D ? -2.0 * P.a[j] : 2.0 * P.a[j] * P.a[j];
  } else if constexpr (FAM == kC0) {
    return k < D ? -1.0 : P.a[j];
  } else {
    return k < D ? 1.0 : 0.0;
  }
}

// Visit every node of region (c, h) in the rule's class order, calling
// fn(class_weight_index, x) (the node-by-node path of dimensions above
// kAdjFactorMaxDim).
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
      return fm::rcp(P.inv_a2[j] + t * t);
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
  // phi on N independent arguments at once (the N-wide outer functions
  // interleave their dependent FMA chains)
  template <int D, int N>
  __device__ static __forceinline__ void phi_n(const DevParams& P, const double (&s)[N],
                                               double (&f)[N]) {
    double a[N];
    if constexpr (FAM == kOsc) {
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = P.c0 + s[i];
      fm::sin_n<N>(a, f);
    } else if constexpr (FAM == kProductPeak) {
#pragma unroll
      for (int i = 0; i < N; ++i) f[i] = s[i];
    } else if constexpr (FAM == kCornerPeak) {
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = ipow<D + 2>(1.0 + s[i]);
      fm::rcp_n<N>(a, f);
    } else if constexpr (FAM == kGaussian || FAM == kC0) {
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = -s[i];
      fm::exp_n<N>(a, f);
    } else {
      fm::exp_n<N>(s, f);  // the discontinuous family: exp(-inf) = 0 outside its box
    }
  }
  template <int D>
  __device__ static __forceinline__ double phi(const DevParams& P, double s) {
    const double a[1] = {s};
    double f[1];
    phi_n<D, 1>(P, a, f);
    return f[0];
  }
  // add w psi(x) for axis j into the factored sums
  template <int D>
  __device__ static __forceinline__ void add_point(const DevParams& P, int j, double x, double w,
                                                   double (&acc)[2 * D]) {
    if constexpr (FAM == kOsc || FAM == kCornerPeak || FAM == kDiscontinuous) {
      acc[j] = fma(w, x, acc[j]);
    } else if constexpr (FAM == kProductPeak) {
      const double t = x - P.u[j];
      const double r = w * fm::rcp(P.inv_a2[j] + t * t);
      acc[j] += r;
      acc[D + j] = fma(r, t, acc[D + j]);
    } else if constexpr (FAM == kGaussian) {
      const double t = x - P.u[j];
      acc[j] = fma(w * t, t, acc[j]);
      acc[D + j] = fma(w, t, acc[D + j]);
    } else {
      const double t = x - P.u[j];
      acc[j] = fma(w, fabs(t), acc[j]);
      acc[D + j] += (t > 0.0) ? w : ((t < 0.0) ? -w : 0.0);
    }
  }
  // add w (psi(+) Phi^+ + psi(-) Phi^-) for axis j into the factored sums
  template <int D>
  __device__ static __forceinline__ void add_axis(const DevParams& P, int j, double xp, double xm,
                                                  double wp, double wm, double (&acc)[2 * D]) {
    if constexpr (FAM == kOsc || FAM == kCornerPeak || FAM == kDiscontinuous) {
      acc[j] = fma(wp, xp, fma(wm, xm, acc[j]));
    } else if constexpr (FAM == kProductPeak) {
      const double tp = xp - P.u[j], tm = xm - P.u[j];
      const double rp = wp * fm::rcp(P.inv_a2[j] + tp * tp);
      const double rm = wm * fm::rcp(P.inv_a2[j] + tm * tm);
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
  } else if constexpr (J == D - 2) {
    // the last two levels: the four leaves' outer functions run interleaved
    const double sp = S::comb(s, tp[J]), sm = S::comb(s, tm[J]);
    const double a[4] = {S::comb(sp, tp[J + 1]), S::comb(sp, tm[J + 1]), S::comb(sm, tp[J + 1]),
                         S::comb(sm, tm[J + 1])};
    double f[4];
    S::template phi_n<D, 4>(P, a, f);
    fp[J + 1] += f[0] + f[2];
    fm_[J + 1] += f[1] + f[3];
    const double l = f[0] + f[1], r = f[2] + f[3];
    fp[J] += l;
    fm_[J] += r;
    return l + r;
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
  // (kept a loop: unrolled, its body would be scheduled into the preceding
  // node groups and hold both groups' registers at once)
#pragma unroll 1
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

// A copy of x the optimiser cannot relate to x (no instruction is emitted).
__device__ __forceinline__ double opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Factored node groups.  A node's contribution to axis j is phi(s) psi_j(x_j)
// (weights included in phi), and x_j is c_j for every node that does not move
// coordinate j.  Per axis the sum over a group's nodes is therefore
//   psi_j(c_j) (W - sum_o G_j(o)) + sum_o psi_j(c_j + o h_j) G_j(o)
// with W the weighted phi sum of the group and G_j(o) that of its nodes with
// x_j = c_j + o h_j, o one of the offsets +-l2, +-l3 (= +-l4) and +-l6.  A
// node then costs its argument chain (prefixes of centre terms shared, left to
// right as in the rule kernel), phi and an add into W and into the G of each
// coordinate it moves, instead of 2d multiply-adds; acc is formed once per
// region.  The G sums of a lane live in its own column of an LDS table
// (kind * D + axis rows; kinds +l2, -l2, +l3, -l3, +l6, -l6) and are
// accumulated with LDS atomic adds, which keeps them out of the registers the
// unrolled sweep needs; each lane touches only its own column, so the order
// of its adds is its program order.
constexpr int kG2p = 0, kG2m = 1, kG3p = 2, kG3m = 3, kG6p = 4, kG6m = 5;

template <int D>
__device__ __forceinline__ void gadd(double (*tab)[kAdjBlock], int tid, int kind, int j,
                                     double v) {
  atomicAdd(&tab[kind * D + j][tid], v);
}

// Finish of a group with NK kinds of offsets: acc from W and the G table.
// The coordinates are recomputed from copies the compiler cannot match with
// the sweep's own terms (matching them would keep every coordinate's terms
// live through the sweep).
template <int D, int FAM, int NK>
__device__ __forceinline__ void adj_finish_group(const DevParams& P, const RuleConsts& K,
                                                 double W, double (*tab)[kAdjBlock], int tid,
                                                 const double (&c)[D], const double (&h)[D],
                                                 double (&acc)[2 * D]) {
  using S = AdjSplit<FAM>;
  if constexpr (FAM == kOsc) acc[D] += W;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const double cj = opaque(c[j]), hj = opaque(h[j]);
    const double g2p = tab[kG2p * D + j][tid], g2m = tab[kG2m * D + j][tid];
    const double g3p = tab[kG3p * D + j][tid], g3m = tab[kG3m * D + j][tid];
    double moved = (g2p + g2m) + (g3p + g3m);
    if constexpr (NK == 6) {
      const double g6p = tab[kG6p * D + j][tid], g6m = tab[kG6m * D + j][tid];
      moved += g6p + g6m;
      S::template add_axis<D>(P, j, fma(K.lam6, hj, cj), fma(-K.lam6, hj, cj), g6p, g6m, acc);
    }
    S::template add_point<D>(P, j, cj, W - moved, acc);
    S::template add_axis<D>(P, j, fma(K.lam2, hj, cj), fma(-K.lam2, hj, cj), g2p, g2m, acc);
    S::template add_axis<D>(P, j, fma(K.lam3, hj, cj), fma(-K.lam3, hj, cj), g3p, g3m, acc);
  }
}

// Centre terms and their prefixes: pc[k] = tc[0] (+) ... (+) tc[k-1].
template <int D, int FAM>
__device__ __forceinline__ void centre_chain(const DevParams& P, const double (&c)[D],
                                             double (&tc)[D], double (&pc)[D + 1]) {
  using S = AdjSplit<FAM>;
#pragma unroll
  for (int j = 0; j < D; ++j) tc[j] = S::term(P, j, c[j]);
  pc[0] = S::kEmpty;
  pc[1] = tc[0];
#pragma unroll
  for (int k = 2; k <= D; ++k) pc[k] = S::comb(pc[k - 1], tc[k - 1]);
}

// Nodes that move only coordinate i, to c_i + off_q h_i (q < N): their
// weighted phi values f[q] (weight w).
template <int D, int FAM, int N>
__device__ __forceinline__ void axis_nodes(const DevParams& P, int i, const double (&xo)[N],
                                           const double (&tc)[D], const double (&pc)[D + 1],
                                           double w, double (&f)[N]) {
  using S = AdjSplit<FAM>;
  double a[N], g[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const double ti = S::term(P, i, xo[q]);
    double s = (i == 0) ? ti : S::comb(pc[i], ti);
#pragma unroll
    for (int k = i + 1; k < D; ++k) s = S::comb(s, tc[k]);
    a[q] = s;
  }
  S::template phi_n<D, N>(P, a, g);
#pragma unroll
  for (int q = 0; q < N; ++q) f[q] = w * g[q];
}

// Classes 1-4 (the centre, +-l2 e_i, +-l3 e_i, +-l4 (e_i +- e_j)), weights
// w[0..3], of region (c, h) added into acc.
template <int D, int FAM>
__device__ __forceinline__ void adj_classes14(const DevParams& P, const RuleConsts& K,
                                              const double* w, const double (&c)[D],
                                              const double (&h)[D], double (*tab)[kAdjBlock],
                                              int tid, double (&acc)[2 * D]) {
  using S = AdjSplit<FAM>;
#pragma unroll
  for (int s = 0; s < 4 * D; ++s) tab[s][tid] = 0.0;
  double tc[D], pc[D + 1];
  centre_chain<D, FAM>(P, c, tc, pc);
  double W = w[0] * S::template phi<D>(P, pc[D]);
  // classes 2 and 3: the four nodes on axis i
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double xo[4] = {fma(K.lam2, h[i], c[i]), fma(-K.lam2, h[i], c[i]),
                          fma(K.lam3, h[i], c[i]), fma(-K.lam3, h[i], c[i])};
    double f2[2], f3[2];
    axis_nodes<D, FAM, 2>(P, i, {xo[0], xo[1]}, tc, pc, w[1], f2);
    axis_nodes<D, FAM, 2>(P, i, {xo[2], xo[3]}, tc, pc, w[2], f3);
    gadd<D>(tab, tid, kG2p, i, f2[0]);
    gadd<D>(tab, tid, kG2m, i, f2[1]);
    gadd<D>(tab, tid, kG3p, i, f3[0]);
    gadd<D>(tab, tid, kG3m, i, f3[1]);
    W += (f2[0] + f2[1]) + (f3[0] + f3[1]);
  }
  // class 4: rows (i, sign_i) share the chain up to coordinate i
  double t3p[D], t3m[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    t3p[j] = S::term(P, j, fma(K.lam4, h[j], c[j]));
    t3m[j] = S::term(P, j, fma(-K.lam4, h[j], c[j]));
  }
#pragma unroll
  for (int i = 0; i < D - 1; ++i) {
#pragma unroll
    for (int si = 0; si < 2; ++si) {
      const double ti = si ? t3m[i] : t3p[i];
      double m = (i == 0) ? ti : S::comb(pc[i], ti);
      double row = 0.0;
#pragma unroll
      for (int j = i + 1; j < D; ++j) {
        double a[2], f[2];
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          double s = S::comb(m, sj ? t3m[j] : t3p[j]);
#pragma unroll
          for (int k = j + 1; k < D; ++k) s = S::comb(s, tc[k]);
          a[sj] = s;
        }
        S::template phi_n<D, 2>(P, a, f);
        const double fp = w[3] * f[0], fmn = w[3] * f[1];
        gadd<D>(tab, tid, kG3p, j, fp);
        gadd<D>(tab, tid, kG3m, j, fmn);
        row += fp + fmn;
        m = S::comb(m, tc[j]);
      }
      gadd<D>(tab, tid, si ? kG3m : kG3p, i, row);
      W += row;
    }
  }
  adj_finish_group<D, FAM, 4>(P, K, W, tab, tid, c, h, acc);
}

// The degree-9 rule's classes 6-8 (+-l6 e_i; +-l2 e_i +- l3 e_j for ordered
// pairs i != j; +-l4 (e_i +- e_j +- e_k) for i < j < k), weights w9[5..7].
template <int D, int FAM>
__device__ __forceinline__ void adj_classes678(const DevParams& P, const RuleConsts& K,
                                               const double (&c)[D], const double (&h)[D],
                                               double (*tab)[kAdjBlock], int tid,
                                               double (&acc)[2 * D]) {
  using S = AdjSplit<FAM>;
  const double w6 = K.w9[5], w7 = K.w9[6], w8 = K.w9[7];
#pragma unroll
  for (int s = 0; s < 6 * D; ++s) tab[s][tid] = 0.0;
  double tc[D], pc[D + 1];
  centre_chain<D, FAM>(P, c, tc, pc);
  double W = 0.0;
  // class 6: the two nodes +-l6 on axis i
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double f[2];
    axis_nodes<D, FAM, 2>(P, i, {fma(K.lam6, h[i], c[i]), fma(-K.lam6, h[i], c[i])}, tc, pc,
                          w6, f);
    gadd<D>(tab, tid, kG6p, i, f[0]);
    gadd<D>(tab, tid, kG6m, i, f[1]);
    W += f[0] + f[1];
  }
  double t2p[D], t2m[D], t3p[D], t3m[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    t2p[j] = S::term(P, j, fma(K.lam2, h[j], c[j]));
    t2m[j] = S::term(P, j, fma(-K.lam2, h[j], c[j]));
    t3p[j] = S::term(P, j, fma(K.lam3, h[j], c[j]));
    t3m[j] = S::term(P, j, fma(-K.lam3, h[j], c[j]));
  }
  // class 7: the lower coordinate lo of the pair at one of its four offsets,
  // the higher one at the other length (l2 <-> l3)
#pragma unroll
  for (int lo = 0; lo < D - 1; ++lo) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {  // lo at +l2, -l2, +l3, -l3
      const double tl = v == 0 ? t2p[lo] : v == 1 ? t2m[lo] : v == 2 ? t3p[lo] : t3m[lo];
      double m = (lo == 0) ? tl : S::comb(pc[lo], tl);
      double row = 0.0;
#pragma unroll
      for (int hi = lo + 1; hi < D; ++hi) {
        double a[2], f[2];
#pragma unroll
        for (int sh = 0; sh < 2; ++sh) {
          const double th = (v < 2) ? (sh ? t3m[hi] : t3p[hi]) : (sh ? t2m[hi] : t2p[hi]);
          double s = S::comb(m, th);
#pragma unroll
          for (int k = hi + 1; k < D; ++k) s = S::comb(s, tc[k]);
          a[sh] = s;
        }
        S::template phi_n<D, 2>(P, a, f);
        const double fp = w7 * f[0], fmn = w7 * f[1];
        gadd<D>(tab, tid, v < 2 ? kG3p : kG2p, hi, fp);
        gadd<D>(tab, tid, v < 2 ? kG3m : kG2m, hi, fmn);
        row += fp + fmn;
        m = S::comb(m, tc[hi]);
      }
      gadd<D>(tab, tid, v, lo, row);  // the kind index of lo's offset is v
      W += row;
    }
  }
  // class 8: triples; rows (i, s_i, j, s_j) share the chain up to coordinate j
#pragma unroll
  for (int i = 0; i < D - 2; ++i) {
#pragma unroll
    for (int si = 0; si < 2; ++si) {
      double mi = (i == 0) ? (si ? t3m[i] : t3p[i]) : S::comb(pc[i], si ? t3m[i] : t3p[i]);
      double rowi = 0.0;
#pragma unroll
      for (int j = i + 1; j < D - 1; ++j) {
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          double m = S::comb(mi, sj ? t3m[j] : t3p[j]);
          double rowj = 0.0;
#pragma unroll
          for (int k = j + 1; k < D; ++k) {
            double a[2], f[2];
#pragma unroll
            for (int sk = 0; sk < 2; ++sk) {
              double s = S::comb(m, sk ? t3m[k] : t3p[k]);
#pragma unroll
              for (int q = k + 1; q < D; ++q) s = S::comb(s, tc[q]);
              a[sk] = s;
            }
            S::template phi_n<D, 2>(P, a, f);
            const double fp = w8 * f[0], fmn = w8 * f[1];
            gadd<D>(tab, tid, kG3p, k, fp);
            gadd<D>(tab, tid, kG3m, k, fmn);
            rowj += fp + fmn;
            m = S::comb(m, tc[k]);
          }
          gadd<D>(tab, tid, sj ? kG3m : kG3p, j, rowj);
          rowi += rowj;
        }
        mi = S::comb(mi, tc[j]);
      }
      gadd<D>(tab, tid, si ? kG3m : kG3p, i, rowi);
      W += rowi;
    }
  }
  adj_finish_group<D, FAM, 6>(P, K, W, tab, tid, c, h, acc);
}

// Sum over the wavefront (a fixed butterfly; lane 0's result is used).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

#ifndef GM_ADJ_WAVES
#define GM_ADJ_WAVES 2
#endif
// Dimensions up to which the non-corner classes are swept in factored form
// (fully unrolled, as the one-lane rule kernel); above it node by node.
constexpr int kAdjFactorMaxDim = 10;
// Steps a lane sums on its own before its sums join the wavefront totals (the
// degree-9 classes 6-8 launch has no registers to spare for the sums).
template <int PART>
constexpr int kAdjFlush = PART == 0 ? 8 : 1;

// PART 0: the degree-7 rule's node set (classes 1-4 and the corners; with
// the degree-9 weights when R9); PART 2: the degree-9 rule's classes 6-8, a
// launch of its own.  A wavefront takes 64 consecutive regions per step; each
// lane sums its regions' contributions (times the region volume) over
// kAdjFlush steps, then the 64 lanes' sums are added by a fixed butterfly
// into the wavefront's double-double totals in LDS (a fixed order: the result
// does not depend on timing); the parameter-dependent factor of each
// component is applied once per block.
template <int D, int FAM, bool R9, int PART>
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(GM_ADJ_WAVES)))
void adjoint_kernel(AdjArgs A) {
  constexpr bool kFactor = D <= kAdjFactorMaxDim;
  constexpr int kSlots = !kFactor ? 1 : (PART == 0 ? 4 * D : 6 * D);
  __shared__ double tab[kSlots][kAdjBlock];
  __shared__ dd wtot[kAdjBlock / 64][2 * D];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) wtot[wv][j] = dd{0.0, 0.0};
  // per-lane sums over up to kAdjFlush steps, then into the wavefront totals
  double part[2 * D];
#pragma unroll
  for (int j = 0; j < 2 * D; ++j) part[j] = 0.0;
  int steps = 0;
  auto flush = [&]() {
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) {
      const double v = wave_sum_f64(part[j]);
      if (lane == 0) dd_add(wtot[wv][j], v);
      part[j] = 0.0;
    }
  };
  for (int64_t base = (int64_t)blockIdx.x * kAdjBlock + 64 * wv; base < A.n;
       base += (int64_t)gridDim.x * kAdjBlock) {
    const int64_t r = base + lane;
    double acc[2 * D];
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) acc[j] = 0.0;
    double vol = 0.0;
    if (r < A.n) {
      double c[D], h[D];
      const int lvl = load_region<D>(A.R, r, c, h);
      vol = ldexp(A.vol_omega, -lvl);
      if constexpr (PART == 0) {
        const double* w = R9 ? A.K.w9 : A.K.w;
        adj_corners<D, FAM>(A.P, A.K, w[4], c, h, acc);
        double cc[D], hh[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          cc[j] = opaque(c[j]);
          hh[j] = opaque(h[j]);
        }
        if constexpr (kFactor) {
          adj_classes14<D, FAM>(A.P, A.K, w, cc, hh, tab, tid, acc);
        } else {
          visit_nodes<D, false>(A.K, cc, hh, [&](int cls, const double (&x)[D]) {
            adj_node<D, FAM>(A.P, x, w[cls], acc);
          });
        }
      } else if constexpr (kFactor) {
        adj_classes678<D, FAM>(A.P, A.K, c, h, tab, tid, acc);
      } else {
        visit_nodes9_extra<D>(A.K, c, h, [&](int cls, const double (&x)[D]) {
          adj_node<D, FAM>(A.P, x, A.K.w9[cls], acc);
        });
      }
    }
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) part[j] = fma(vol, acc[j], part[j]);
    if (++steps == kAdjFlush<PART>) {
      flush();
      steps = 0;
    }
  }
  if (steps) flush();
  __syncthreads();
  if (tid < 2 * D) {
    dd v = wtot[0][tid];
    for (int k = 1; k < kAdjBlock / 64; ++k) v = dd_sum(v, wtot[k][tid]);
    const double sc = adj_scale<D, FAM>(A.P, tid);
    double* p = A.partials + ((int64_t)blockIdx.x * 2 * kMaxDim + threadIdx.x) * 2;
    p[0] = v.hi * sc;
    p[1] = v.lo * sc;
  }
}

#ifndef GM_FAMILY
#error "compile with -DGM_FAMILY=<1..7>"
#endif

template <int D>
static AdjFn adj_d(bool r9, int part) {
  constexpr int F = GM_FAMILY;
  if constexpr (F >= 1 && F <= 6) {
    if (part == 0) return r9 ? adjoint_kernel<D, F, true, 0> : adjoint_kernel<D, F, false, 0>;
    if (part == 2 && r9) return adjoint_kernel<D, F, true, 2>;
  }
  return nullptr;
}

#define GM_CAT2(a, b) a##b
#define GM_CAT(a, b) GM_CAT2(a, b)

AdjFn GM_CAT(adjoint_kernel_f, GM_FAMILY)(int d, bool r9, int part) {
  switch (d) {
    case 2: return adj_d<2>(r9, part);
    case 3: return adj_d<3>(r9, part);
    case 4: return adj_d<4>(r9, part);
    case 5: return adj_d<5>(r9, part);
    case 6: return adj_d<6>(r9, part);
    case 7: return adj_d<7>(r9, part);
    case 8: return adj_d<8>(r9, part);
    case 9: return adj_d<9>(r9, part);
    case 10: return adj_d<10>(r9, part);
    case 11: return adj_d<11>(r9, part);
    case 12: return adj_d<12>(r9, part);
    case 13: return adj_d<13>(r9, part);
    case 14: return adj_d<14>(r9, part);
    case 15: return adj_d<15>(r9, part);
    case 16: return adj_d<16>(r9, part);
    default: return nullptr;
  }
}

GM_CHECK_UNIT_F(adjoint, GM_FAMILY)

}  // namespace gm
