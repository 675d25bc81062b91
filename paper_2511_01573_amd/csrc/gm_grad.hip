// gm_grad.hip -- gradient mode: the derivative of the fixed-tree Genz-Malik
// quadrature with respect to the integrand parameters (a, u).
//
// The forward run (Sec. 3 loop) retains every retired region; together with
// the last evaluated active set they form the frozen tree whose rule values
// sum to the estimate.  The adjoint kernel evaluates
//     dI/dtheta = sum_leaves vol * sum_nodes w_class * df/dtheta(x_node)
// with the nodes and weights of the rule kernel (Sec. 2).  Per family the
// node derivative is accumulated in factored form (e.g. the Gaussian keeps
// sum w f (x_j - u_j)^2 and sum w f (x_j - u_j) per axis) and scaled once.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/gm.h"
#include "gm_common.hpp"
#include "gm_internal.hpp"

namespace gm {

constexpr int kAdjBlock = 128;
constexpr int kMaxAdjGrid = 4096;

struct AdjArgs {
  DevParams P;
  RuleConsts K;
  const double* C;
  const double* H;
  const uint16_t* L;
  int64_t cap;
  int64_t n;
  double vol_omega;
  double* partials;  // [grid][2*kMaxDim][2] double-double
};

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
template <int D, typename Fn>
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

template <int D, int FAM>
__global__ __launch_bounds__(kAdjBlock) void adjoint_kernel(AdjArgs A) {
  dd tot[2 * D];
#pragma unroll
  for (int j = 0; j < 2 * D; ++j) tot[j] = dd{0.0, 0.0};
  for (int64_t r = (int64_t)blockIdx.x * kAdjBlock + threadIdx.x; r < A.n;
       r += (int64_t)gridDim.x * kAdjBlock) {
    double c[D], h[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      c[j] = A.C[j * A.cap + r];
      h[j] = A.H[j * A.cap + r];
    }
    const double vol = ldexp(A.vol_omega, -(int)A.L[r]);
    double acc[2 * D];
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) acc[j] = 0.0;
    visit_nodes<D>(A.K, c, h, [&](int cls, const double (&x)[D]) {
      adj_node<D, FAM>(A.P, x, A.K.w[cls], acc);
    });
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

__global__ void adjoint_reduce_kernel(const double* partials, int np, int nparam, double* out) {
  const int j = threadIdx.x;
  if (j >= nparam) return;
  dd v = {0.0, 0.0};
  for (int b = 0; b < np; ++b) {
    const double* p = partials + ((int64_t)b * 2 * kMaxDim + j) * 2;
    v = dd_sum(v, dd{p[0], p[1]});
  }
  out[j] = dd_val(v);
}

using AdjFn = void (*)(AdjArgs);

template <int D>
static AdjFn adj_fn_d(int fam) {
  switch (fam) {
    case 1: return adjoint_kernel<D, 1>;
    case 2: return adjoint_kernel<D, 2>;
    case 3: return adjoint_kernel<D, 3>;
    case 4: return adjoint_kernel<D, 4>;
    case 5: return adjoint_kernel<D, 5>;
    case 6: return adjoint_kernel<D, 6>;
    default: return nullptr;
  }
}

static AdjFn adj_fn(int d, int fam) {
  switch (d) {
    case 2: return adj_fn_d<2>(fam);
    case 3: return adj_fn_d<3>(fam);
    case 4: return adj_fn_d<4>(fam);
    case 5: return adj_fn_d<5>(fam);
    case 6: return adj_fn_d<6>(fam);
    case 7: return adj_fn_d<7>(fam);
    case 8: return adj_fn_d<8>(fam);
    case 9: return adj_fn_d<9>(fam);
    case 10: return adj_fn_d<10>(fam);
    case 11: return adj_fn_d<11>(fam);
    case 12: return adj_fn_d<12>(fam);
    case 13: return adj_fn_d<13>(fam);
    case 14: return adj_fn_d<14>(fam);
    case 15: return adj_fn_d<15>(fam);
    case 16: return adj_fn_d<16>(fam);
    default: return nullptr;
  }
}

}  // namespace gm

using namespace gm;

extern "C" int gm_integrate_grad(int integrand_id, const double* params, int d, const double* lo,
                                 const double* hi, double rel_tol, double abs_tol,
                                 int64_t max_regions, double* out_est, double* out_err,
                                 double* out_grad, void* stream) {
  int rc = validate(integrand_id, params, d, lo, hi, rel_tol, abs_tol);
  if (rc != GM_OK) return rc;
  if (!out_est || !out_err || !out_grad) return GM_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  hipStream_t s = (hipStream_t)stream;
  RunResult rr;
  rc = run_adaptive(integrand_id, params, d, lo, hi, rel_tol, abs_tol, max_regions, s, true, &rr);
  if (rc != GM_OK) return rc;
  if (rr.status == GM_NONFINITE) {
    *out_est = rr.I;
    *out_err = rr.E;
    for (int j = 0; j < 2 * d; ++j) out_grad[j] = NAN;
    return rr.status;
  }
  std::vector<double> grad(2 * d, 0.0);
  if (integrand_id != kPolyF7) {
    const LeafView lv = leaf_view();
    AdjArgs A;
    std::memset(&A, 0, sizeof A);
    fill_params(integrand_id, d, params, A.P);
    fill_consts(d, A.K);
    A.vol_omega = rr.vol_omega;
    // Partials: leaves first, then the last active set, reduced together.
    const int64_t n1 = rr.leaf_count, n2 = rr.final_n;
    const int g1 = (int)std::max<int64_t>(1, std::min<int64_t>((n1 + kAdjBlock - 1) / kAdjBlock, kMaxAdjGrid / 2));
    const int g2 = (int)std::max<int64_t>(1, std::min<int64_t>((n2 + kAdjBlock - 1) / kAdjBlock, kMaxAdjGrid / 2));
    double* part = nullptr;
    double* dout = nullptr;
    const size_t pbytes = sizeof(double) * 2 * 2 * kMaxDim * (size_t)(g1 + g2);
    if (hipMalloc(&part, pbytes) != hipSuccess || hipMalloc(&dout, sizeof(double) * 2 * kMaxDim) != hipSuccess) {
      (void)hipGetLastError();
      if (part) (void)hipFree(part);
      return GM_ENOMEM;
    }
    AdjFn fn = adj_fn(d, integrand_id);
    A.partials = part;
    A.C = lv.C;
    A.H = lv.H;
    A.L = lv.L;
    A.cap = lv.cap;
    A.n = n1;
    hipLaunchKernelGGL(fn, dim3(g1), dim3(kAdjBlock), 0, s, A);
    A.partials = part + (size_t)g1 * 2 * kMaxDim * 2;
    A.C = (const double*)(rr.base + rr.lay.C[rr.buf]);
    A.H = (const double*)(rr.base + rr.lay.H[rr.buf]);
    A.L = (const uint16_t*)(rr.base + rr.lay.L[rr.buf]);
    A.cap = rr.cap;
    A.n = n2;
    hipLaunchKernelGGL(fn, dim3(g2), dim3(kAdjBlock), 0, s, A);
    hipLaunchKernelGGL(adjoint_reduce_kernel, dim3(1), dim3(64), 0, s, part, g1 + g2, 2 * d, dout);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(grad.data(), dout, sizeof(double) * 2 * d, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(part);
    (void)hipFree(dout);
    if (e != hipSuccess) return record_hip_error(e);
  }
  *out_est = rr.I;
  *out_err = rr.E;
  for (int j = 0; j < 2 * d; ++j) out_grad[j] = grad[j];
  return rr.status;
}
