// gm_grad.hip -- gradient mode: the derivative of the fixed-tree Genz-Malik
// quadrature with respect to the integrand parameters (a, u).
//
// The forward run (Sec. 3 loop) retains every retired region; together with
// the last evaluated active set they form the frozen tree whose rule values
// sum to the estimate.  The adjoint kernels (gm_adjoint.hip) evaluate
//     dI/dtheta = sum_leaves vol * sum_nodes w_class * df/dtheta(x_node)
// and a one-workgroup kernel reduces their double-double block partials.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/gm.h"
#include "gm_adjoint.hpp"
#include "gm_common.hpp"
#include "gm_internal.hpp"

namespace gm {

// Sum of the np block partials of each of the nparam components (double-
// double, in a fixed order: thread t adds blocks t, t + 256, ... and the 256
// per-thread sums are combined by a fixed tree).
__global__ __launch_bounds__(256) void adjoint_reduce_kernel(const double* partials, int np,
                                                             int nparam, double* out) {
  __shared__ dd sh[256];
  const int t = threadIdx.x;
  for (int j = 0; j < nparam; ++j) {
    dd v = {0.0, 0.0};
    for (int b = t; b < np; b += 256) {
      const double* p = partials + ((int64_t)b * 2 * kMaxDim + j) * 2;
      v = dd_sum(v, dd{p[0], p[1]});
    }
    sh[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) sh[t] = dd_sum(sh[t], sh[t + s]);
      __syncthreads();
    }
    if (t == 0) out[j] = dd_val(sh[0]);
    __syncthreads();
  }
}

static AdjFn adj_fn(int d, int fam, bool r9, int part) {
  switch (fam) {
    case 1: return adjoint_kernel_f1(d, r9, part);
    case 2: return adjoint_kernel_f2(d, r9, part);
    case 3: return adjoint_kernel_f3(d, r9, part);
    case 4: return adjoint_kernel_f4(d, r9, part);
    case 5: return adjoint_kernel_f5(d, r9, part);
    case 6: return adjoint_kernel_f6(d, r9, part);
    default: return nullptr;
  }
}

GM_CHECK_UNIT(grad)

}  // namespace gm

using namespace gm;

extern "C" int gm_integrate_grad(int integrand_id, const double* params, int d, const double* lo,
                                 const double* hi, double rel_tol, double abs_tol,
                                 int64_t max_regions, double* out_est, double* out_err,
                                 double* out_grad, void* stream) {
  int rc = validate(integrand_id, params, d, lo, hi, rel_tol, abs_tol);
  if (rc != GM_OK) return rc;
  if (!out_est || !out_err || !out_grad) return GM_EINVAL;
  // the adjoint covers the Genz-Malik rules (degree 7 and 9), not Gauss-Kronrod
  if (options().rule == 1) return GM_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  hipStream_t s = (hipStream_t)stream;
  RunResult rr;
  rc = check_bounds(
      run_adaptive(integrand_id, params, d, lo, hi, rel_tol, abs_tol, max_regions, s, true, &rr));
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
    // One launch per node group (classes 1-5 and, for the degree-9 rule, its
    // classes 6-8) over each region set (the leaf store, then the
    // last active set); every launch writes its own block partials, reduced
    // together.
    const bool r9 = options().rule == 2;
    const int parts[2] = {0, 2};  // classes 1-5; the degree-9 rule's classes 6-8
    const int nparts = r9 ? 2 : 1;
    const int64_t n1 = rr.leaf_count, n2 = rr.final_n;
    const int g1 = (int)std::max<int64_t>(1, std::min<int64_t>((n1 + kAdjBlock - 1) / kAdjBlock, kMaxAdjGrid / 2));
    const int g2 = (int)std::max<int64_t>(1, std::min<int64_t>((n2 + kAdjBlock - 1) / kAdjBlock, kMaxAdjGrid / 2));
    const int nblocks = nparts * (g1 + g2);
    double* part = nullptr;
    double* dout = nullptr;
    const size_t pbytes = sizeof(double) * 2 * 2 * kMaxDim * (size_t)nblocks;
    if (hipMalloc(&part, pbytes) != hipSuccess || hipMalloc(&dout, sizeof(double) * 2 * kMaxDim) != hipSuccess) {
      (void)hipGetLastError();
      if (part) (void)hipFree(part);
      return GM_ENOMEM;
    }
    const RegionSrc leaves{lv.C, lv.H, lv.L, nullptr, lv.cap, 0, 0};
    const RegionSrc active{(const double*)(rr.base + rr.lay.C[rr.buf]),
                           (const double*)(rr.base + rr.lay.H[rr.buf]),
                           (const uint16_t*)(rr.base + rr.lay.L[rr.buf]),
                           (const uint8_t*)(rr.base + rr.lay.PAX[rr.buf]), rr.cap, rr.final_npar,
                           rr.final_split};
    int64_t blk = 0;
    for (int pt = 0; pt < nparts; ++pt) {
      AdjFn fn = adj_fn(d, integrand_id, r9, parts[pt]);
      for (int set = 0; set < 2; ++set) {
        const int g = set ? g2 : g1;
        A.partials = part + (size_t)blk * 2 * kMaxDim * 2;
        A.R = set ? active : leaves;
        A.n = set ? n2 : n1;
        hipLaunchKernelGGL(fn, dim3(g), dim3(kAdjBlock), 0, s, A);
        blk += g;
      }
    }
    hipLaunchKernelGGL(adjoint_reduce_kernel, dim3(1), dim3(256), 0, s, part, nblocks, 2 * d, dout);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(grad.data(), dout, sizeof(double) * 2 * d, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(part);
    (void)hipFree(dout);
    if (e != hipSuccess) return record_hip_error(e);
    rc = check_bounds(GM_OK);
    if (rc != GM_OK) return rc;
  }
  *out_est = rr.I;
  *out_err = rr.E;
  for (int j = 0; j < 2 * d; ++j) out_grad[j] = grad[j];
  return rr.status;
}
