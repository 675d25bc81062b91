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

static AdjFn adj_fn(int d, int fam, bool r9) {
  switch (fam) {
    case 1: return adjoint_kernel_f1(d, r9);
    case 2: return adjoint_kernel_f2(d, r9);
    case 3: return adjoint_kernel_f3(d, r9);
    case 4: return adjoint_kernel_f4(d, r9);
    case 5: return adjoint_kernel_f5(d, r9);
    case 6: return adjoint_kernel_f6(d, r9);
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
  // the adjoint covers the Genz-Malik rules (degree 7 and 9), not Gauss-Kronrod
  if (options().rule == 1) return GM_EINVAL;
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
    AdjFn fn = adj_fn(d, integrand_id, options().rule == 2);
    A.partials = part;
    A.R = RegionSrc{lv.C, lv.H, lv.L, nullptr, lv.cap, 0, 0};
    A.n = n1;
    hipLaunchKernelGGL(fn, dim3(g1), dim3(kAdjBlock), 0, s, A);
    A.partials = part + (size_t)g1 * 2 * kMaxDim * 2;
    A.R = RegionSrc{(const double*)(rr.base + rr.lay.C[rr.buf]),
                    (const double*)(rr.base + rr.lay.H[rr.buf]),
                    (const uint16_t*)(rr.base + rr.lay.L[rr.buf]),
                    (const uint8_t*)(rr.base + rr.lay.PAX[rr.buf]), rr.cap, rr.final_npar,
                    rr.final_split};
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
