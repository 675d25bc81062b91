// gm_common.hpp -- device-side types shared by the libgm kernels (gfx950, FP64).
//
// Method: arXiv 2511.01573 (adaptive Genz-Malik cubature, Sec. 2-4).  This
// header holds the kernel argument blocks, the device status block that drives
// the iteration (Sec. 3 loop), the integrand parameter block (Sec. 4 test
// functions and their Genz families) and compensated (double-double) summation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gm {

constexpr int kMaxDim = 16;
constexpr int kMinDim = 2;

// ---------------------------------------------------------------------------
// Bounds checks of the -DGM_CHECK build.  GM_INB(i, n) is true when
// 0 <= i < n.  In a GM_CHECK build a false result also counts a violation and
// records the first one (source line, index, bound) in this translation
// unit's device record; the caller skips the access it guards, so the kernel
// still ends normally, and the host turns a nonzero count into GM_EHIP after
// the call (gm_check_poll_* of every unit).  Without GM_CHECK the check is the
// constant true and compiles to nothing; GM_GUARD(i, n) is the same check for
// accesses that are guarded in every build.
// ---------------------------------------------------------------------------
struct CheckRec {
  unsigned long long count;
  long long index, bound;
  int line;
  int pad;
};

#ifdef GM_CHECK
static __device__ CheckRec g_chk;

__device__ __noinline__ inline void check_fail(int64_t i, int64_t n, int line) {
  if (atomicAdd(&g_chk.count, 1ull) == 0ull) {
    g_chk.index = i;
    g_chk.bound = n;
    g_chk.line = line;
  }
}

__device__ __forceinline__ bool in_bounds(int64_t i, int64_t n, int line) {
  if (i >= 0 && i < n) return true;
  check_fail(i, n, line);
  return false;
}
#define GM_INB(i, n) ::gm::in_bounds((int64_t)(i), (int64_t)(n), __LINE__)

// Host: copy this unit's record to *out and clear it; 0 or -1 (HIP error).
#define GM_CHECK_POLL_BODY                                                              \
  {                                                                                     \
    const ::gm::CheckRec z = {};                                                        \
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(::gm::g_chk), sizeof *out) != hipSuccess)   \
      return -1;                                                                        \
    if (out->count != 0 &&                                                              \
        hipMemcpyToSymbol(HIP_SYMBOL(::gm::g_chk), &z, sizeof z) != hipSuccess)         \
      return -1;                                                                        \
    return 0;                                                                           \
  }
#define GM_CAT3_(a, b, c) a##b##c
#define GM_CAT3(a, b, c) GM_CAT3_(a, b, c)
// One poll function per translation unit: gm_check_poll_<name>[_f<family>].
#define GM_CHECK_UNIT(name) \
  int GM_CAT3(gm_check_poll_, name, )(::gm::CheckRec* out) GM_CHECK_POLL_BODY
#define GM_CHECK_UNIT_F(name, fam) \
  int GM_CAT3(gm_check_poll_, name, GM_CAT3(_f, fam, ))(::gm::CheckRec* out) GM_CHECK_POLL_BODY
#define GM_GUARD(i, n) GM_INB(i, n)
#else
#define GM_INB(i, n) true
#define GM_CHECK_UNIT(name)
#define GM_CHECK_UNIT_F(name, fam)
// A guard that stays in every build (the access is skipped when the index
// is out of range); a GM_CHECK build also counts it as a violation.
#define GM_GUARD(i, n) ((int64_t)(i) >= 0 && (int64_t)(i) < (int64_t)(n))
#endif

// Integrand families (the numbering of include/gm.h).
enum Family : int {
  kOsc = 1,
  kProductPeak = 2,
  kCornerPeak = 3,
  kGaussian = 4,
  kC0 = 5,
  kDiscontinuous = 6,
  kPolyF7 = 7
};

// Integrand parameters as the kernels consume them.  a, u are the caller's;
// inv_a2 = 1/(a*a) (product peak) and c0 = 2*pi*u_0 (oscillatory) are formed
// once on the host with the same single roundings the definitions imply.
struct DevParams {
  double a[kMaxDim];
  double u[kMaxDim];
  double inv_a2[kMaxDim];
  double c0;
  int d;
  int fam;
};

// Rule constants for one dimension d (Sec. 2; degree-7 fully symmetric rule
// with generators 0, l2 e_i, l3 e_i, l4 (e_i +- e_j), l5 (+-1,...,+-1) and
// its embedded degree-5 rule).  w = degree-7 weights, e = w - v (v the
// degree-5 weights), r7 = l2^2 / l3^2 = 1/7.
struct RuleConsts {
  double lam2, lam3, lam4, lam5;
  double w[5];
  double e[5];
  double r7;
  double axis_band;  // relative noise band of the split-axis comparison
  // Degree-9 rule (classes 1..8: the five above, +-l6 e_i, (+-l2 e_i, +-l3 e_j)
  // for ordered pairs i != j, +-l4 (e_i + e_j + e_k) for i < j < k).
  double lam6;
  double w9[8];   // degree-9 weights
  double e9[8];   // degree-9 minus degree-7 weights
  double q3[2];   // degree-3 rule on the centre and the +-l3 e_i nodes
  int32_t err_model;  // 0: |Q9 - Q7|; 1: null-rule ratio test
};

// Device status block: the only state the host reads between iterations.
struct Status {
  int64_t n_active;     // regions in the current active set
  int64_t n_prev;       // active count of the iteration being split
  int64_t n_keep;       // regions kept (to be split) this iteration
  int64_t iter;         // evaluate steps done
  int64_t done;         // 1 once a final status is set
  int64_t status;       // GM_* code
  int32_t nonfinite;    // set by the rule kernel
  int32_t buf;          // ping-pong buffer that holds the active set
  int64_t regions_evaluated;
  int64_t finished;
  int64_t max_active;
  int64_t leaf_base;    // first leaf slot of this iteration's retired regions
  int64_t leaf_count;   // retired leaves stored so far (gradient mode)
  int64_t cap;          // active-set capacity
  int64_t max_iters;
  double I, E, T;
  double ifin_hi, ifin_lo, efin_hi, efin_lo;
  double rel_tol, abs_tol;
  int32_t prune_on;     // memory-pressure pruning enabled
  int32_t pruned;       // pruning happened in this run
  int32_t reclassify;   // this iteration is classified again with the relaxed budget
  int32_t prune_k;      // budget factor 2^prune_k of that second pass
  int64_t n_par;        // parent records behind a split active set
  int32_t split;        // 1: the active set is the 2 n_par children of the stored parents
  int32_t split_in;     // split / n_par of the set being compacted (read by the scatter)
  int64_t n_par_in;
};

// ---------------------------------------------------------------------------
// Compensated summation.  TwoSum (Knuth) is exact in binary64 as long as the
// compiler does not reassociate; the library is built with -ffp-contract=off.
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

__device__ __forceinline__ void dd_add(dd& x, double y) {
  double s, e;
  two_sum(x.hi, y, s, e);
  x.hi = s;
  x.lo += e;
}

__device__ __forceinline__ dd dd_sum(dd x, dd y) {
  double s, e;
  two_sum(x.hi, y.hi, s, e);
  e += x.lo + y.lo;
  dd r;
  r.hi = s + e;
  r.lo = e - (r.hi - s);
  return r;
}

__device__ __forceinline__ double dd_val(dd x) { return x.hi + x.lo; }

__device__ __forceinline__ dd shfl_xor_dd(dd v, int m) {
  dd r;
  r.hi = __shfl_xor(v.hi, m, 64);
  r.lo = __shfl_xor(v.lo, m, 64);
  return r;
}

// Sum of a double-double over the 64 lanes of a wavefront (butterfly; every
// lane ends with the same value).
__device__ __forceinline__ dd wave_sum_dd(dd v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = dd_sum(v, shfl_xor_dd(v, m));
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// The active set as stored.  After the first split the store holds one
// record per region kept in the previous iteration (c, h, lvl and its split
// axis PAX), and the active set is their 2 n_par children: region r < n_par is
// the "-" child of record r, region n_par + r the "+" child (Sec. 3 split:
// along the axis, c -+ h/2, h/2, level + 1 -- exact for these dyadic boxes).
// Before the first split (and for region lists) records are the regions.
struct RegionSrc {
  const double* C;
  const double* H;
  const uint16_t* L;
  const uint8_t* PAX;
  int64_t cap;
  int64_t npar;
  int split;
};

// Region r of the active set: centre, half-widths, level.
template <int D>
__device__ __forceinline__ int load_region(const RegionSrc& R, int64_t r, double (&c)[D],
                                           double (&h)[D]) {
  const bool plus = R.split && r >= R.npar;
  const int64_t q = plus ? r - R.npar : r;
  if (!GM_INB(q, R.cap)) {
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = h[j] = 0.0;
    return 0;
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    c[j] = R.C[j * R.cap + q];
    h[j] = R.H[j * R.cap + q];
  }
  int lvl = R.L[q];
  if (R.split) {
    const int ax = R.PAX[q];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (j == ax) {
        const double hp = h[j] * 0.5;
        c[j] = plus ? c[j] + hp : c[j] - hp;
        h[j] = hp;
      }
    }
    lvl += 1;
  }
  return lvl;
}

// Level of region r of the active set.
__device__ __forceinline__ int region_level(const RegionSrc& R, int64_t r) {
  if (!R.split) return R.L[r];
  return R.L[r >= R.npar ? r - R.npar : r] + 1;
}

// Kernel arguments of the rule kernel (Sec. 2 evaluation of every region).
struct RuleArgs {
  DevParams P;
  RuleConsts K;
  const double* C[2];     // SoA centres  [j * cap + r], ping-pong
  const double* H[2];     // SoA half-widths
  const uint16_t* L[2];   // levels: region volume = vol_omega * 2^-lvl
  const uint8_t* PAX[2];  // split axis of each stored record (split active sets)
  int64_t cap;
  double* Q;              // [cap] rule value
  double* ERR;            // [cap] error estimate
  uint8_t* AXIS;          // [cap] split axis, bit 7 = geometry guard
  double* partials;       // [grid][4] double-double (Q, err) per block
  Status* st;
  double vol_omega;
  int64_t n_fixed;        // >= 0: evaluate this many regions of buffer 0, ignore st
  // Batch mode (the BATCH kernels): regions [grp[0], grp[1]) of one (d, family)
  // group of a batch store; region r belongs to item IT[buf][r] with parameters
  // PARAMS[item] and domain volume VOL[item]; buf = *bbuf.
  const uint32_t* IT[2];
  const DevParams* PARAMS;
  const double* VOL;
  const int64_t* grp;
  const int32_t* bbuf;
};

// AXIS byte: bits 0-5 split axis, bit 6 non-finite rule sums, bit 7 geometry guard.
constexpr uint8_t kAxisMask = 0x3f;
constexpr uint8_t kNonfiniteBit = 0x40;
constexpr uint8_t kGeoBit = 0x80;

// One launcher per family (each built in its own translation unit).
// log2l < 0: one lane per region (d <= kTprMaxDim); else 2^log2l lanes per
// region (log2l in {2, 4, 6}, d >= 6, 8, 10 respectively).
// batch = true selects the batch-store kernels (per-region item parameters).
using RuleKernelFn = void (*)(RuleArgs);
RuleKernelFn rule_kernel_f1(int d, int log2l, bool batch);
RuleKernelFn rule_kernel_f2(int d, int log2l, bool batch);
RuleKernelFn rule_kernel_f3(int d, int log2l, bool batch);
RuleKernelFn rule_kernel_f4(int d, int log2l, bool batch);
RuleKernelFn rule_kernel_f5(int d, int log2l, bool batch);
RuleKernelFn rule_kernel_f6(int d, int log2l, bool batch);
RuleKernelFn rule_kernel_f7(int d, int log2l, bool batch);
constexpr int kTprMaxDim = 10;
constexpr int kBatchMaxDim = kTprMaxDim;  // batch items have 2 <= d <= 10
constexpr int kRuleBlockSize = 256;

// Threads of the Gauss-Kronrod kernel per region: one wavefront up to d = 3, the
// whole workgroup from d = 4 on (15^d nodes per region).
constexpr int gk_threads(int d) { return d >= 4 ? kRuleBlockSize : 64; }

// Tensor-product Gauss-Kronrod rule kernels (gk_threads(d) per region), one
// launcher per family, 2 <= d <= kGkMaxDim (batch: the batch-store variant).
RuleKernelFn gk_kernel_f1(int d, bool batch);
RuleKernelFn gk_kernel_f2(int d, bool batch);
RuleKernelFn gk_kernel_f3(int d, bool batch);
RuleKernelFn gk_kernel_f4(int d, bool batch);
RuleKernelFn gk_kernel_f5(int d, bool batch);
RuleKernelFn gk_kernel_f6(int d, bool batch);
RuleKernelFn gk_kernel_f7(int d, bool batch);
constexpr int kGkMaxDim = 6;

// Degree-9 fully symmetric rule kernels, one launcher per family, 2 <= d <= 16
// (batch-store kernels: d <= kBatchMaxDim); 2^rule9_log2l(d) lanes of one
// wavefront per region (at least one corner and at most 64 lanes per region),
// or 2^rule9_log2l_wide(d) with `wide` (single-store kernels only).
RuleKernelFn rule9_kernel_f1(int d, bool batch, bool wide);
RuleKernelFn rule9_kernel_f2(int d, bool batch, bool wide);
RuleKernelFn rule9_kernel_f3(int d, bool batch, bool wide);
RuleKernelFn rule9_kernel_f4(int d, bool batch, bool wide);
RuleKernelFn rule9_kernel_f5(int d, bool batch, bool wide);
RuleKernelFn rule9_kernel_f6(int d, bool batch, bool wide);
RuleKernelFn rule9_kernel_f7(int d, bool batch, bool wide);
constexpr int rule9_log2l(int d) { return d - 5 < 2 ? 2 : (d - 5 > 6 ? 6 : d - 5); }
// The wide mapping of the degree-9 kernel for active sets too small to fill
// the GPU at rule9_log2l(d): up to 64 lanes per region (at least one corner
// per lane).
constexpr int rule9_log2l_wide(int d) { return d < 6 ? d : 6; }

}  // namespace gm
