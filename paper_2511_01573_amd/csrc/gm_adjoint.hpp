// gm_adjoint.hpp -- declarations of the gradient-mode adjoint kernels.
#pragma once

#include "gm_common.hpp"

namespace gm {

constexpr int kAdjBlock = 128;
constexpr int kMaxAdjGrid = 4096;

struct AdjArgs {
  DevParams P;
  RuleConsts K;
  RegionSrc R;  // the regions (a stored split active set or the leaf store)
  int64_t n;
  double vol_omega;
  double* partials;  // [grid][2*kMaxDim][2] double-double
};

using AdjFn = void (*)(AdjArgs);
// One per family translation unit (r9: the degree-9 rule's nodes and weights;
// part: the node group a launch covers, 0 = the degree-7 node set (classes
// 1-5), 2 = the degree-9 rule's classes 6-8); nullptr for the polynomial (no
// parameters) and for part 2 of the degree-7 rule.
AdjFn adjoint_kernel_f1(int d, bool r9, int part);
AdjFn adjoint_kernel_f2(int d, bool r9, int part);
AdjFn adjoint_kernel_f3(int d, bool r9, int part);
AdjFn adjoint_kernel_f4(int d, bool r9, int part);
AdjFn adjoint_kernel_f5(int d, bool r9, int part);
AdjFn adjoint_kernel_f6(int d, bool r9, int part);
AdjFn adjoint_kernel_f7(int d, bool r9, int part);

}  // namespace gm
