// gm_stubs.hip -- temporary: batch and gradient entry points.
#include "../../include/gm.h"
#include "gm_internal.hpp"
namespace gm {
size_t batch_layout_bytes(int dmax, int64_t cap) { return make_layout(dmax, cap).total; }
}
extern "C" {
int gm_integrate_batch(int, const int*, const double*, const int*, const double*, const double*,
                       const double*, const double*, int64_t, double*, double*, int*, void*) {
  return GM_EINVAL;
}
}
