// Host build of the kernels' FP64 exp/cos/sin (paper_2511_01573_amd/csrc/gm_math.hpp)
// for tests/test_device_math.py.
#include "gm_math.hpp"
extern "C" {
void gm_test_exp(const double* x, double* y, long n) { for (long i = 0; i < n; ++i) y[i] = gm::fm::exp(x[i]); }
void gm_test_cos(const double* x, double* y, long n) { for (long i = 0; i < n; ++i) y[i] = gm::fm::cos(x[i]); }
void gm_test_sin(const double* x, double* y, long n) { for (long i = 0; i < n; ++i) y[i] = gm::fm::sin(x[i]); }
}
