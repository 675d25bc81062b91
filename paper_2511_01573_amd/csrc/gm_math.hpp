// gm_math.hpp -- FP64 exp and cos for the rule kernel's outer functions.
//
// Written for the node sweep, where every integrand evaluation ends in one
// transcendental: both functions are almost entirely FP64 FMAs (no table
// lookups, no branches on the common path).
//
// exp(x): Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2, with k = rint(x /
//   ln2) obtained by the 1.5 * 2^52 rounding shift (its low word is k), r from
//   two FMAs against ln2 split in two doubles; e^r from a degree-11 polynomial
//   (Chebyshev approximation on [-ln2/2, ln2/2], max error 3.2e-18, Horner
//   form); the result is scaled by 2^k with ldexp, which also produces the
//   correct underflow to 0 and overflow to +inf.  Arguments below -1100 are
//   clamped (e^-1100 underflows to 0), which also maps -inf to 0.
// cos(x): reduction by pi/2 (three-part Cody-Waite with FMAs: pi/2 carried in
//   three doubles, each product formed exactly inside an FMA; accurate while
//   |x| < 2^48, the range the kernels admit), cos(r) = C(r^2) (degree 7 in r^2)
//   and sin(r) = r S(r^2) (degree 6), quadrant select.  No branch.
// Coefficients: csrc/gen_math_coeffs.py (mpmath, 50 digits).  Both functions
// compile unchanged for the host, where tests/test_device_math.py measures
// their error against 50-digit references.
#pragma once

#include <stdint.h>

#include <cmath>
#include <cstring>

#ifndef GM_HD
#if defined(__HIPCC__) || defined(__CUDACC__)
#define GM_HD __host__ __device__ __forceinline__
#else
#define GM_HD inline
#endif
#endif

namespace gm {
namespace fm {

constexpr double kExpPoly[12] = {
    0x1.af631d0059becp-26, 0x1.28b4057f44145p-22, 0x1.71ddf5749d126p-19, 0x1.a01991ac8730ap-16,
    0x1.a01a01b14378fp-13, 0x1.6c16c187fbe02p-10, 0x1.111111110f225p-7,  0x1.555555554f0cfp-5,
    0x1.555555555555ap-3,  0x1.0000000000011p-1,  0x1.0000000000000p+0,  0x1.0000000000000p+0};
constexpr double kCosPoly[8] = {-0x1.8f762711e61e0p-37, 0x1.1ee96d0192650p-29,
                                -0x1.27e4f727f10b7p-22, 0x1.a01a019b1e24dp-16,
                                -0x1.6c16c16c13a05p-10, 0x1.5555555555536p-5,
                                -0x1.0000000000000p-1,  0x1.0000000000000p+0};
constexpr double kSinPoly[7] = {0x1.5d87699eb6a31p-33,  -0x1.ae5e37e850d20p-26,
                                0x1.71de3530aa14dp-19,  -0x1.a01a019ba956dp-13,
                                0x1.111111110f3dcp-7,   -0x1.5555555555543p-3,
                                0x1.0000000000000p+0};
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kPio2_1 = 0x1.921fb54442d18p+0;
constexpr double kPio2_2 = 0x1.1a62633145c07p-54;
constexpr double kPio2_3 = -0x1.f1976b7ed8fbcp-110;
constexpr double k2OverPi = 0x1.45f306dc9c883p-1;
constexpr double kShift = 0x1.8p52;  // 1.5 * 2^52: adding it rounds to an integer

GM_HD int32_t low_word(double t) {
  uint64_t b;
  std::memcpy(&b, &t, sizeof b);
  return (int32_t)(uint32_t)b;
}

GM_HD double exp(double x) {
  x = fmax(x, -1100.0);
  const double t = fma(x, kInvLn2, kShift);
  const double kd = t - kShift;
  const int32_t k = low_word(t);
  double r = fma(-kd, kLn2Hi, x);
  r = fma(-kd, kLn2Lo, r);
  double p = kExpPoly[0];
#pragma unroll
  for (int i = 1; i < 12; ++i) p = fma(p, r, kExpPoly[i]);
  return ldexp(p, k);
}

GM_HD double cos(double x) {
  const double t = fma(x, k2OverPi, kShift);
  const double kd = t - kShift;
  const int32_t q = low_word(t);
  double r = fma(-kd, kPio2_1, x);
  r = fma(-kd, kPio2_2, r);
  r = fma(-kd, kPio2_3, r);
  const double z = r * r;
  double c = kCosPoly[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) c = fma(c, z, kCosPoly[i]);
  double s = kSinPoly[0];
#pragma unroll
  for (int i = 1; i < 7; ++i) s = fma(s, z, kSinPoly[i]);
  s = s * r;
  // cos(r + q pi/2) = cos r, -sin r, -cos r, sin r for q = 0, 1, 2, 3 (mod 4)
  const double v = (q & 1) ? s : c;
  return (((q + 1) & 2) != 0) ? -v : v;
}

}  // namespace fm
}  // namespace gm
