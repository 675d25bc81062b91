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
// cos(x): reduction by pi (three-part Cody-Waite with FMAs: pi carried in
//   three doubles, each product formed exactly inside an FMA; accurate while
//   |x| < 2^48, the range the kernels admit), |r| <= pi/2, cos(r) = C(r^2)
//   (degree 9 in r^2, max error 6.4e-21) evaluated as (1 - z/2) + z^2 Q(z)
//   with the rounding error of 1 - z/2 carried into the tail, sign (-1)^k.
//   No branch.  Measured error: <= 1.5 ulp of 1 absolute, <= 1 ulp relative
//   where |cos| >= 1/2; near the zeros of cos the relative error grows (the
//   rule sums are compared in absolute terms).
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
constexpr double kCosPoly[10] = {-0x1.5ca3b5d23666ap-53, 0x1.ae432cc0bd5d4p-45,
                                 -0x1.93969c9c98d05p-37, 0x1.1eed8dcee263bp-29,
                                 -0x1.27e4fb74f50a4p-22, 0x1.a01a01a0132f7p-16,
                                 -0x1.6c16c16c16b71p-10, 0x1.5555555555554p-5,
                                 -0x1.0000000000000p-1,  0x1.0000000000000p+0};
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kPi_1 = 0x1.921fb54442d18p+1;
constexpr double kPi_2 = 0x1.1a62633145c07p-53;
constexpr double kPi_3 = -0x1.f1976b7ed8fbcp-109;
constexpr double kInvPi = 0x1.45f306dc9c883p-2;
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
  const double t = fma(x, kInvPi, kShift);
  const double kd = t - kShift;
  const int32_t k = low_word(t);
  // r = x - k pi as rh + rl: the first step is exact (Cody-Waite), the
  // rounding error of the second is recovered with one more FMA.
  const double r1 = fma(-kd, kPi_1, x);
  const double rh = fma(-kd, kPi_2, r1);
  const double rl = fma(-kd, kPi_3, fma(-kd, kPi_2, r1 - rh));
  const double z = rh * rh;
  // cos r = (1 - z/2) + z^2 Q(z) - sin(rh) rl: the leading part is rounded
  // once and its rounding error is carried into the small tail.
  double q = kCosPoly[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) q = fma(q, z, kCosPoly[i]);
  const double hi = fma(z, -0.5, 1.0);
  const double lo = fma(-rh, rl, fma(z, -0.5, 1.0 - hi));
  const double c = hi + fma(z * z, q, lo);
  // cos(r + k pi) = (-1)^k cos r: bit 0 of k moved into the sign bit
#if defined(__HIP_DEVICE_COMPILE__)
  return __hiloint2double(__double2hiint(c) ^ (int)((uint32_t)k << 31), __double2loint(c));
#else
  uint32_t w[2];
  std::memcpy(w, &c, sizeof w);
  w[1] ^= (uint32_t)k << 31;
  double out;
  std::memcpy(&out, w, sizeof out);
  return out;
#endif
}

// 1/x: the hardware reciprocal estimate refined by two Newton steps
// e = 1 - x r, r += r e (each step squares the relative error), within 1 ulp
// for |x| in [2^-1022, 2^1022].  Outside that range (reciprocals beyond the
// normal range) the result may flush to 0 or be non-finite; x = 0 gives NaN.
// The host build starts from 1.0 / x.
GM_HD double rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
#else
  double r = 1.0 / x;
#endif
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  return r;
}

}  // namespace fm
}  // namespace gm
