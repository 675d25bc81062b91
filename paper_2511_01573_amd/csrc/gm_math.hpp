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
#if defined(__HIPCC__)
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
// sin r = r (1 + z Q(z)), z = r^2 <= (pi/2)^2
constexpr double kSinPoly[9] = {-0x1.275f3132d0bb5p-57, 0x1.9507ff1d2eab1p-49,
                                -0x1.ae7ee3a7e62e7p-41, 0x1.612460b6ab17ep-33,
                                -0x1.ae64567e733b7p-26, 0x1.71de3a556b9b6p-19,
                                -0x1.a01a01a01a00dp-13, 0x1.1111111111111p-7,
                                -0x1.5555555555555p-3};
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

// N-wide forms: the same operations on N independent arguments, written
// step by step across the N values so the dependent FMA chains of neighbouring
// nodes interleave (each element gets exactly the scalar function's result).
template <int N>
GM_HD void exp_n(const double (&xin)[N], double (&y)[N]) {
  double x[N], t[N], kd[N], r[N], p[N];
  int32_t k[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x[i] = fmax(xin[i], -1100.0);
    t[i] = fma(x[i], kInvLn2, kShift);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    kd[i] = t[i] - kShift;
    k[i] = low_word(t[i]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = fma(-kd[i], kLn2Hi, x[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = fma(-kd[i], kLn2Lo, r[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = kExpPoly[0];
#pragma unroll
  for (int c = 1; c < 12; ++c) {
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = fma(p[i], r[i], kExpPoly[c]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) y[i] = ldexp(p[i], k[i]);
}

template <int N>
GM_HD void cos_n(const double (&x)[N], double (&y)[N]) {
  double t[N], kd[N], r1[N], rh[N], rl[N], z[N], q[N], hi[N], lo[N], c[N];
  int32_t k[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    t[i] = fma(x[i], kInvPi, kShift);
    kd[i] = t[i] - kShift;
    k[i] = low_word(t[i]);
  }
  // r = x - k pi as rh + rl: the first step is exact (Cody-Waite), the
  // rounding error of the second is recovered with one more FMA.
#pragma unroll
  for (int i = 0; i < N; ++i) r1[i] = fma(-kd[i], kPi_1, x[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) rh[i] = fma(-kd[i], kPi_2, r1[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) rl[i] = fma(-kd[i], kPi_3, fma(-kd[i], kPi_2, r1[i] - rh[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) {
    z[i] = rh[i] * rh[i];
    q[i] = kCosPoly[0];
  }
  // cos r = (1 - z/2) + z^2 Q(z) - sin(rh) rl: the leading part is rounded
  // once and its rounding error is carried into the small tail.
#pragma unroll
  for (int cc = 1; cc < 8; ++cc) {
#pragma unroll
    for (int i = 0; i < N; ++i) q[i] = fma(q[i], z[i], kCosPoly[cc]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    hi[i] = fma(z[i], -0.5, 1.0);
    lo[i] = fma(-rh[i], rl[i], fma(z[i], -0.5, 1.0 - hi[i]));
    c[i] = hi[i] + fma(z[i] * z[i], q[i], lo[i]);
  }
  // cos(r + k pi) = (-1)^k cos r: bit 0 of k moved into the sign bit
#pragma unroll
  for (int i = 0; i < N; ++i) {
#if defined(__HIP_DEVICE_COMPILE__)
    y[i] = __hiloint2double(__double2hiint(c[i]) ^ (int)((uint32_t)k[i] << 31),
                            __double2loint(c[i]));
#else
    uint32_t w[2];
    std::memcpy(w, &c[i], sizeof w);
    w[1] ^= (uint32_t)k[i] << 31;
    std::memcpy(&y[i], w, sizeof w);
#endif
  }
}

// sin x with the reduction of cos_n: x = r + k pi, r = rh + rl, sin x =
// (-1)^k sin r, sin r = rh + (rh z Q(z) + rl (1 - z/2)) with z = rh^2 (the
// first-order term of rl; its square is below 2^-100 |x|^2).
template <int N>
GM_HD void sin_n(const double (&x)[N], double (&y)[N]) {
  double t[N], kd[N], r1[N], rh[N], rl[N], z[N], q[N], s[N];
  int32_t k[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    t[i] = fma(x[i], kInvPi, kShift);
    kd[i] = t[i] - kShift;
    k[i] = low_word(t[i]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) r1[i] = fma(-kd[i], kPi_1, x[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) rh[i] = fma(-kd[i], kPi_2, r1[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) rl[i] = fma(-kd[i], kPi_3, fma(-kd[i], kPi_2, r1[i] - rh[i]));
#pragma unroll
  for (int i = 0; i < N; ++i) {
    z[i] = rh[i] * rh[i];
    q[i] = kSinPoly[0];
  }
#pragma unroll
  for (int cc = 1; cc < 9; ++cc) {
#pragma unroll
    for (int i = 0; i < N; ++i) q[i] = fma(q[i], z[i], kSinPoly[cc]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    s[i] = rh[i] + fma(rh[i] * z[i], q[i], rl[i] * fma(z[i], -0.5, 1.0));
#pragma unroll
  for (int i = 0; i < N; ++i) {
#if defined(__HIP_DEVICE_COMPILE__)
    y[i] = __hiloint2double(__double2hiint(s[i]) ^ (int)((uint32_t)k[i] << 31),
                            __double2loint(s[i]));
#else
    uint32_t w[2];
    std::memcpy(w, &s[i], sizeof w);
    w[1] ^= (uint32_t)k[i] << 31;
    std::memcpy(&y[i], w, sizeof w);
#endif
  }
}

// 1/x: the hardware reciprocal estimate refined by two Newton steps
// e = 1 - x r, r += r e (each step squares the relative error), within 1 ulp
// for |x| in [2^-1022, 2^1022].  Outside that range (reciprocals beyond the
// normal range) the result may flush to 0 or be non-finite; x = 0 gives NaN.
// The host build starts from 1.0 / x.
template <int N>
GM_HD void rcp_n(const double (&x)[N], double (&y)[N]) {
  double r[N], e[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#if defined(__HIP_DEVICE_COMPILE__)
    r[i] = __builtin_amdgcn_rcp(x[i]);
#else
    r[i] = 1.0 / x[i];
#endif
  }
#pragma unroll
  for (int i = 0; i < N; ++i) e[i] = fma(-x[i], r[i], 1.0);
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = fma(r[i], e[i], r[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) e[i] = fma(-x[i], r[i], 1.0);
#pragma unroll
  for (int i = 0; i < N; ++i) y[i] = fma(r[i], e[i], r[i]);
}

GM_HD double exp(double x) {
  const double a[1] = {x};
  double y[1];
  exp_n<1>(a, y);
  return y[0];
}

GM_HD double cos(double x) {
  const double a[1] = {x};
  double y[1];
  cos_n<1>(a, y);
  return y[0];
}

GM_HD double sin(double x) {
  const double a[1] = {x};
  double y[1];
  sin_n<1>(a, y);
  return y[0];
}

GM_HD double rcp(double x) {
  const double a[1] = {x};
  double y[1];
  rcp_n<1>(a, y);
  return y[0];
}

}  // namespace fm
}  // namespace gm
