// Log-sum-exp statistics in FP64 (the normalisation of eq. 2.4): a running
// maximum m and the sum s of exp(a - m) over the terms a seen so far.
//
// exp_nonpos(x) is exp(x) in FP64 for x <= 0, the only arguments such
// statistics produce.  The method is the classical
// range reduction of Cody and Waite: x = k ln 2 + r with k = rint(x / ln 2),
// so |r| <= ln 2 / 2, and e^x = 2^k e^r, with e^r from its Taylor series.
//
// * ln 2 is split into a 42-bit head and an FP64 tail; k needs at most 11 bits
//   here (|k| <= 1077 for x >= -746), so k * head is exact and r carries no
//   more than one rounding.
// * The series stops at degree 13: the remainder is below |r|^14 / 14! <
//   4.3e-18 of e^r, a twentieth of an FP64 unit.  Horner's scheme with
//   positive coefficients and |r| < 0.35 adds about one rounding.
// * Arguments below -746 are taken as -746, whose 2^k underflows to 0; so
//   -inf (an empty running maximum) gives 0.  NaN also gives 0: callers skip
//   non-finite terms before calling.
// * Subnormal results come from the hardware's exact scaling by 2^k.
//
// On the host the same arithmetic (std::fma) builds with a plain C++ compiler,
// for tests against a high-precision reference.
#pragma once

#include <cmath>

namespace emc {

// Taylor coefficients of exp_nonpos: c[i] = 1 / (13 - i)!, i = 0 .. 11 (each
// factorial is exact in FP64).  A kernel makes them once, before its loop; on
// the GPU the empty asm turns them into opaque values that stay in scalar
// registers (the compiler would otherwise re-create each constant, or copy it,
// before every multiply-add).
struct ExpCoef {
  double c[12];
};
__host__ __device__ __forceinline__ ExpCoef exp_coef() {
  ExpCoef e = {{1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0, 1.0 / 362880.0,
                1.0 / 40320.0, 1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5}};
#ifdef __HIP_DEVICE_COMPILE__
#pragma unroll
  for (int i = 0; i < 12; ++i) asm("" : "+s"(e.c[i]));
#endif
  return e;
}

// a * b + c with one rounding; on the GPU one v_fma_f64 that reads c from scalar
// registers (the compiler's own choice, a copy of c into the destination and
// v_fmac_f64, takes two instructions)
__host__ __device__ __forceinline__ double fma_coef(double a, double b, double c) {
#ifdef __HIP_DEVICE_COMPILE__
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
#else
  return fma(a, b, c);
#endif
}

__host__ __device__ __forceinline__ double exp_nonpos(double x, const ExpCoef& e) {
  constexpr double kLog2e = 0x1.71547652b82fep+0;   // 1 / ln 2
  constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;   // ln 2 rounded to 42 bits
  constexpr double kLn2Lo = 0x1.ef35793c76730p-45;  // ln 2 - kLn2Hi
  x = fmax(x, -746.0);
  const double k = rint(x * kLog2e);
  const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
  double p = fma_coef(e.c[0], r, e.c[1]);  // Horner from degree 13 down
#pragma unroll
  for (int i = 2; i < 12; ++i) p = fma_coef(p, r, e.c[i]);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

__host__ __device__ __forceinline__ double exp_nonpos(double x) { return exp_nonpos(x, exp_coef()); }

// Terms more than kLseDrop below the running maximum are not evaluated: each is
// below e^-64 = 1.6e-28 of the largest term, so all of them together (fewer than
// 2^31) stay below the FP64 rounding of a sum that is at least 1.
constexpr double kLseDrop = 64.0;

// (m, s) <- the statistics with term a added: one exponential, of the smaller of
// a and m measured from the larger (from m = -inf: s = 1, m = a).  NaN terms are
// skipped.
__host__ __device__ __forceinline__ void lse_push(double& m, double& s, double a, const ExpCoef& e) {
  if (a > m - kLseDrop) {
    const bool up = a > m;
    const double t = exp_nonpos(up ? m - a : a - m, e);
    s = up ? fma(s, t, 1.0) : s + t;
    m = up ? a : m;
  }
}

// (m, s) <- the statistics of the union of (m, s) and (m2, s2)
__host__ __device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
  if (m2 > m) {
    s = fma(s, exp_nonpos(m - m2), s2);
    m = m2;
  } else if (m2 > -INFINITY) {
    s = fma(s2, exp_nonpos(m2 - m), s);
  }
}

}  // namespace emc
