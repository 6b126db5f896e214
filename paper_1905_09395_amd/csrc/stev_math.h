// FP64 exp and log from small tables, and division through the hardware
// reciprocal: the arithmetic the integration kernels share.  The tables
// (kXtabBytes, filled on the host by fill_xtab) sit in LDS; each function
// takes their base address.
#pragma once

#include <hip/hip_runtime.h>

#include "stev_internal.h"

namespace stev {

// exp in FP64: x = (64 k + j) ln2/64 + r with |r| <= ln2/128 (Cody-Waite
// split of ln2/64, the high part exact for any product with n), so
// e^x = 2^k 2^(j/64) (1 + p(r)), 2^(j/64) from the table as hi + lo and
// p(r) = e^r - 1 from its Taylor series through r^6 (truncation < 2^-58).
// Arguments are clamped to [-1e4, 1e4], which leaves 0 and inf where they
// belong; a NaN argument comes out as 0 (every NaN input to the kernel also
// reaches the state through other terms and fails the cell there).
constexpr double kExpInvL = 0x1.71547652b82fep+6;   // 64 / ln 2
constexpr double kLn2Hi = 0x1.62e42p-1;             // ln 2, 20 significant bits
constexpr double kLn2Lo = 0x1.fdf473de6af28p-22;    // ln 2 - kLn2Hi
__device__ __forceinline__ double exp_tab(const double *t, double x) {
  x = fmin(fmax(x, -1.0e4), 1.0e4);
  const double n = rint(x * kExpInvL);
  const int ni = (int)n;
  const double r = fma(-n, kLn2Lo / kExpTab, fma(-n, kLn2Hi / kExpTab, x));
  double p = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  p = fma(r, p, 1.0 / 24.0);
  p = fma(r, p, 1.0 / 6.0);
  p = fma(r, p, 0.5);
  p = fma(r * r, p, r);
  const int j = ni & (kExpTab - 1);
  const double th = t[2 * j], tl = t[2 * j + 1];
  return ldexp(fma(th, p, tl) + th, ni >> 6);
}
// log in FP64: x = 2^e m with m in [1, 2) and j the top five fraction bits
// of m; with ic from the table, r = m ic - 1 carries a single rounding and
// |r| < 1/64, and log x = e ln2 - log(ic) + log1p(r), log1p from its series
// through r^8 (truncation < 2^-56).  The special arguments are selected,
// not branched to: 0 gives -inf, +inf gives +inf, negatives and NaN give NaN.
// A branch here opens a region that runs with part of the wavefront masked
// off, and the register allocator has been seen to place copies of values
// that live across the whole loop (the per-lane statistics) inside such a
// region, so lanes holding a bad temperature lost them.
__device__ __forceinline__ double log_tab(const double *xt, double x) {
  const double *t = xt + 2 * kExpTab;
  int e;
  const double m = 2.0 * frexp(x, &e);
  const int j = (__double2hiint(m) >> 15) & (kLogTab - 1);
  const double ic = t[3 * j], lh = t[3 * j + 1], ll = t[3 * j + 2];
  const double r = fma(m, ic, -1.0);
  double q = fma(r, -1.0 / 8.0, 1.0 / 7.0);
  q = fma(r, q, -1.0 / 6.0);
  q = fma(r, q, 1.0 / 5.0);
  q = fma(r, q, -0.25);
  q = fma(r, q, 1.0 / 3.0);
  q = fma(r, q, -0.5);
  const double de = (double)(e - 1);
  const double res = fma(de, kLn2Hi, lh) + (fma(r * r, q, r) + fma(de, kLn2Lo, ll));
  const double sp = (x == 0.0) ? -__builtin_inf() : ((x > 0.0) ? x : __builtin_nan(""));
  return (x > 0.0 && x < __builtin_inf()) ? res : sp;
}

// a / b from the hardware reciprocal: Newton steps on 1/b, then one
// correction of the quotient by its exact remainder (an FMA).  The result
// is within an ulp of the IEEE quotient and equal to it in nearly every
// case; a zero, infinite or NaN divisor gives a non-finite result.
__device__ __forceinline__ double qdiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}
__device__ __forceinline__ float qdiv(float a, float b) {
  float r = __builtin_amdgcn_rcpf(b);
  r = fmaf(fmaf(-b, r, 1.0f), r, r);
  const float q = a * r;
  return fmaf(fmaf(-b, q, a), r, q);
}

}  // namespace stev
