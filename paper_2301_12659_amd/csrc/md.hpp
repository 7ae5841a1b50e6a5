// Multiple-double arithmetic: double double (L=2), quad double (L=4) and
// octo double (L=8) numbers as unevaluated sums of L nonoverlapping doubles
// (Section 1.2).  Every routine takes its operands as limbs held in
// registers, never as arrays in memory, like the paper's inlined
// arithmetical kernels (Section 6); arrays in device memory are stored limb by
// limb (structure of arrays) by the callers.
//
// The error-free transformations must be evaluated exactly as written: this
// header turns floating-point contraction off and the library is compiled
// with -ffp-contract=off and without fast-math.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

#pragma clang fp contract(off)

#define MD_INLINE __host__ __device__ __forceinline__

namespace md {

// Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b).
MD_INLINE void two_sum(const double a, const double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Dekker's FastTwoSum, exact when the exponent of a is at least that of b.
MD_INLINE void fast_two_sum(const double a, const double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}

// TwoProd with one fused multiply-add: p + e == a * b exactly.
MD_INLINE void two_prod(const double a, const double b, double &p, double &e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

template <int L> struct MD;

#include "md_gen.inc"

template <int L> MD_INLINE void zero(double (&a)[L]) {
#pragma unroll
  for (int i = 0; i < L; ++i) a[i] = 0.0;
}

template <int L> MD_INLINE void copy(const double (&a)[L], double (&r)[L]) {
#pragma unroll
  for (int i = 0; i < L; ++i) r[i] = a[i];
}

template <int L> MD_INLINE void neg(const double (&a)[L], double (&r)[L]) {
#pragma unroll
  for (int i = 0; i < L; ++i) r[i] = -a[i];
}

// Multiplication by a power of two is exact limb by limb.
template <int L> MD_INLINE void scale2(double (&a)[L], const double p2) {
#pragma unroll
  for (int i = 0; i < L; ++i) a[i] *= p2;
}

// a times a small integer (the exponent of a variable in a monomial).
template <int L> MD_INLINE void mul_int(double (&a)[L], const int k) {
  if (k == 1) return;
  if (k == 2 || k == 4 || k == 8) {
    scale2<L>(a, (double)k);
    return;
  }
  double r[L];
  MD<L>::mul_d(a, (double)k, r);
  copy<L>(r, a);
}

// Quotient a / b by long division on the leading limb (L + 1 quotient digits,
// each the IEEE quotient of the current remainder by b's leading limb), then
// renormalization of the digits; the method of the quad-double library of
// Hida, Li and Bailey, applied to any L.
template <int L> MD_INLINE void div(const double (&a)[L], const double (&b)[L], double (&q)[L]) {
  double r[L], t[L], qd[L + 1];
  copy<L>(a, r);
#pragma unroll
  for (int k = 0; k <= L; ++k) {
    qd[k] = r[0] / b[0];
    if (k < L) {
      MD<L>::mul_d(b, qd[k], t);
      double s[L];
      MD<L>::sub(r, t, s);
      copy<L>(s, r);
    }
  }
  MD<L>::renorm_extra(qd, q);
}

// Square root by Newton's iteration y := y + (a - y^2) / (2 y) from the
// double square root of the leading limb; each step doubles the number of
// correct bits (53, 106, 212, 424), one extra step for safety.
template <int L> MD_INLINE void sqrt(const double (&a)[L], double (&y)[L]) {
  zero<L>(y);
  if (!(a[0] > 0.0)) {
    y[0] = (a[0] == 0.0) ? 0.0 : NAN;
    return;
  }
  y[0] = ::sqrt(a[0]);
  constexpr int iters = (L == 2) ? 2 : (L == 4) ? 3 : 4;
#pragma unroll
  for (int it = 0; it < iters; ++it) {
    double y2[L], d[L], two_y[L], c[L], yn[L];
    MD<L>::mul(y, y, y2);
    MD<L>::sub(a, y2, d);
    copy<L>(y, two_y);
    scale2<L>(two_y, 2.0);
    div<L>(d, two_y, c);
    MD<L>::add(y, c, yn);
    copy<L>(yn, y);
  }
}

}  // namespace md
