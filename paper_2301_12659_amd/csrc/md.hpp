// Multiple-double arithmetic: double double (L=2), quad double (L=4) and
// octo double (L=8) numbers as unevaluated sums of L nonoverlapping doubles
// (Section 1.2); L=1 is plain double arithmetic (the paper's precision D in
// its comparisons across precisions, Section 7).  Every routine takes its operands as limbs held in
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
  if constexpr (L == 1) {  // plain double: the IEEE quotient
    q[0] = a[0] / b[0];
    return;
  }
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
  constexpr int iters = (L == 1) ? 0 : (L == 2) ? 2 : (L == 4) ? 3 : 4;
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

// Leading P limbs of an L-limb expansion (its truncation, within about
// 2^(-53 P) relatively), and the way back with zero limbs.
template <int P, int L>
MD_INLINE void head(const double (&a)[L], double (&h)[P]) {
#pragma unroll
  for (int i = 0; i < P; ++i) h[i] = a[i];
}
template <int P, int L>
MD_INLINE void widen(const double (&h)[P], double (&a)[L]) {
#pragma unroll
  for (int i = 0; i < L; ++i) a[i] = (i < P) ? h[i] : 0.0;
}

// c = x e at H limbs (H = 1: one double multiplication), widened to P limbs.
template <int P, int H>
MD_INLINE void correction(const double (&x)[P], const double (&e)[P], double (&c)[P]) {
  if constexpr (H == 1) {
    zero<P>(c);
    c[0] = x[0] * e[0];
  } else {
    double xh[H], eh[H], ch[H];
    head<H>(x, xh);
    head<H>(e, eh);
    MD<H>::mul(xh, eh, ch);
    widen<H>(ch, c);
  }
}

// Newton steps for 1/sqrt(a) and 1/v with precision doubling.  A step
// y := y + y (1 - a y^2) / 2 (or r := r + r (1 - v r)) doubles the number of
// correct bits, so the step that brings y from P/2 to P correct limbs runs at
// P limbs; its residual 1 - a y^2 is below about 2^(-26.5 P), so the
// correction y (1 - a y^2) / 2 needs only H = P/2 limbs of it, provided the
// residual's leading H limbs are its leading H * 53 bits.  The sums here
// leave zero limbs inside an expansion after a deep cancellation (a zero
// limb 1 or 2 followed by significant ones), so a truncated residual can
// hold fewer bits: at 2 and 4 limbs the last step below repairs that, at 8
// limbs the correction is taken at full width.  After the doublings (53
// bits from the double start, then 2, 4, 8 limbs) a last step at L limbs
// with a one-limb correction brings the result to a few units in its last
// limb.
template <int L, int P, int H>
MD_INLINE void rsqrt_step(const double (&a)[L], double (&y)[L]) {
  double ap[P], yp[P], t[P], u[P], e[P], c[P], one[P];
  head<P>(a, ap);
  head<P>(y, yp);
  zero<P>(one);
  one[0] = 1.0;
  MD<P>::mul(yp, yp, t);
  MD<P>::mul(ap, t, u);
  MD<P>::sub(one, u, e);
  correction<P, H>(yp, e, c);
  scale2<P>(c, 0.5);
  MD<P>::add(yp, c, t);
  widen<P>(t, y);
}

template <int L, int P, int H>
MD_INLINE void recip_step(const double (&v)[L], double (&r)[L]) {
  double vp[P], rp[P], t[P], e[P], c[P], one[P];
  head<P>(v, vp);
  head<P>(r, rp);
  zero<P>(one);
  one[0] = 1.0;
  MD<P>::mul(vp, rp, t);
  MD<P>::sub(one, t, e);
  correction<P, H>(rp, e, c);
  MD<P>::add(rp, c, t);
  widen<P>(t, r);
}

template <int L>
MD_INLINE void rsqrt_newton(const double (&a)[L], double (&y)[L]) {
  zero<L>(y);
  y[0] = 1.0 / ::sqrt(a[0]);
  if constexpr (L == 1) return;  // plain double
  rsqrt_step<L, 2, 1>(a, y);
  if constexpr (L >= 4) rsqrt_step<L, 4, 2>(a, y);
  if constexpr (L >= 8) rsqrt_step<L, 8, 8>(a, y);
  rsqrt_step<L, L, 1>(a, y);
}

template <int L>
MD_INLINE void recip_newton(const double (&v)[L], double (&r)[L]) {
  zero<L>(r);
  r[0] = 1.0 / v[0];
  if constexpr (L == 1) return;  // plain double
  recip_step<L, 2, 1>(v, r);
  if constexpr (L >= 4) recip_step<L, 4, 2>(v, r);
  if constexpr (L >= 8) recip_step<L, 8, 8>(v, r);
  recip_step<L, L, 1>(v, r);
}

// The last doubling of quad doubles with the residual formed by one fused
// multiply-subtract (1 - (a y) y, or 1 - v r) and renormalized a second
// time, which moves significant bits into any zero limb that a deep
// cancellation left inside it: its leading two limbs are then its leading
// 106 bits, all that the correction, itself about 2^(-106) of the result,
// needs; the correction is taken at two limbs.
MD_INLINE void rsqrt_last4(const double (&a)[4], double (&y)[4]) {
  double t[4], e[4] = {1.0, 0.0, 0.0, 0.0}, en[4], yn[4];
  MD<4>::mul(a, y, t);
  MD<4>::fms(e, t, y);
  MD<4>::renorm(e, en);
  const double yh[2] = {y[0], y[1]}, eh[2] = {en[0], en[1]};
  double ch[2];
  MD<2>::mul(yh, eh, ch);
  const double c[4] = {0.5 * ch[0], 0.5 * ch[1], 0.0, 0.0};
  MD<4>::add(y, c, yn);
  copy<4>(yn, y);
}

MD_INLINE void recip_last4(const double (&v)[4], double (&r)[4]) {
  double e[4] = {1.0, 0.0, 0.0, 0.0}, en[4], rn[4];
  MD<4>::fms(e, v, r);
  MD<4>::renorm(e, en);
  const double rh[2] = {r[0], r[1]}, eh[2] = {en[0], en[1]};
  double ch[2];
  MD<2>::mul(rh, eh, ch);
  const double c[4] = {ch[0], ch[1], 0.0, 0.0};
  MD<4>::add(r, c, rn);
  copy<4>(rn, r);
}

// The same doublings with every correction at full width and no repair
// step, for double and quad doubles: the residual is never truncated, so a
// zero limb inside it costs nothing, and the last doubling leaves a relative
// error of about 2^(-53 L + 6) instead of a few units in the last limb, for
// one full-precision step less; for quad doubles the last doubling is
// rsqrt_last4 / recip_last4.  Used where the result is on a chain of
// dependent operations (the reflector of a Householder step).  Octo doubles
// keep the full sequence (a shortened one would stop near 2^(-412)).
template <int L>
MD_INLINE void rsqrt_short(const double (&a)[L], double (&y)[L]) {
  if constexpr (L == 1) {
    y[0] = 1.0 / ::sqrt(a[0]);
  } else if constexpr (L >= 8) {
    rsqrt_newton<L>(a, y);
  } else {
    zero<L>(y);
    y[0] = 1.0 / ::sqrt(a[0]);
    rsqrt_step<L, 2, (L == 2 ? 2 : 1)>(a, y);
    if constexpr (L == 4) rsqrt_last4(a, y);
  }
}

template <int L>
MD_INLINE void recip_short(const double (&v)[L], double (&r)[L]) {
  if constexpr (L == 1) {
    r[0] = 1.0 / v[0];
  } else if constexpr (L >= 8) {
    recip_newton<L>(v, r);
  } else {
    zero<L>(r);
    r[0] = 1.0 / v[0];
    recip_step<L, 2, (L == 2 ? 2 : 1)>(v, r);
    if constexpr (L == 4) recip_last4(v, r);
  }
}

}  // namespace md
