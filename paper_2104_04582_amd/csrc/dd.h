// Double-double ("dd") arithmetic for the binary64 phase path.
//
// A dd value is an unevaluated sum hi + lo with |lo| <= ulp(hi)/2, giving
// about 106 significant bits.  The error-free transformations are the
// classical ones: Knuth's TwoSum, and TwoProd through a fused multiply-add.
// The phases of an EMRI reach 1e5-1e6 rad, and the harmonic index multiplies
// their error by up to |m| + |n| ~ 40, so the spline solve and the per-sample
// phase evaluation of the binary64 path run in dd; the result is reduced
// modulo 2 pi before anything is rounded to binary64.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

struct dd {
    double hi, lo;
};

// 2 pi as a double-double (hi = RN(2 pi), lo = RN(2 pi - hi)).
#define FEW_TWO_PI_HI 6.283185307179586232e+00
#define FEW_TWO_PI_LO 2.449293598294706414e-16
// RN(1 / (2 pi)): the quotient that picks the multiple of 2 pi.  A product
// instead of a division (a long dependent sequence on the GPU); the integer
// it rounds to can differ from that of the exact quotient only when the
// quotient is within a few ulps of a half-integer, and the remainder then
// still lies within [-pi, pi] up to those ulps.
#define FEW_INV_TWO_PI 1.591549430918953358e-01
// RN(2 / pi), for the choice of the quadrant.
#define FEW_TWO_OVER_PI 6.366197723675813431e-01

__host__ __device__ inline dd dd_make(double h, double l = 0.0) { return dd{h, l}; }

// Knuth TwoSum: s + e == a + b exactly.
__host__ __device__ inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd{s, e};
}

// Fast TwoSum, requires |a| >= |b|.
__host__ __device__ inline dd quick_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    return dd{s, e};
}

// TwoProd via FMA: p + e == a * b exactly.
__host__ __device__ inline dd two_prod(double a, double b) {
    double p = a * b;
    double e = fma(a, b, -p);
    return dd{p, e};
}

__host__ __device__ inline dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__host__ __device__ inline dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo = fma(a.hi, b.lo, p.lo);
    p.lo = fma(a.lo, b.hi, p.lo);
    return quick_two_sum(p.hi, p.lo);
}

__host__ __device__ inline dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo = fma(a.lo, b, p.lo);
    return quick_two_sum(p.hi, p.lo);
}

// a / b by one Newton correction of the binary64 quotient.
__host__ __device__ inline dd dd_div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, dd_make(q3));
}

// Reduce a to [-pi, pi] modulo 2 pi.  k = nearest integer of a / (2 pi);
// k * 2pi_hi is formed exactly with TwoProd, so the result carries only the
// rounding of the final dd additions.
__host__ __device__ inline dd dd_reduce_2pi(dd a) {
    double k = rint(a.hi * FEW_INV_TWO_PI);
    dd p = two_prod(k, FEW_TWO_PI_HI);
    dd r = dd_sub(a, p);
    r = dd_sub(r, dd_make(k * FEW_TWO_PI_LO, fma(k, FEW_TWO_PI_LO, -k * FEW_TWO_PI_LO)));
    // one more pass keeps the result in range when a.hi / 2pi rounded badly
    double k2 = rint(r.hi * FEW_INV_TWO_PI);
    if (k2 != 0.0) {
        r = dd_sub(r, two_prod(k2, FEW_TWO_PI_HI));
        r = dd_sub(r, dd_make(k2 * FEW_TWO_PI_LO));
    }
    return r;
}

// binary64 reduction to [-pi, pi] (for quantities already accurate only to
// binary64): a - k 2pi_hi by FMA, then - k 2pi_lo.
__host__ __device__ inline double d_reduce_2pi(double a) {
    double k = rint(a * FEW_INV_TWO_PI);
    double r = fma(-k, FEW_TWO_PI_HI, a);
    return fma(-k, FEW_TWO_PI_LO, r);
}

#pragma clang fp contract(on)
