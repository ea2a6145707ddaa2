// Spin-weighted spherical harmonic -2Y_lm(theta, phi) on the device.
//
// In the Schwarzschild limit the spheroidal harmonic times e^{i m phi} of
// Eq. (1) becomes -2Y_lm(theta, phi) (Sec. IV), a per-request constant.  It is
// evaluated here through the Wigner small-d function,
//   -2Y_lm(theta, phi) = sqrt((2l+1)/(4 pi)) d^l_{m,2}(theta) e^{i m phi},
//   d^l_{m'm}(b) = sum_k (-1)^{k-m+m'} sqrt((l+m')!(l-m')!(l+m)!(l-m)!)
//                  / ((l+m-k)! k! (l-k-m')! (k-m+m')!)
//                  cos(b/2)^{2l-2k+m-m'} sin(b/2)^{2k-m+m'},
// which reproduces the standard convention
//   -2Y_22 = sqrt(5/(64 pi)) (1 + cos theta)^2 e^{2 i phi}.
// binary64; the alternating sum is well conditioned for the l <= 30 accepted.
#pragma once

#include <hip/hip_runtime.h>

__host__ __device__ inline double few_fact(int n) {
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= (double)k;
    return f;
}

__host__ __device__ inline double few_ipow(double x, int k) {
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

// Wigner small-d d^l_{mp,m}(beta) from its half-angle cosine and sine.
__host__ __device__ inline double few_wigner_d(int l, int mp, int m, double c, double s) {
    double norm = sqrt(few_fact(l + mp) * few_fact(l - mp) * few_fact(l + m) * few_fact(l - m));
    int k_lo = (m - mp) > 0 ? (m - mp) : 0;
    int k_hi = (l + m) < (l - mp) ? (l + m) : (l - mp);
    double sum = 0.0;
    for (int k = k_lo; k <= k_hi; ++k) {
        double den = few_fact(l + m - k) * few_fact(k) * few_fact(l - k - mp) * few_fact(k - m + mp);
        double term = few_ipow(c, 2 * l - 2 * k + m - mp) * few_ipow(s, 2 * k - m + mp) / den;
        sum += ((k - m + mp) & 1) ? -term : term;
    }
    return norm * sum;
}

// -2Y_lm(theta, phi); zero when |m| > l.
__host__ __device__ inline void few_swsh_m2(int l, int m, double theta, double phi,
                                            double *re, double *im) {
    if (m > l || -m > l || l < 2) {
        *re = 0.0;
        *im = 0.0;
        return;
    }
    const double inv_4pi = 0.07957747154594767;   // 1 / (4 pi)
    double c = cos(0.5 * theta), s = sin(0.5 * theta);
    double d = few_wigner_d(l, m, 2, c, s);
    double a = sqrt((2 * l + 1) * inv_4pi) * d;
    double sp, cp;
    sincos((double)m * phi, &sp, &cp);
    *re = a * cp;
    *im = a * sp;
}
