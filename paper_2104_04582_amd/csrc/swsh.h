// Spin-weighted spherical harmonic -2Y_lm(theta, phi) on the device.
//
// In the Schwarzschild limit the spheroidal harmonic times e^{i m phi} of
// Eq. (1) becomes -2Y_lm(theta, phi) (Sec. IV), a per-request constant; the
// generic-Kerr spherical projection (Sec. VII) uses the same functions.  It is
// evaluated through the Wigner small-d function,
//   -2Y_lm(theta, phi) = sqrt((2l+1)/(4 pi)) d^l_{m,2}(theta) e^{i m phi},
// which reproduces the standard convention
//   -2Y_22 = sqrt(5/(64 pi)) (1 + cos theta)^2 e^{2 i phi}.
// d is written through a Jacobi polynomial (mu = |m - m'|, nu = |m + m'|,
// n = l - (mu + nu) / 2):
//   d^l_{m',m}(b) = xi sqrt(n! (n+mu+nu)! / ((n+mu)! (n+nu)!))
//                   sin(b/2)^mu cos(b/2)^nu P_n^{(mu,nu)}(cos b),
// xi = 1 for m >= m', else (-1)^{m-m'}, and P_n is formed by its three-term
// recurrence in the degree, which is stable on [-1, 1].  (The explicit
// alternating sum over k cancels by ~1e-9 of its largest term at l = 30.)
#pragma once

#include <hip/hip_runtime.h>

__host__ __device__ inline double few_ipow(double x, int k) {
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

// Wigner small-d d^l_{mp,m}(b) from its half-angle cosine c and sine s.  The
// factorial ratio n! (n+mu+nu)! / ((n+mu)! (n+nu)!) is taken as
// prod_{k=1..mu} (n+nu+k) / (n+k), and each step of the degree recurrence
// multiplies by the reciprocal of its leading factor (formed off the
// recurrence's dependent chain).
__host__ __device__ inline double few_wigner_d(int l, int mp, int m, double c, double s) {
    const int mu = m > mp ? m - mp : mp - m;
    const int nu = m + mp > 0 ? m + mp : -(m + mp);
    const int n = l - (mu + nu) / 2;
    const double x = c * c - s * s;                     // cos b
    const double a = mu, b = nu;
    double p0 = 1.0, p = 1.0;
    if (n >= 1) {
        double p1 = (a + 1.0) + 0.5 * (a + b + 2.0) * (x - 1.0);
        for (int k = 2; k <= n; ++k) {
            const double t = 2.0 * k + a + b;
            const double c1 = 2.0 * k * (k + a + b) * (t - 2.0);
            const double c2 = (t - 1.0) * (t * (t - 2.0) * x + a * a - b * b);
            const double c3 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * t;
            const double ic1 = 1.0 / c1;
            const double pk = (c2 * p1 - c3 * p0) * ic1;
            p0 = p1;
            p1 = pk;
        }
        p = p1;
    }
    const double xi = (m >= mp || ((m - mp) & 1) == 0) ? 1.0 : -1.0;
    double num = 1.0, den = 1.0;
    for (int k = 1; k <= mu; ++k) {
        num *= (double)(n + nu + k);
        den *= (double)(n + k);
    }
    const double norm = sqrt(num / den);
    return xi * norm * few_ipow(s, mu) * few_ipow(c, nu) * p;
}

// -2Y_lm(theta, phi) from c = cos(theta/2), s = sin(theta/2) and
// (cos m phi, sin m phi); zero when |m| > l or l < 2.
__host__ __device__ inline void few_swsh_m2_cs(int l, int m, double c, double s, double cmp,
                                               double smp, double *re, double *im) {
    if (m > l || -m > l || l < 2) {
        *re = 0.0;
        *im = 0.0;
        return;
    }
    const double inv_4pi = 0.07957747154594767;   // 1 / (4 pi)
    const double d = few_wigner_d(l, m, 2, c, s);
    const double a = sqrt((2 * l + 1) * inv_4pi) * d;
    *re = a * cmp;
    *im = a * smp;
}

// -2Y_lm(theta, phi); zero when |m| > l.
__host__ __device__ inline void few_swsh_m2(int l, int m, double theta, double phi,
                                            double *re, double *im) {
    if (m > l || -m > l || l < 2) {
        *re = 0.0;
        *im = 0.0;
        return;
    }
    double sp, cp;
    sincos((double)m * phi, &sp, &cp);
    few_swsh_m2_cs(l, m, cos(0.5 * theta), sin(0.5 * theta), cp, sp, re, im);
}
