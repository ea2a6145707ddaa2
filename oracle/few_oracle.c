/*
 * CPU ORACLE for the interpolated harmonic-mode summation -- TEST
 * INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes (paper Sec. III C "Waveform Summation Module" and Sec. IV,
 * Eq. (10)):
 *
 *   h(t_j) = scale * sum_{listed (l,m,n)} [ A_lmn(t_j) Y+_lm
 *                                          + [m>0] conj(A_lmn(t_j)) Y-_lm ]
 *                                        * e^{-i (m Phi_phi(t_j) + n Phi_r(t_j))}
 *
 * with the negative-m modes supplied by the amplitude symmetry of Eq. (9)
 * (k = 0 in Schwarzschild): A_{l,-m,-n} = (-1)^l conj(A_lmn), so the mirror
 * mode contributes (-1)^l conj(A) Y_{l,-m} e^{+i(m Phi_phi + n Phi_r)}.
 * Y+_lm = -2Y_lm(theta, phi), Y-_lm = (-1)^l -2Y_{l,-m}(theta, phi).
 *
 * Every time series (Phi_phi, Phi_r, Re A, Im A of each mode) is a not-a-knot
 * cubic spline on the shared sparse knot grid (Sec. III C).  Samples sit on
 * t_j = t_start + j dt, evaluated in IEEE binary64 exactly as written.
 *
 * Precision: x87 extended ("long double", 64-bit significand) throughout, with
 * the phase constant of each knot interval reduced modulo 2 pi in binary128 and
 * the alternating sum of each spin-weighted harmonic formed in binary128.
 * Adding a multiple of 2 pi to a phase leaves e^{-i(m Phi_phi + n Phi_r)}
 * unchanged for integer m, n, so the reduction is an identity, not an
 * approximation.  Binary64 here would put the oracle's own phase error
 * (~1e-12 rad at 5e5 rad of accumulated phase) near the tolerance it is used
 * to check.
 *
 * Generic-Kerr spherical-projected sum (Sec. VII, Eq. (spherical projection)
 * of the waveform, with the amplitude symmetry of Eq. (9) for general k):
 *
 *   h = scale * sum_{listed (l,m,k,n)} [ A Y+_lm + [m>0] conj(A) Y-_lmk ]
 *                                     * e^{-i (m Phi_phi + k Phi_theta + n Phi_r)}
 *
 * with A_{l,-m,-k,-n} = (-1)^{l+k} conj(A_lmkn), i.e. Y-_lmk = (-1)^{l+k}
 * -2Y_{l,-m}; a third phase Phi_theta is splined like the other two.  The
 * Schwarzschild sum above is the case k = 0 without Phi_theta.
 *
 * Plain and slow on purpose: dense LU with partial pivoting for the spline
 * system, a binary search per sample, libm sincosl per mode and sample,
 * Neumaier-compensated accumulation.  OpenMP over samples only.
 */
#define _GNU_SOURCE
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

/* Status codes of this library (its own; unrelated to the GPU library's). */
#define OR_OK 0
#define OR_E_ARG -1
#define OR_E_KNOTS -2
#define OR_E_MODES -3
#define OR_E_RANGE -4
#define OR_E_NOMEM -6

/* ------------------------------------------------------------------------ */
/* Not-a-knot cubic spline (Sec. III C).                                    */
/*                                                                          */
/* On [t_i, t_{i+1}] with x = t - t_i, h_i = t_{i+1} - t_i and              */
/* delta_i = (y_{i+1} - y_i) / h_i, the cubic with end values y_i, y_{i+1}  */
/* and end slopes s_i, s_{i+1} is                                           */
/*   y_i + s_i x + c_i x^2 + d_i x^3,                                       */
/*   c_i = (3 delta_i - 2 s_i - s_{i+1}) / h_i,                              */
/*   d_i = (s_i + s_{i+1} - 2 delta_i) / h_i^2.                              */
/* Continuity of the second derivative at the interior knots t_1..t_{K-2}   */
/* gives, for i = 1..K-2,                                                   */
/*   h_i s_{i-1} + 2 (h_{i-1} + h_i) s_i + h_{i-1} s_{i+1}                  */
/*       = 3 (h_i delta_{i-1} + h_{i-1} delta_i).                            */
/* The not-a-knot conditions make the third derivative continuous at t_1    */
/* and t_{K-2} (d_0 = d_1, d_{K-3} = d_{K-2}).  Eliminating s_2 (resp.      */
/* s_{K-3}) between that condition and the neighbouring continuity row      */
/* gives the two end rows:                                                  */
/*   h_1 s_0 + (h_0 + h_1) s_1                                              */
/*       = [(h_0 + 2 (h_0 + h_1)) h_1 delta_0 + h_0^2 delta_1] / (h_0 + h_1) */
/*   (h_{K-2} + h_{K-3}) s_{K-2} + h_{K-3} s_{K-1}                           */
/*       = [h_{K-2}^2 delta_{K-3}                                           */
/*          + (2 (h_{K-3} + h_{K-2}) + h_{K-2}) h_{K-3} delta_{K-2}]         */
/*         / (h_{K-3} + h_{K-2})                                             */
/* K >= 4 is required (with K = 4 the spline is the single interpolating    */
/* cubic).                                                                  */
/* ------------------------------------------------------------------------ */

/* Dense K x K matrix of the slope system (row-major), built from the knots. */
static void slope_matrix(int K, const ld *h, ld *A) {
    memset(A, 0, sizeof(ld) * (size_t)K * K);
    A[0 * K + 0] = h[1];
    A[0 * K + 1] = h[0] + h[1];
    for (int i = 1; i <= K - 2; ++i) {
        A[i * K + i - 1] = h[i];
        A[i * K + i] = 2.0L * (h[i - 1] + h[i]);
        A[i * K + i + 1] = h[i - 1];
    }
    A[(K - 1) * K + K - 2] = h[K - 2] + h[K - 3];
    A[(K - 1) * K + K - 1] = h[K - 3];
}

static void slope_rhs(int K, const ld *h, const ld *dl, ld *r) {
    r[0] = ((h[0] + 2.0L * (h[0] + h[1])) * h[1] * dl[0] + h[0] * h[0] * dl[1]) /
           (h[0] + h[1]);
    for (int i = 1; i <= K - 2; ++i) r[i] = 3.0L * (h[i] * dl[i - 1] + h[i - 1] * dl[i]);
    r[K - 1] = (h[K - 2] * h[K - 2] * dl[K - 3] +
                (2.0L * (h[K - 3] + h[K - 2]) + h[K - 2]) * h[K - 3] * dl[K - 2]) /
               (h[K - 3] + h[K - 2]);
}

/* In-place LU factorisation with partial (row) pivoting; piv[i] = source row. */
static void lu_factor(int K, ld *A, int *piv) {
    for (int i = 0; i < K; ++i) piv[i] = i;
    for (int c = 0; c < K; ++c) {
        int p = c;
        ld best = fabsl(A[c * K + c]);
        for (int r = c + 1; r < K; ++r) {
            ld v = fabsl(A[r * K + c]);
            if (v > best) { best = v; p = r; }
        }
        if (p != c) {
            for (int k = 0; k < K; ++k) {
                ld tmp = A[c * K + k]; A[c * K + k] = A[p * K + k]; A[p * K + k] = tmp;
            }
            int tp = piv[c]; piv[c] = piv[p]; piv[p] = tp;
        }
        for (int r = c + 1; r < K; ++r) {
            ld f = A[r * K + c] / A[c * K + c];
            A[r * K + c] = f;
            for (int k = c + 1; k < K; ++k) A[r * K + k] -= f * A[c * K + k];
        }
    }
}

static void lu_solve(int K, const ld *LU, const int *piv, const ld *b, ld *x) {
    for (int i = 0; i < K; ++i) {              /* forward: L z = P b */
        ld s = b[piv[i]];
        for (int k = 0; k < i; ++k) s -= LU[i * K + k] * x[k];
        x[i] = s;
    }
    for (int i = K - 1; i >= 0; --i) {         /* backward: U x = z */
        ld s = x[i];
        for (int k = i + 1; k < K; ++k) s -= LU[i * K + k] * x[k];
        x[i] = s / LU[i * K + i];
    }
}

static int check_knots(int K, const double *t) {
    if (K < 4) return OR_E_KNOTS;
    for (int i = 0; i < K; ++i)
        if (!isfinite(t[i])) return OR_E_KNOTS;
    for (int i = 0; i + 1 < K; ++i)
        if (!(t[i + 1] > t[i])) return OR_E_KNOTS;
    return OR_OK;
}

/* Spline coefficients of S series given knot-major values y[i * S + s].
 * out[(i * S + s) * 4 + p] = coefficient of x^p on interval i (long double). */
static int spline_ld(int K, const double *t, int S, const double *y, ld *out) {
    int rc = check_knots(K, t);
    if (rc) return rc;
    ld *h = malloc(sizeof(ld) * K), *dl = malloc(sizeof(ld) * K);
    ld *A = malloc(sizeof(ld) * (size_t)K * K), *r = malloc(sizeof(ld) * K);
    ld *s = malloc(sizeof(ld) * K);
    int *piv = malloc(sizeof(int) * K);
    if (!h || !dl || !A || !r || !s || !piv) {
        free(h); free(dl); free(A); free(r); free(s); free(piv);
        return OR_E_NOMEM;
    }
    for (int i = 0; i + 1 < K; ++i) h[i] = (ld)t[i + 1] - (ld)t[i];
    slope_matrix(K, h, A);
    lu_factor(K, A, piv);
    for (int q = 0; q < S; ++q) {
        for (int i = 0; i + 1 < K; ++i)
            dl[i] = ((ld)y[(size_t)(i + 1) * S + q] - (ld)y[(size_t)i * S + q]) / h[i];
        slope_rhs(K, h, dl, r);
        lu_solve(K, A, piv, r, s);
        for (int i = 0; i + 1 < K; ++i) {
            ld *o = out + ((size_t)i * S + q) * 4;
            o[0] = (ld)y[(size_t)i * S + q];
            o[1] = s[i];
            o[2] = (3.0L * dl[i] - 2.0L * s[i] - s[i + 1]) / h[i];
            o[3] = (s[i] + s[i + 1] - 2.0L * dl[i]) / (h[i] * h[i]);
        }
    }
    free(h); free(dl); free(A); free(r); free(s); free(piv);
    return OR_OK;
}

/* Exported for the spline pins: coefficients rounded to binary64. */
int few_oracle_spline(int K, const double *t, int S, const double *y, double *out) {
    if (!t || !y || !out || S < 1) return OR_E_ARG;
    ld *tmp = malloc(sizeof(ld) * (size_t)(K > 1 ? K - 1 : 1) * S * 4);
    if (!tmp) return OR_E_NOMEM;
    int rc = spline_ld(K, t, S, y, tmp);
    if (rc == OR_OK)
        for (size_t k = 0; k < (size_t)(K - 1) * S * 4; ++k) out[k] = (double)tmp[k];
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Spin-weighted spherical harmonics sY_lm(theta, phi) (Sec. III D, Sec. IV: */
/* the Schwarzschild limit of S_lmkn e^{i m phi}).  Goldberg et al.'s       */
/* explicit sum:                                                            */
/*   sY_lm = (-1)^m sqrt[(l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!)]           */
/*           sin^{2l}(theta/2)                                              */
/*           sum_r C(l-s, r) C(l+s, r+s-m) (-1)^{l-r-s}                     */
/*                 e^{i m phi} cot^{2r+s-m}(theta/2)                        */
/* The power of cot is k = 2r+s-m >= 0 and 2l - k >= 0 for every r in the    */
/* summation range, so sin^{2l} cot^k = sin^{2l-k} cos^k is finite at        */
/* theta = 0 and pi.  The sum alternates and cancels by up to ~1e-9 of its   */
/* largest term at l = 30, so it is formed in binary128 (113-bit            */
/* significand) and only the result is rounded.                            */
/* ------------------------------------------------------------------------ */
typedef __float128 q128;

static q128 factq(int n) {
    q128 f = 1;
    for (int k = 2; k <= n; ++k) f *= (q128)k;
    return f;
}

static q128 binomq(int n, int k) {
    if (k < 0 || k > n) return 0;
    return factq(n) / (factq(k) * factq(n - k));
}

static q128 ipowq(q128 x, int k) {
    q128 r = 1;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

static void swsh_ld(int s, int l, int m, ld theta, ld phi, ld *re, ld *im) {
    if (l < abs(s) || l < abs(m)) { *re = 0.0L; *im = 0.0L; return; }
    q128 pref = sqrtq(factq(l + m) * factq(l - m) * (q128)(2 * l + 1) /
                      (4 * M_PIq * factq(l + s) * factq(l - s)));
    if (m & 1) pref = -pref;
    const q128 half = (q128)theta / 2;
    const q128 sh = sinq(half), ch = cosq(half);
    q128 sum = 0;
    for (int r = 0; r <= l - s; ++r) {
        int j = r + s - m;
        if (j < 0 || j > l + s) continue;
        int k = 2 * r + s - m;
        q128 term = binomq(l - s, r) * binomq(l + s, j) * ipowq(sh, 2 * l - k) * ipowq(ch, k);
        if ((l - r - s) & 1) term = -term;
        sum += term;
    }
    const q128 a = pref * sum;
    const q128 mphi = (q128)m * (q128)phi;
    *re = (ld)(a * cosq(mphi));
    *im = (ld)(a * sinq(mphi));
}

/* Exported for the harmonic pins. */
int few_oracle_swsh(int s, int l, int m, double theta, double phi, double *re, double *im) {
    if (!re || !im) return OR_E_ARG;
    ld r, i;
    swsh_ld(s, l, m, (ld)theta, (ld)phi, &r, &i);
    *re = (double)r;
    *im = (double)i;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase reduction: y mod 2 pi in binary128, returned in [-pi, pi).         */
/* ------------------------------------------------------------------------ */
static const __float128 TWO_PI_Q = 6.28318530717958647692528676655900576839433879875021Q;

static ld reduce_q(__float128 y) {
    __float128 k = (__float128)nearbyintl((ld)(y / TWO_PI_Q));
    __float128 r = y - k * TWO_PI_Q;
    const __float128 half = TWO_PI_Q / 2;
    while (r >= half) r -= TWO_PI_Q;
    while (r < -half) r += TWO_PI_Q;
    return (ld)r;
}

/* Sample time, binary64 exactly as written: t_start + j * dt. */
static double sample_time(double t_start, double dt, int64_t j) {
    volatile double prod = (double)j * dt;
    return t_start + prod;
}

/* Interval of t: the largest i in [0, K-2] with t_i <= t (last one closed). */
static int find_interval(int K, const double *t, double x) {
    int lo = 0, hi = K - 2;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (t[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Exported for the phase pin: reduced spline phase in [-pi, pi) at times tq. */
int few_oracle_phase(int K, const double *t, const double *y, int64_t nq,
                     const double *tq, double *out) {
    if (!t || !y || !tq || !out) return OR_E_ARG;
    ld *c = malloc(sizeof(ld) * (size_t)(K > 1 ? K - 1 : 1) * 4);
    if (!c) return OR_E_NOMEM;
    int rc = spline_ld(K, t, 1, y, c);
    if (rc) { free(c); return rc; }
    for (int64_t q = 0; q < nq; ++q) {
        if (!(tq[q] >= t[0] && tq[q] <= t[K - 1])) { free(c); return OR_E_RANGE; }
        int i = find_interval(K, t, tq[q]);
        ld x = (ld)tq[q] - (ld)t[i];
        ld r0 = reduce_q((__float128)y[i]);
        ld v = r0 + x * (c[i * 4 + 1] + x * (c[i * 4 + 2] + x * c[i * 4 + 3]));
        out[q] = (double)reduce_q((__float128)v);
    }
    free(c);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Direct interpolated summation (Sec. III C, Eqs. (9)-(10)).               */
/* ------------------------------------------------------------------------ */
typedef struct { ld s, c; } neum_t;   /* Neumaier running sum + compensation */

static void neum_add(neum_t *a, ld v) {
    ld t = a->s + v;
    if (fabsl(a->s) >= fabsl(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/*
 * h at the samples j = idx[q] (q < n_out), or j = q when idx is NULL.
 * amp is knot-major [K][M][2].  Modes: `mode` is [M][width], width 3 for
 * (l, m, n) (k = 0, phi_theta unused) or 4 for (l, m, k, n) with phi_theta
 * given; l >= 2, 0 <= m <= l.  out is complex128 interleaved
 * (re = h_plus, im = -h_cross).
 */
static int sum_general(int K, const double *t, const double *phi_phi,
                       const double *phi_theta, const double *phi_r, int M,
                       const int32_t *mode, int width, const double *amp, double theta,
                       double phi, double scale, double t_start, double dt, int64_t n_samples,
                       const int64_t *idx, int64_t n_out, double *out, int n_threads) {
    const int kerr = width == 4;
    if (!t || !phi_phi || !phi_r || (kerr && !phi_theta) || !mode || !amp || !out || M < 1 ||
        n_samples < 1)
        return OR_E_ARG;
    if (!(dt > 0.0) || !isfinite(dt) || !isfinite(t_start) || !isfinite(theta) ||
        !isfinite(phi) || !isfinite(scale))
        return OR_E_ARG;
    int rc = check_knots(K, t);
    if (rc) return rc;
    for (int k = 0; k < M; ++k) {
        int l = mode[width * k], m = mode[width * k + 1];
        if (l < 2 || m < 0 || m > l) return OR_E_MODES;
    }
    if (!(t_start >= t[0]) || !(sample_time(t_start, dt, n_samples - 1) <= t[K - 1]))
        return OR_E_RANGE;
    if (idx)
        for (int64_t q = 0; q < n_out; ++q)
            if (idx[q] < 0 || idx[q] >= n_samples) return OR_E_RANGE;
    if (!idx) n_out = n_samples;

    /* Splines of every series: Phi_phi, Phi_r, Phi_theta, then Re/Im of each
     * mode (Phi_theta is all zero in the width-3 case and never used). */
    const int S = 3 + 2 * M;
    double *y = malloc(sizeof(double) * (size_t)K * S);
    ld *c = malloc(sizeof(ld) * (size_t)(K - 1) * S * 4);
    ld *red = malloc(sizeof(ld) * (size_t)(K - 1) * 3);
    ld *yp = malloc(sizeof(ld) * (size_t)M * 2), *ym = malloc(sizeof(ld) * (size_t)M * 2);
    if (!y || !c || !red || !yp || !ym) {
        free(y); free(c); free(red); free(yp); free(ym);
        return OR_E_NOMEM;
    }
    for (int i = 0; i < K; ++i) {
        y[(size_t)i * S + 0] = phi_phi[i];
        y[(size_t)i * S + 1] = phi_r[i];
        y[(size_t)i * S + 2] = kerr ? phi_theta[i] : 0.0;
        for (int k = 0; k < 2 * M; ++k) y[(size_t)i * S + 3 + k] = amp[(size_t)i * 2 * M + k];
    }
    rc = spline_ld(K, t, S, y, c);
    if (rc) { free(y); free(c); free(red); free(yp); free(ym); return rc; }
    /* Constant term of each phase cubic, reduced mod 2 pi (exact identity). */
    for (int i = 0; i + 1 < K; ++i) {
        red[3 * i + 0] = reduce_q((__float128)phi_phi[i]);
        red[3 * i + 1] = reduce_q((__float128)phi_r[i]);
        red[3 * i + 2] = kerr ? reduce_q((__float128)phi_theta[i]) : 0.0L;
    }
    /* Harmonics: Y+ = -2Y_lm; Y- = (-1)^{l+k} -2Y_{l,-m} for m > 0 (Eq. (9)). */
    for (int k = 0; k < M; ++k) {
        int l = mode[width * k], m = mode[width * k + 1];
        int kk = kerr ? mode[width * k + 2] : 0;
        swsh_ld(-2, l, m, (ld)theta, (ld)phi, &yp[2 * k], &yp[2 * k + 1]);
        if (m > 0) {
            ld r, i;
            swsh_ld(-2, l, -m, (ld)theta, (ld)phi, &r, &i);
            ld sg = ((l + kk) & 1) ? -1.0L : 1.0L;
            ym[2 * k] = sg * r;
            ym[2 * k + 1] = sg * i;
        } else {
            ym[2 * k] = ym[2 * k + 1] = 0.0L;
        }
    }

    int64_t q;
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads > 0 ? n_threads : 1)
    for (q = 0; q < n_out; ++q) {
        int64_t j = idx ? idx[q] : q;
        double tj = sample_time(t_start, dt, j);
        int i = find_interval(K, t, tj);
        ld x = (ld)tj - (ld)t[i];
        const ld *cf = c + ((size_t)i * S + 0) * 4;
        const ld *cr = c + ((size_t)i * S + 1) * 4;
        const ld *ct = c + ((size_t)i * S + 2) * 4;
        ld pf = reduce_q((__float128)(red[3 * i] + x * (cf[1] + x * (cf[2] + x * cf[3]))));
        ld pr = reduce_q((__float128)(red[3 * i + 1] + x * (cr[1] + x * (cr[2] + x * cr[3]))));
        ld pt = kerr ? reduce_q((__float128)(red[3 * i + 2] + x * (ct[1] + x * (ct[2] + x * ct[3]))))
                     : 0.0L;
        neum_t hr = {0.0L, 0.0L}, hi = {0.0L, 0.0L};
        for (int k = 0; k < M; ++k) {
            int m = mode[width * k + 1], n = mode[width * k + width - 1];
            int kk = kerr ? mode[width * k + 2] : 0;
            const ld *ar = c + ((size_t)i * S + 3 + 2 * k) * 4;
            const ld *ai = c + ((size_t)i * S + 4 + 2 * k) * 4;
            ld a_r = ar[0] + x * (ar[1] + x * (ar[2] + x * ar[3]));
            ld a_i = ai[0] + x * (ai[1] + x * (ai[2] + x * ai[3]));
            ld psi = (ld)m * pf + (ld)kk * pt + (ld)n * pr;
            ld sn, cs;
            sincosl(psi, &sn, &cs);
            /* z = A e^{-i psi} */
            ld z_r = a_r * cs + a_i * sn;
            ld z_i = a_i * cs - a_r * sn;
            /* Y+ z */
            neum_add(&hr, yp[2 * k] * z_r - yp[2 * k + 1] * z_i);
            neum_add(&hi, yp[2 * k] * z_i + yp[2 * k + 1] * z_r);
            /* Y- conj(z) */
            if (m > 0) {
                neum_add(&hr, ym[2 * k] * z_r + ym[2 * k + 1] * z_i);
                neum_add(&hi, ym[2 * k + 1] * z_r - ym[2 * k] * z_i);
            }
        }
        out[2 * q] = (double)((ld)scale * (hr.s + hr.c));
        out[2 * q + 1] = (double)((ld)scale * (hi.s + hi.c));
    }
    free(y); free(c); free(red); free(yp); free(ym);
    return OR_OK;
}

/* Schwarzschild eccentric sum (Eq. (10)); lmn is [M][3]. */
int few_oracle_sum(int K, const double *t, const double *phi_phi, const double *phi_r,
                   int M, const int32_t *lmn, const double *amp,
                   double theta, double phi, double scale,
                   double t_start, double dt, int64_t n_samples,
                   const int64_t *idx, int64_t n_out, double *out, int n_threads) {
    return sum_general(K, t, phi_phi, NULL, phi_r, M, lmn, 3, amp, theta, phi, scale, t_start,
                       dt, n_samples, idx, n_out, out, n_threads);
}

/* Generic-Kerr spherical-projected sum; lmkn is [M][4] = (l, m, k, n). */
int few_oracle_sum_kerr(int K, const double *t, const double *phi_phi, const double *phi_theta,
                        const double *phi_r, int M, const int32_t *lmkn, const double *amp,
                        double theta, double phi, double scale,
                        double t_start, double dt, int64_t n_samples,
                        const int64_t *idx, int64_t n_out, double *out, int n_threads) {
    return sum_general(K, t, phi_phi, phi_theta, phi_r, M, lmkn, 4, amp, theta, phi, scale,
                       t_start, dt, n_samples, idx, n_out, out, n_threads);
}
