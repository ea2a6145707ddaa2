// gfx950 kernels of libfew: the interpolated harmonic-mode summation of
// arXiv:2104.04582, Sec. III C (spline stage, then summation stage) for the
// Schwarzschild sum of Eq. (10) with the mirror modes of Eq. (9), and the
// generic-Kerr sum of Sec. VII (a third phase).
//
//  upload_kernel   copies a batch's host tables (knots, term layouts, job
//                  descriptors) from pinned host memory, ordered on the
//                  compute queue (a single-request fit carries its own copy).
//  fit_kernel      not-a-knot cubic splines of every series on the shared knot
//                  grid.  Amplitude series: binary64, one lane per real series,
//                  rows split over the workgroup's four waves and joined by
//                  the multipliers' products; the grid's tridiagonal factor by
//                  one wave's scan.  Phase series: double-double (one
//                  refinement step, scan solves).
//  fold_pack_kernel  matrix-core requests: interval starts; per interval and
//                  row tile, -2Y_lm, the fold of the l-sum, the row scales and
//                  the fp16 hi/lo operand table.
//  prepare_kernel  vector-path requests: interval starts and tile prefixes;
//                  -2Y_lm and the fold of the l-sum into one complex cubic per
//                  signed (m, [k,] n) term.
//  sum_mfma_kernel binary32 result on the matrix cores: per interval the
//                  product of the coefficient matrix (signed m rows) with the
//                  harmonics f^|n| of the samples, v_mfma_f32_16x16x32_f16 on
//                  fp16 hi/lo parts with fp32 accumulation, a Horner
//                  recurrence in u on the accumulators, rows combined with
//                  e^{-i m Phi_phi}.
//  sum_wg_kernel   binary32 on the vector units: one workgroup of 4 waves = one
//                  tile of consecutive samples inside one knot interval; the
//                  term coefficients are staged in LDS and broadcast to VGPR
//                  operands.  Per sample: phases in binary64 reduced mod 2 pi,
//                  one sincos each; then for every segment of terms a Horner
//                  recurrence in e^{-i Phi_r} over n, seeded by
//                  e^{-i(m Phi_phi + n_lo Phi_r)} (chained across consecutive
//                  m or k), Kahan-compensated within four term groups whose
//                  values are added in order; the end of a launch uses
//                  term-split tiles (the four waves take one group each).
//  sum_kernel      binary64: one wave = one tile; phases in double-double;
//                  coefficients read by scalar loads into SGPR operands.
//  select_kernel   the mode selector of Sec. III D: per knot a radix select
//                  with error-bounded sums, the sorted sequential sums when a
//                  comparison falls inside the bound.
#include "dd.h"
#include "few_internal.h"
#include "swsh.h"

#include <climits>
#include <cstring>
#include <mutex>
#include <type_traits>

namespace few {

#define FEW_AS4 __attribute__((address_space(4)))

// Minimum waves per SIMD (a register cap) of the single-request binary32
// summation kernel: 4, i.e. at most 128 registers, which keeps the three-phase
// (generic-Kerr) instantiation at four workgroups per CU as well.
#ifndef FEW_SUM_WAVES
#define FEW_SUM_WAVES 4
#endif
#define FEW_SUM_ATTR __attribute__((amdgpu_waves_per_eu(FEW_SUM_WAVES)))
// Binary64: the five-FMA chains per component need more waves in flight than
// the register count alone allows (4 per SIMD); 5 costs one spill outside the
// term loop.
#ifndef FEW_F64_WAVES
#define FEW_F64_WAVES 5
#endif
#define FEW_F64_ATTR __attribute__((amdgpu_waves_per_eu(FEW_F64_WAVES)))

// Wave-uniform read-only data: the constant address space makes the compiler
// use scalar loads (SGPR destinations) for uniform addresses.
template <typename T>
__device__ __forceinline__ const FEW_AS4 T *cptr(const T *p) {
    return (const FEW_AS4 T *)(p);
}

// Copy a trivially copyable object from a wave-uniform address as 32-bit
// scalar loads.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "4-byte granularity");
    T v;
    const FEW_AS4 uint32_t *s = (const FEW_AS4 uint32_t *)(p);
    uint32_t *d = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = s[i];
    return v;
}

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Binary64 sample time exactly as written: t_start + j * dt.
__device__ __forceinline__ double dev_sample_time(double t_start, double dt, long long j) {
    return __dadd_rn(t_start, __dmul_rn((double)j, dt));
}

// ===========================================================================
// Spline stage (Sec. III C: not-a-knot spline, all series on one knot grid).
//
// Slope form: on [t_i, t_{i+1}], x = t - t_i, h_i = t_{i+1} - t_i,
// delta_i = (y_{i+1} - y_i) / h_i and end slopes s_i, s_{i+1}:
//   y = y_i + s_i x + c_i x^2 + d_i x^3,
//   c_i = (3 delta_i - 2 s_i - s_{i+1}) / h_i,  d_i = (s_i + s_{i+1} - 2 delta_i) / h_i^2.
// Tridiagonal system for the slopes (rows: sub, diag, super | rhs):
//   row 0      : -, h_1, h_0 + h_1 | ((h_0 + 2(h_0 + h_1)) h_1 delta_0 + h_0^2 delta_1) / (h_0 + h_1)
//   row 1..K-2 : h_i, 2 (h_{i-1} + h_i), h_{i-1} | 3 (h_i delta_{i-1} + h_{i-1} delta_i)
//   row K-1    : h_{K-2} + h_{K-3}, h_{K-3}, - |
//                (h_{K-2}^2 delta_{K-3} + (2 (h_{K-3} + h_{K-2}) + h_{K-2}) h_{K-3} delta_{K-2})
//                / (h_{K-3} + h_{K-2})
// (interior rows: continuous second derivative; end rows: the not-a-knot
// conditions d_0 = d_1 and d_{K-3} = d_{K-2} with s_2 / s_{K-3} eliminated).
// Solved by forward elimination and back substitution without pivoting.
// ===========================================================================

// LU factor of the slope system on the shared grid: inverse pivots invd[r] and
// multipliers w[r] = c_r invd[r] of the forward sweep (c_r the super-diagonal),
// with pivots den_r = a_r - b_r w_{r-1} (a_r diagonal, b_r sub-diagonal).
// The pivot recurrence is a continued fraction; with w_r = p_r / q_r it is the
// division-free pair
//   q_r = a_r q_{r-1} - b_r p_{r-1},   p_r = c_r q_{r-1},   den_r = q_r / q_{r-1},
// rescaled at every row by a power of two (exact, ratios unchanged) so it
// cannot overflow.  One lane runs it (fit_factor_serial: a multiply, an FMA and
// the rescale per row, knot spacings fetched 16 at a time), storing q_{r-1}
// and q_r per row in invd / wv; then every lane forms the ratios
// (fit_factor_finish).  A division per row on the serial chain was its
// latency bound.
__device__ __forceinline__ void fit_factor_serial(const double *h, int K, double *num,
                                                  double *den) {
    constexpr int C = 16;
    double q = h[1], p = h[0] + h[1];               // row 0: diag h_1, super h_0 + h_1
    num[0] = 1.0;
    den[0] = q;
    double hp = h[0];                               // h_{r-1}
    auto row = [&](int r, double hr) {              // interior row r: b = h_r, a = 2(h_{r-1} + h_r), c = h_{r-1}
        const double Q = (2.0 * (hp + hr)) * q - hr * p;
        num[r] = q;
        den[r] = Q;
        int e;
        const double m = frexp(Q, &e);
        p = ldexp(hp * q, -e);
        q = m;
        hp = hr;
    };
    int r0 = 1;
    for (; r0 + C <= K - 1; r0 += C) {
        double hv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) hv[c] = h[r0 + c];
#pragma unroll
        for (int c = 0; c < C; ++c) row(r0 + c, hv[c]);
    }
    for (; r0 <= K - 2; ++r0) row(r0, h[r0]);
    // row K-1: sub h_{K-2} + h_{K-3}, diag h_{K-3}
    num[K - 1] = q;
    den[K - 1] = h[K - 3] * q - (h[K - 2] + h[K - 3]) * p;
}

// Ratios of the factor: inverse pivots invd[r], back-sweep multipliers
// wv[r] = c_r invd[r] and forward-sweep multipliers bv[r] = b_r invd[r] (b_r
// the sub-diagonal), so each forward step is one fused multiply-add on the
// serial chain: g_r = rhs_r invd_r - bv_r g_{r-1}.
__device__ __forceinline__ void fit_factor_finish(const double *h, int K, double *invd,
                                                  double *wv, double *bv) {
    for (int r = threadIdx.x; r < K; r += blockDim.x) {
        const double id = invd[r] / wv[r];
        const double c = r == 0 ? h[0] + h[1] : (r < K - 1 ? h[r - 1] : 0.0);
        const double b = r == 0 ? 0.0 : (r < K - 1 ? h[r] : h[K - 2] + h[K - 3]);
        invd[r] = id;
        wv[r] = c * id;
        bv[r] = b * id;
    }
}

// LDS writes of one wave made visible to its other lanes (the wave's LDS
// accesses complete in order; this keeps the compiler from moving them).
__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row r of the slope system: sub-diagonal b, diagonal a, super-diagonal c
// (the table above).
__device__ __forceinline__ void slope_row(const double *h, int K, int r, double *b, double *a,
                                          double *c) {
    if (r == 0) {
        *b = 0.0;
        *a = h[1];
        *c = h[0] + h[1];
    } else if (r < K - 1) {
        *b = h[r];
        *a = 2.0 * (h[r - 1] + h[r]);
        *c = h[r - 1];
    } else {
        *b = h[K - 2] + h[K - 3];
        *a = h[K - 3];
        *c = 0.0;
    }
}

// The same factor (invd, wv, bv as fit_factor_finish leaves them) on one wave
// for K <= kFitStageKnots.  With every continuant divided by the diagonals,
// qt_r = q_r / (a_0 ... a_r), the recurrence becomes
//   qt_r = qt_{r-1} - g_r qt_{r-2},  g_r = b_r c_{r-1} / (a_r a_{r-1}),
// qt_{-1} = qt_0 = 1, and den_r = a_r qt_r / qt_{r-1}.  For this system
// 0 <= g_r <= 1/4 on interior rows and g_r = 1/2 on rows 1 and K - 1, so
// qt_r / qt_{r-1} lies in [1/2, 1] on rows 1 .. K - 2 (by induction) and in
// (0, 1) on row K - 1: the qt stay positive and above 2^-K times the last
// ratio, with no rescaling.  In matrix form (qt_r, qt_{r-1}) =
// T_r (qt_{r-1}, qt_{r-2}), T_r = [[1, -g_r], [1, 0]]; lane l takes rows
// 2l + 1 and 2l + 2, and the lanes' products are composed by a log-step scan
// (later rows on the left).
__device__ void fit_factor_wave(const double *h, int K, double *invd, double *wv, double *bv) {
    const int lane = threadIdx.x & (kWave - 1);
    const int r0 = 2 * lane + 1, r1 = r0 + 1;
    double bb0 = 0.0, aa0 = 1.0, cc0 = 0.0, bb1 = 0.0, aa1 = 1.0, cc1 = 0.0;
    double g0 = 0.0, g1 = 0.0;
    if (r0 < K) {
        double bp, ap, cp;
        slope_row(h, K, r0 - 1, &bp, &ap, &cp);
        slope_row(h, K, r0, &bb0, &aa0, &cc0);
        g0 = bb0 * cp / (aa0 * ap);
    }
    if (r1 < K) {
        slope_row(h, K, r1, &bb1, &aa1, &cc1);
        g1 = bb1 * cc0 / (aa1 * aa0);
    }
    // this lane's product T_{r1} T_{r0} (identity rows past the end)
    double m00, m01, m10, m11;
    if (r1 < K) {
        m00 = 1.0 - g1; m01 = -g0; m10 = 1.0; m11 = -g0;
    } else if (r0 < K) {
        m00 = 1.0; m01 = -g0; m10 = 1.0; m11 = 0.0;
    } else {
        m00 = 1.0; m01 = 0.0; m10 = 0.0; m11 = 1.0;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double o00 = __shfl_up(m00, d), o01 = __shfl_up(m01, d);
        const double o10 = __shfl_up(m10, d), o11 = __shfl_up(m11, d);
        if (lane >= d) {
            const double n00 = fma(m00, o00, m01 * o10), n01 = fma(m00, o01, m01 * o11);
            const double n10 = fma(m10, o00, m11 * o10), n11 = fma(m10, o01, m11 * o11);
            m00 = n00; m01 = n01; m10 = n10; m11 = n11;
        }
    }
    // (qt_{r0-1}, qt_{r0-2}) = (rows before this lane's) applied to (1, 1)
    double p00 = __shfl_up(m00, 1), p01 = __shfl_up(m01, 1);
    double p10 = __shfl_up(m10, 1), p11 = __shfl_up(m11, 1);
    if (lane == 0) { p00 = 1.0; p01 = 0.0; p10 = 0.0; p11 = 1.0; }
    const double qa = p00 + p01, qb = p10 + p11;    // qt_{r0-1}, qt_{r0-2}
    if (r0 < K) {
        const double q0 = fma(-g0, qb, qa);           // qt_{r0}
        const double id0 = qa / (aa0 * q0);
        invd[r0] = id0;
        wv[r0] = cc0 * id0;
        bv[r0] = bb0 * id0;
        if (r1 < K) {
            const double q1 = fma(-g1, qa, q0);
            const double id1 = q0 / (aa1 * q1);
            invd[r1] = id1;
            wv[r1] = cc1 * id1;
            bv[r1] = bb1 * id1;
        }
    }
    if (lane == 0) {                                 // row 0: den_0 = a_0
        const double id = 1.0 / h[1];
        invd[0] = id;
        wv[0] = (h[0] + h[1]) * id;
        bv[0] = 0.0;
    }
}

// y_r = a(r) + m(r) y_{r-1} for r < n <= 2 kWave, y_{-1} = 0, on one wave:
// lane l takes rows 2l and 2l + 1, and the lanes' affine maps y -> A + M y are
// composed by a log-step scan (later rows on the left).  Returns this lane's
// two values (y_{2l}, y_{2l+1}); rows past n are identities.
template <typename FA, typename FM>
__device__ __forceinline__ double2 wave_affine(int n, FA a, FM m) {
    const int lane = threadIdx.x & (kWave - 1);
    const int r0 = 2 * lane, r1 = r0 + 1;
    double a0 = 0.0, m0 = 1.0, a1 = 0.0, m1 = 1.0;
    if (r0 < n) { a0 = a(r0); m0 = m(r0); }
    if (r1 < n) { a1 = a(r1); m1 = m(r1); }
    double A = fma(m1, a0, a1), M = m1 * m0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double Ao = __shfl_up(A, d), Mo = __shfl_up(M, d);
        if (lane >= d) {
            A = fma(M, Ao, A);
            M = M * Mo;
        }
    }
    double yin = __shfl_up(A, 1);
    if (lane == 0) yin = 0.0;
    const double y0 = fma(m0, yin, a0);
    return make_double2(y0, fma(m1, y0, a1));
}

// Phase series ph (workgroup ph), to double-double accuracy by one step of
// iterative refinement: solve the slope system in binary64 (Thomas), form
// the residual with the exact double-double matrix and right-hand side, solve
// again for the correction and add it.  After one step the error is of order
// (eps cond)^2, far below double-double rounding, and only the two binary64
// sweeps are serial.  pcoef[((i * 2 + ph) * 4 + p) * 2 + {0, 1}] = (hi, lo) of
// coefficient p on interval i; p = 0 holds y_i reduced mod 2 pi.
// LDS (binary64 arrays of length K): h hi/lo, delta hi/lo, w, inverse pivot,
// first solution s0, right-hand side / residual / correction.
__device__ void fit_phase_dd(const FitJob &jb, const double *t, int ph, double *lds) {
    const double *y = ph == 0 ? jb.phi_phi : (ph == 1 ? jb.phi_r : jb.phi_theta);
    const int K = jb.K;
    const int tid = threadIdx.x, bs = blockDim.x;
    double *Hh = lds, *Hl = lds + K, *Dh = lds + 2 * K, *Dl = lds + 3 * K;
    double *wv = lds + 4 * K, *invd = lds + 5 * K, *s0 = lds + 6 * K, *rr = lds + 7 * K;
    double *bv = lds + 8 * K;
    auto H = [&](int i) { return dd_make(Hh[i], Hl[i]); };
    auto D = [&](int i) { return dd_make(Dh[i], Dl[i]); };
    // row r of the slope system: sub, diag, super (double-double)
    auto row = [&](int r, dd *sub, dd *diag, dd *sup) {
        if (r == 0) {
            *sub = dd_make(0.0);
            *diag = H(1);
            *sup = dd_add(H(0), H(1));
        } else if (r < K - 1) {
            *sub = H(r);
            *diag = dd_mul_d(dd_add(H(r - 1), H(r)), 2.0);
            *sup = H(r - 1);
        } else {
            *sub = dd_add(H(K - 2), H(K - 3));
            *diag = H(K - 3);
            *sup = dd_make(0.0);
        }
    };
    auto rhs = [&](int r) {
        if (r == 0) {
            const dd h0 = H(0), h1 = H(1), sup = dd_add(h0, h1);
            return dd_div(dd_add(dd_mul(dd_mul(dd_add(h0, dd_mul_d(sup, 2.0)), h1), D(0)),
                                 dd_mul(dd_mul(h0, h0), D(1))),
                          sup);
        }
        if (r < K - 1)
            return dd_mul_d(dd_add(dd_mul(H(r), D(r - 1)), dd_mul(H(r - 1), D(r))), 3.0);
        const dd ha = H(K - 3), hb = H(K - 2), sum = dd_add(ha, hb);
        return dd_div(dd_add(dd_mul(dd_mul(hb, hb), D(K - 3)),
                             dd_mul(dd_mul(dd_add(dd_mul_d(sum, 2.0), hb), ha), D(K - 2))),
                      sum);
    };
    // binary64 Thomas sweeps with the factor in invd / wv / bv (of the rounded
    // matrix; the refinement step uses the exact rows): x <- A^-1 x in place.
    // K <= kFitStageKnots: wave 0 takes each sweep as one affine scan
    // (wave_affine; the back sweep in reversed row order).  Otherwise one lane
    // carries the recurrence in registers: the LDS operands of C rows are
    // loaded together, the rows eliminated (one fused multiply-add each on
    // the serial chain), and the C results stored after the batch.
    const bool wave_solve = K <= kFitStageKnots;
    auto solve_wave = [&](double *x) {
        const int r0 = 2 * tid, r1 = r0 + 1;
        const double2 g = wave_affine(
            K, [&](int r) { return x[r] * invd[r]; }, [&](int r) { return -bv[r]; });
        if (r0 < K) x[r0] = g.x;
        if (r1 < K) x[r1] = g.y;
        lds_wave_sync();
        const double2 v = wave_affine(
            K, [&](int r) { return x[K - 1 - r]; }, [&](int r) { return -wv[K - 1 - r]; });
        lds_wave_sync();
        if (r0 < K) x[K - 1 - r0] = v.x;
        if (r1 < K) x[K - 1 - r1] = v.y;
    };
    auto solve = [&](double *x) {
        constexpr int C = 16;
        double g = x[0] * invd[0];
        x[0] = g;
        int r0 = 1;
        for (; r0 + C <= K; r0 += C) {
            double xv[C], bb[C], iv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xv[c] = x[r0 + c];
                bb[c] = bv[r0 + c];
                iv[c] = invd[r0 + c];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) xv[c] = xv[c] * iv[c];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                g = fma(-bb[c], g, xv[c]);
                xv[c] = g;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) x[r0 + c] = xv[c];
        }
        for (; r0 < K; ++r0) {
            g = fma(-bv[r0], g, x[r0] * invd[r0]);
            x[r0] = g;
        }
        double nx = x[K - 1];
        r0 = K - 2;
        for (; r0 - C + 1 >= 0; r0 -= C) {
            double xv[C], wr[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xv[c] = x[r0 - c];
                wr[c] = wv[r0 - c];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xv[c] = fma(-wr[c], nx, xv[c]);
                nx = xv[c];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) x[r0 - c] = xv[c];
        }
        for (; r0 >= 0; --r0) {
            x[r0] = fma(-wv[r0], nx, x[r0]);
            nx = x[r0];
        }
    };

    for (int i = tid; i < K - 1; i += bs) {
        const dd h = two_sum(t[i + 1], -t[i]);
        const dd d = dd_div(two_sum(y[i + 1], -y[i]), h);
        Hh[i] = h.hi; Hl[i] = h.lo;
        Dh[i] = d.hi; Dl[i] = d.lo;
    }
    __syncthreads();
    // binary64 factor of the rounded matrix (wave 0, or one lane of it) while
    // the other waves form the right-hand side, then the first solve
    if (wave_solve) {
        if (tid < kWave) fit_factor_wave(Hh, K, invd, wv, bv);
    } else if (tid == 0) {
        fit_factor_serial(Hh, K, invd, wv);
    }
    if (tid >= kWave)
        for (int r = tid - kWave; r < K; r += bs - kWave) s0[r] = rhs(r).hi;
    __syncthreads();
    if (!wave_solve) {
        fit_factor_finish(Hh, K, invd, wv, bv);
        __syncthreads();
    }
    if (wave_solve ? tid < kWave : tid == 0) {
        if (wave_solve) solve_wave(s0); else solve(s0);
    }
    __syncthreads();
    // residual of the exact (double-double) system at s0
    for (int r = tid; r < K; r += bs) {
        dd sub, diag, sup;
        row(r, &sub, &diag, &sup);
        dd ax = dd_mul_d(diag, s0[r]);
        if (r > 0) ax = dd_add(ax, dd_mul_d(sub, s0[r - 1]));
        if (r < K - 1) ax = dd_add(ax, dd_mul_d(sup, s0[r + 1]));
        rr[r] = dd_sub(rhs(r), ax).hi;
    }
    __syncthreads();
    if (wave_solve ? tid < kWave : tid == 0) {
        if (wave_solve) solve_wave(rr); else solve(rr);
    }
    __syncthreads();
    double *pc = jb.pcoef;
    for (int r = tid; r < K - 1; r += bs) {
        const dd sa = two_sum(s0[r], rr[r]), sb = two_sum(s0[r + 1], rr[r + 1]);
        const dd h = H(r), d = D(r);
        const dd c = dd_div(dd_sub(dd_sub(dd_mul_d(d, 3.0), dd_mul_d(sa, 2.0)), sb), h);
        const dd e = dd_div(dd_sub(dd_add(sa, sb), dd_mul_d(d, 2.0)), dd_mul(h, h));
        const dd a = dd_reduce_2pi(dd_make(y[r]));
        double *o = pc + ((size_t)r * jb.n_ph + ph) * 8;
        o[0] = a.hi; o[1] = a.lo;
        o[2] = sa.hi; o[3] = sa.lo;
        o[4] = c.hi; o[5] = c.lo;
        o[6] = e.hi; o[7] = e.lo;
    }
}

// The two sweeps of one real amplitude series q (lane tid of wave 0) for
// grids of more than kFitStageKnots knots: knot values stream from global
// memory, the forward results go through the coefficient array, and each
// row's coefficients are stored as its slope is found.
__device__ __forceinline__ void fit_sweeps(const FitJob &jb, int tid, int q, int K, int M,
                                           const double *hs, const double *invd,
                                           const double *wv, const double *ih,
                                           const double *bv) {
    constexpr int C = 16;
    const size_t ys_stride = 2 * (size_t)M;
    // coefficient p of series q on interval r at o[r * cs + p * ps]
    // ([K-1][4][2M] or [K-1][M][4][2])
    const bool pm = jb.acoef_pmajor != 0;
    const size_t ps = pm ? 2 * (size_t)M : 2, cs = 8 * (size_t)M;
    const int k = q >> 1, comp = q & 1;
    const double *__restrict__ y = jb.amp + 2 * (size_t)k + comp;
    double *__restrict__ o = jb.acoef + (pm ? (size_t)q : 8 * (size_t)k + comp);
    // knot value idx (clamped to the grid: in bounds, unused past it)
    auto ldy = [&](int idx) {
        const int i = min(max(idx, 0), K - 1);
        return y[(size_t)i * ys_stride];
    };
    auto stg = [&](int r, double gv) { o[(size_t)r * cs + ps] = gv; };
    auto ldg = [&](int r) { return o[(size_t)max(r, 0) * cs + ps]; };

    // Forward elimination.  Knot idx gives delta_{idx-1}; rows 0 and 1 close
    // at knot 2, row idx - 1 at every later knot, row K - 1 after the last.
    double yprev = ldy(0);
    double dm1, d0, g;
    {
        const double y1 = ldy(1), y2 = ldy(2);
        const double h0 = hs[0], h1 = hs[1];
        dm1 = (y1 - yprev) * ih[0];
        d0 = (y2 - y1) * ih[1];
        yprev = y2;
        g = ((h0 + 2.0 * (h0 + h1)) * h1 * dm1 + h0 * h0 * d0) / (h0 + h1) * invd[0];
        stg(0, g);
        const double rhs = 3.0 * (h1 * dm1 + h0 * d0);
        g = fma(-bv[1], g, rhs * invd[1]);
        stg(1, g);
    }
    // one row: r = idx - 1 closes at knot idx
    auto fwd = [&](int idx, double yi) {
        const int r = idx - 1;
        dm1 = d0;
        d0 = (yi - yprev) * ih[r];
        yprev = yi;
        g = fma(-bv[r], g, (3.0 * (hs[r] * dm1 + hs[r - 1] * d0)) * invd[r]);
        stg(r, g);
    };
    // C rows: operands first, then the chain, then the stores
    auto fwd_batch = [&](int i0, const double *ya) {
        double hr[C], hm[C], iv[C], bb[C], rv[C];
        const int rb = i0 - 1;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            hr[c] = hs[rb + c];
            hm[c] = hs[rb + c - 1];
            rv[c] = ih[rb + c];
            iv[c] = invd[rb + c];
            bb[c] = bv[rb + c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            dm1 = d0;
            d0 = (ya[c] - yprev) * rv[c];
            yprev = ya[c];
            rv[c] = (3.0 * (hr[c] * dm1 + hm[c] * d0)) * iv[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            g = fma(-bb[c], g, rv[c]);
            rv[c] = g;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) stg(rb + c, rv[c]);
    };
    double ya[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ya[c] = ldy(3 + c);
    int i0 = 3;
    for (; i0 + C <= K; i0 += C) {
        double yb[C];
#pragma unroll
        for (int c = 0; c < C; ++c) yb[c] = ldy(i0 + C + c);
        fwd_batch(i0, ya);
#pragma unroll
        for (int c = 0; c < C; ++c) ya[c] = yb[c];
    }
    for (int c = 0; i0 + c < K; ++c) fwd(i0 + c, ya[c]);
    {
        const double ha = hs[K - 3], hb = hs[K - 2];
        const double rhs = (hb * hb * dm1 + (2.0 * (ha + hb) + hb) * ha * d0) / (ha + hb);
        g = fma(-bv[K - 1], g, rhs * invd[K - 1]);
    }
    // Back substitution and coefficients, interval K-2 down to 0, in batches
    // of C rows r0, r0 - 1, ...: operands first (the batch's forward results
    // and knot values, and the next batch's in flight), then the chain.
    double s_next = g;
    double yr1 = yprev;                              // y_{K-1}
    double ga[C], yv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ga[c] = ldg(K - 2 - c);
        yv[c] = ldy(K - 2 - c);
    }
    auto back = [&](int r, double gr, double yv0) {
        const double ir = ih[r];
        const double dr = (yr1 - yv0) * ir;
        const double sv = fma(-wv[r], s_next, gr);
        double *orow = o + (size_t)r * cs;
        orow[0] = yv0;
        orow[ps] = sv;
        orow[2 * ps] = (3.0 * dr - 2.0 * sv - s_next) * ir;
        orow[3 * ps] = (sv + s_next - 2.0 * dr) * (ir * ir);
        s_next = sv;
        yr1 = yv0;
    };
    int r0 = K - 2;
    for (; r0 - C + 1 >= 0; r0 -= C) {
        double gb[C], yw[C], irv[C], wrv[C], sv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            gb[c] = ldg(r0 - C - c);
            yw[c] = ldy(r0 - C - c);
            irv[c] = ih[r0 - c];
            wrv[c] = wv[r0 - c];
        }
        double sn = s_next;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            sn = fma(-wrv[c], sn, ga[c]);
            sv[c] = sn;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int r = r0 - c;
            const double sh = c == 0 ? s_next : sv[c - 1];    // slope at knot r + 1
            const double yh = c == 0 ? yr1 : yv[c - 1];       // value at knot r + 1
            const double ir = irv[c];
            const double dr = (yh - yv[c]) * ir;
            double *orow = o + (size_t)r * cs;
            orow[0] = yv[c];
            orow[ps] = sv[c];
            orow[2 * ps] = (3.0 * dr - 2.0 * sv[c] - sh) * ir;
            orow[3 * ps] = (sv[c] + sh - 2.0 * dr) * (ir * ir);
        }
        s_next = sn;
        yr1 = yv[C - 1];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            ga[c] = gb[c];
            yv[c] = yw[c];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (r0 - c >= 0) back(r0 - c, ga[c], yv[c]);
}

// The upload carried by a single-request fit launch: amplitude workgroup blk
// copies its share of the 16-byte words (the tail word may run into the
// block's alignment padding; the staging slot is at least 1 MiB), on the
// lanes of waves 1-3, which do not take part in the sweeps.
__device__ __forceinline__ void fit_copy_upload(const FitJob &jb, int blk) {
    if (jb.up_bytes <= 0) return;
    const long long words = (jb.up_bytes + 15) / 16;
    const long long per = (words + jb.amp_blocks - 1) / jb.amp_blocks;
    const long long w0 = (long long)blk * per, w1 = min(words, w0 + per);
    const int lanes = (int)blockDim.x - kWave;
    for (long long x = w0 + ((int)threadIdx.x - kWave); x < w1; x += lanes)
        jb.up_dst[x] = jb.up_src[x];
}

// Binary64 solve of the amplitude series handled by this workgroup for grids
// of more than kFitStageKnots knots, one lane of wave 0 per real series.  LDS:
// h[K], inverse pivots invd[K], multipliers wv[K] and bv[K] and 1 / h[K] of
// the shared grid (the sweeps multiply by 1 / h_i instead of dividing: a
// division is a long dependent sequence on this hardware, and the sweeps are
// latency bound).  Wave 0 forms the grid and one of its lanes the factor;
// each lane streams its knot values from global memory, both sweeps working in
// batches of C rows (operands first, the serial chain in registers, the
// results stored after it).
__device__ void fit_amplitudes_stream(const FitJob &jb, const double *t, int blk, double *lds) {
    const int K = jb.K, M = jb.M;
    const int tid = threadIdx.x;
    double *hs = lds, *invd = lds + K, *wv = lds + 2 * K, *ih = lds + 3 * K, *bv = lds + 4 * K;
    const int q0 = blk * kFitSeriesPerBlock;
    if (tid < kWave) {
        for (int i = tid; i < K - 1; i += kWave) {
            const double h = t[i + 1] - t[i];
            hs[i] = h;
            ih[i] = 1.0 / h;
        }
        __builtin_amdgcn_wave_barrier();
        if (tid == 0) fit_factor_serial(hs, K, invd, wv);
    }
    __syncthreads();
    fit_factor_finish(hs, K, invd, wv, bv);
    __syncthreads();
    const int q = q0 + tid;
    if (tid < kFitSeriesPerBlock && q < 2 * M) fit_sweeps(jb, tid, q, K, M, hs, invd, wv, ih, bv);
    if (tid >= kWave) fit_copy_upload(jb, blk);
}

// Row l of a wave-uniform value held by lane l (both halves by readlane).
__device__ __forceinline__ double lane_value(double v, int l) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Binary64 solve of the amplitude series of workgroup blk (64 real series,
// lane = series) for K <= kFitStageKnots.  The rows are split over the four
// waves: wave w takes rows [R_w, R_{w+1}) and keeps its lanes' knot values
// y_{R_w - 1} .. y_{R_{w+1}} and its forward results and slopes in
// registers; row-wise constants are formed lane-parallel (lane c for row
// R_w + c) and broadcast with readlane.  Wave 0 forms the factor
// (fit_factor_wave) while every wave's knot values are in flight.  Row r's
// forward input rhs_r invd_r is
//   al_r (y_{a+1} - y_a) + be_r (y_{a+2} - y_{a+1}),  a = clamp(r - 1, 0, K - 3)
// (its two divided differences).  Each wave runs its rows from a zero start
// and the chunks are joined afterwards, since a first-order recurrence at row
// r is its zero-start value plus the product of the multipliers since the
// chunk start times the value entering the chunk:
//   forward g_r = rhs_r invd_r - bv_r g_{r-1}:  g_r = gl_r + F_r G,
//           F_r = prod_{j = R_w .. r} (-bv_j), G = g_{R_w - 1};
//   back    s_r = g_r - wv_r s_{r+1}:          s_r = sl_r + B_r S,
//           B_r = prod_{j = r .. R_{w+1} - 1} (-wv_j), S = s_{R_{w+1}}.
// The values entering the chunks follow from the chunk ends (exchanged in
// LDS) in at most three steps.  Each wave then writes the coefficients of its
// intervals.
__device__ void fit_amplitudes_staged(const FitJob &jb, const double *t, int blk, double *lds) {
    constexpr int NW = 4;                            // waves (launched with 256 lanes)
    constexpr int LC = (kFitStageKnots + NW - 1) / NW;   // most rows of a chunk
    const int K = jb.K, M = jb.M;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    double *hs = lds, *invd = lds + K, *wv = lds + 2 * K, *bv = lds + 3 * K;
    double *cf = lds + 4 * K;                        // [NW][64] forward values at chunk ends
    double *cb = cf + NW * kWave;                    // [NW][64] back values at chunk starts
    double *fe = cb + NW * kWave;                    // [NW] F at chunk ends
    double *bs0 = fe + NW;                           // [NW] B at chunk starts
    const int q = blk * kFitSeriesPerBlock + lane;
    const bool live = q < 2 * M;
    const int L = (K + NW - 1) / NW;
    const int r_lo = min(K, w * L), n = min(K, r_lo + L) - r_lo;
    // The knot times of the spacings h_i = t_{i+1} - t_i that wave 0 forms for
    // the factor (i = lane and lane + 64, clamped), requested first: a wave's
    // loads complete in order, so the factor waits only for these and starts
    // while the knot values and the upload requested below are in flight.
    static_assert(kFitStageKnots <= 2 * kWave + 1, "two spacings per lane");
    double ta0 = t[min(lane, K - 2)], tb0 = t[min(lane, K - 2) + 1];
    double ta1 = t[min(lane + kWave, K - 2)], tb1 = t[min(lane + kWave, K - 2) + 1];
    // the workgroup's share of the upload: each lane's first word requested
    // now (host memory is far) and stored at the end
    long long up_x = -1, up_end = 0;
    uint4 up_w = make_uint4(0u, 0u, 0u, 0u);
    if (jb.up_bytes > 0) {
        const long long words = (jb.up_bytes + 15) / 16;
        const long long per = (words + jb.amp_blocks - 1) / jb.amp_blocks;
        up_end = min(words, (long long)blk * per + per);
        up_x = (long long)blk * per + tid;
        if (up_x < up_end) up_w = jb.up_src[up_x];
    }
    // knot values y_{r_lo - 2 + j} (clamped to the grid), all in flight
    double yv[LC + 4];
    {
        const double *y = jb.amp + q;
        const size_t stride = 2 * (size_t)M;
#pragma unroll
        for (int j = 0; j < LC + 4; ++j) {
            const int i = min(max(r_lo - 2 + j, 0), K - 1);
            yv[j] = live ? y[(size_t)i * stride] : 0.0;
        }
    }
    // the knot times are taken here, after the loads above were issued (this
    // keeps the compiler from moving their loads into the branch below)
    asm volatile("" : "+v"(ta0), "+v"(tb0), "+v"(ta1), "+v"(tb1));
    if (w == 0) {
        if (lane < K - 1) hs[lane] = tb0 - ta0;
        if (lane + kWave < K - 1) hs[lane + kWave] = tb1 - ta1;
        lds_wave_sync();
        fit_factor_wave(hs, K, invd, wv, bv);
    }
    __syncthreads();
    // row-wise constants of row r_lo + c in lane c
    double c_al = 0.0, c_be = 0.0, c_bv = 0.0, c_wv = 0.0, c_ih = 0.0;
    if (lane < n) {
        const int r = r_lo + lane;
        double P, Q;
        int a;
        if (r == 0) {
            const double h0 = hs[0], h1 = hs[1];
            P = (h0 + 2.0 * (h0 + h1)) * h1 / (h0 + h1);
            Q = h0 * h0 / (h0 + h1);
            a = 0;
        } else if (r < K - 1) {
            P = 3.0 * hs[r];
            Q = 3.0 * hs[r - 1];
            a = r - 1;
        } else {
            const double ha = hs[K - 3], hb = hs[K - 2];
            P = hb * hb / (ha + hb);
            Q = (2.0 * (ha + hb) + hb) * ha / (ha + hb);
            a = K - 3;
        }
        const double id = invd[r];
        c_al = id * P / hs[a];
        c_be = id * Q / hs[a + 1];
        c_bv = bv[r];
        c_wv = wv[r];
        c_ih = r < K - 1 ? 1.0 / hs[r] : 0.0;
    }
    // chunk products: F in lane c over rows r_lo .. r_lo + c, B over
    // r_lo + c .. r_lo + n - 1 (log-step scans; identities past the chunk)
    double c_F = lane < n ? -c_bv : 1.0, c_B = lane < n ? -c_wv : 1.0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double fo = __shfl_up(c_F, d), bo = __shfl_down(c_B, d);
        if (lane >= d) c_F *= fo;
        if (lane + d < kWave) c_B *= bo;
    }
    // forward chain of the chunk from a zero start
    double gv[LC];
    double g = 0.0;
#pragma unroll
    for (int c = 0; c < LC; ++c) {
        if (c < n) {
            const int r = r_lo + c;
            // y_a, y_{a+1}, y_{a+2}: yv[c+1 ..] on interior rows (a = r - 1),
            // one further on row 0 (a = 0) and one back on row K - 1 (a = K - 3)
            const int sh = r == 0 ? 1 : (r == K - 1 ? -1 : 0);
            const double y0 = sh > 0 ? yv[c + 2] : (sh < 0 ? yv[c] : yv[c + 1]);
            const double y1 = sh > 0 ? yv[c + 3] : (sh < 0 ? yv[c + 1] : yv[c + 2]);
            const double y2 = sh > 0 ? yv[c + 4] : (sh < 0 ? yv[c + 2] : yv[c + 3]);
            const double v = fma(lane_value(c_al, c), y1 - y0, lane_value(c_be, c) * (y2 - y1));
            g = fma(-lane_value(c_bv, c), g, v);
            gv[c] = g;
        }
    }
    cf[w * kWave + lane] = g;
    if (lane == max(n, 1) - 1) fe[w] = n > 0 ? c_F : 1.0;
    __syncthreads();
    {
        // forward value entering the chunk, then the back chain of the chunk
        // on the joined forward values
        double G = 0.0;
        for (int cc = 0; cc < w; ++cc) G = fma(fe[cc], G, cf[cc * kWave + lane]);
        double sl = 0.0;
#pragma unroll
        for (int c = LC - 1; c >= 0; --c) {
            if (c < n) {
                const double gj = fma(lane_value(c_F, c), G, gv[c]);
                sl = fma(-lane_value(c_wv, c), sl, gj);
                gv[c] = sl;
            }
        }
        cb[w * kWave + lane] = sl;
        if (lane == 0) bs0[w] = n > 0 ? c_B : 1.0;
    }
    __syncthreads();
    // slope entering the chunk from above, s_{r_lo + n}
    double Sx = 0.0;
    for (int cc = NW - 1; cc > w; --cc) Sx = fma(bs0[cc], Sx, cb[cc * kWave + lane]);
#pragma unroll
    for (int c = 0; c < LC; ++c)
        if (c < n) gv[c] = fma(lane_value(c_B, c), Sx, gv[c]);
    // coefficients of the chunk's intervals r = r_lo + c <= K - 2: stored
    // directly in the [K-1][4][2M] layout (each store 512 contiguous bytes);
    // in the [K-1][M][4][2] layout through the wave's 2 KB LDS slot, so that
    // the wave stores each interval's run of 32 modes as two 1 KB pieces
    const bool pm = jb.acoef_pmajor != 0;
    const int k0 = blk * (kFitSeriesPerBlock / 2);
    const int ns = min(kFitSeriesPerBlock, 2 * M - blk * kFitSeriesPerBlock);
    double *slot = bs0 + NW + (size_t)w * 4 * kWave;
#pragma unroll
    for (int c = 0; c < LC; ++c) {
        const int r = r_lo + c;
        if (c < n && r <= K - 2) {
            const double y0 = yv[c + 2], y1 = yv[c + 3];
            // s_{r+1}: past the chunk's last row, the next chunk's first
            const double s1 = (c + 1 < LC && c + 1 < n) ? gv[c + 1 < LC ? c + 1 : c] : Sx;
            const double s0 = gv[c];
            const double ir = lane_value(c_ih, c);
            const double dr = (y1 - y0) * ir;
            const double c2 = (3.0 * dr - 2.0 * s0 - s1) * ir, c3 = (s0 + s1 - 2.0 * dr) * (ir * ir);
            if (pm) {
                if (live) {
                    double *orow = jb.acoef + (size_t)r * 8 * M + q;
                    const size_t ps = 2 * (size_t)M;
                    orow[0] = y0;
                    orow[ps] = s0;
                    orow[2 * ps] = c2;
                    orow[3 * ps] = c3;
                }
            } else {
                double *d = slot + 8 * (lane >> 1) + (lane & 1);
                d[0] = y0;
                d[2] = s0;
                d[4] = c2;
                d[6] = c3;
                lds_wave_sync();
                const double2 *rd = (const double2 *)slot;
                double2 *dst = (double2 *)(jb.acoef + ((size_t)r * M + k0) * 8);
                const double2 v0 = rd[lane], v1 = rd[kWave + lane];
                if (lane < 2 * ns) dst[lane] = v0;               // run of 4 ns doubles
                if (kWave + lane < 2 * ns) dst[kWave + lane] = v1;
                lds_wave_sync();
            }
        }
    }
    if (up_x >= 0) {
        if (up_x < up_end) jb.up_dst[up_x] = up_w;
        for (long long x = up_x + (long long)blockDim.x; x < up_end; x += blockDim.x)
            jb.up_dst[x] = jb.up_src[x];
    }
}

// Workgroups 0 .. n_ph-1 fit the phases, the rest the amplitude series; t:
// the knot times.
__device__ __forceinline__ void fit_body(const FitJob &jb, const double *t, double *lds) {
    if ((int)blockIdx.x < jb.n_ph) {
        fit_phase_dd(jb, t, blockIdx.x, lds);
        return;
    }
    if ((int)blockIdx.x - jb.n_ph >= jb.amp_blocks) return;
    if (jb.K <= kFitStageKnots)
        fit_amplitudes_staged(jb, t, blockIdx.x - jb.n_ph, lds);
    else
        fit_amplitudes_stream(jb, t, blockIdx.x - jb.n_ph, lds);
}

// Single-request fit.  Grids of at most kFitStageKnots knots also arrive in
// the launch's arguments (kt), so no workgroup waits on the host-memory
// staging slot for them.
__global__ __launch_bounds__(256) void fit_kernel(FitJob jb, FitKnots kt) {
    extern __shared__ double lds_fit[];
    fit_body(jb, jb.K <= kFitStageKnots ? kt.t : jb.t, lds_fit);
}

__global__ __launch_bounds__(256) void fit_batch_kernel(const FitJob *jobs) {
    extern __shared__ double lds_fit[];
    const FitJob jb = jobs[blockIdx.y];
    fit_body(jb, jb.t, lds_fit);
}

// ===========================================================================
// Prepare stage.
// ===========================================================================

// starts[i] = min{ j in [0, n] : t_start + j dt >= t_i } (binary64 times).
__device__ long long dev_interval_start(double ti, double t_start, double dt, long long n) {
    double est = ceil((ti - t_start) / dt);
    long long j;
    if (!(est > 0.0)) j = 0;
    else if (est >= (double)n) j = n;
    else j = (long long)est;
    while (j > 0 && dev_sample_time(t_start, dt, j - 1) >= ti) --j;
    while (j < n && dev_sample_time(t_start, dt, j) < ti) ++j;
    return j;
}

// Samples of part p that lie in interval i, [lo, hi), and where its short
// tiles start (every tile lies inside one interval and one part).
struct PieceRange {
    long long lo, hi, split;
};

__device__ __forceinline__ PieceRange piece_range(long long a, long long e, long long n,
                                                  int parts, int p, long long short_len) {
    const long long b0 = part_begin(n, parts, p), b1 = part_begin(n, parts, p + 1);
    PieceRange r;
    r.lo = max(a, b0);
    r.hi = max(r.lo, min(e, b1));
    const long long s0 = b1 - min(b1 - b0, short_len);
    r.split = min(r.hi, max(r.lo, s0));
    return r;
}

// ceil(a / b) for 0 <= a < 2^53 and b > 0, exactly: a binary64 estimate (off
// by at most one) corrected with integer products, instead of the long
// instruction sequence of a 64-bit integer division.
__device__ __forceinline__ long long ceil_div_pos(long long a, int b) {
    long long q = (long long)((double)a / (double)b);
    if (q * b < a) ++q;
    if (q > 0 && (q - 1) * b >= a) --q;
    return q;
}

__device__ int piece_tiles(const PrepJob &jb, int p, int i) {
    const PieceRange r = piece_range(jb.starts[i], jb.starts[i + 1], jb.n, jb.parts, p,
                                     jb.short_len);
    return (int)(ceil_div_pos(r.split - r.lo, jb.tile) +
                 ceil_div_pos(r.hi - r.split, jb.short_tile));
}

__device__ void prep_intervals(const PrepJob &jb) {
    const int tid = threadIdx.x;
    const int K = jb.K;
    for (int i = tid; i < K; i += blockDim.x) {
        long long s;
        if (i == 0) s = 0;
        else if (i == K - 1) s = jb.n;
        else s = dev_interval_start(jb.t[i], jb.t_start, jb.dt, jb.n);
        jb.starts[i] = s;
    }
    __syncthreads();
    // per part (one wave each): tiles per interval and their exclusive prefix,
    // 64 intervals at a time by a shuffle scan
    const int P = K - 1;
    const int lane = tid & (kWave - 1), waves = blockDim.x / kWave;
    for (int pt = tid / kWave; pt < jb.parts; pt += waves) {
        int *tp = jb.tile_pref + (size_t)pt * K;
        int run = 0;
        for (int c0 = 0; c0 < P; c0 += kWave) {
            const int i = c0 + lane;
            const int cnt = (i < P) ? piece_tiles(jb, pt, i) : 0;
            int incl = cnt;
            for (int off = 1; off < kWave; off <<= 1) {
                const int v = __shfl_up(incl, off);
                if (lane >= off) incl += v;
            }
            if (i < P) tp[i] = run + incl - cnt;
            run += __shfl(incl, kWave - 1);
        }
        if (lane == 0) tp[P] = run;
    }
}

// Harmonic weight of one contributor: -2Y_lm for a listed mode and
// (-1)^{l+k} -2Y_{l,-m} for its mirror (Eq. (9); k = 0 in Schwarzschild).
__device__ void prep_harmonic(const PrepJob &jb, int e) {
    if (e >= jb.n_src) return;
    const int2 s = jb.term_src[e];
    const int l = s.y & 255, m = (s.y >> 8) & 255, mir = (s.y >> 16) & 1;
    const int kp = ((s.y >> 17) & 127) - 64;
    double yr, yi;
    if (!mir) {
        few_swsh_m2(l, m, jb.theta, jb.phi, &yr, &yi);
    } else {
        few_swsh_m2(l, -m, jb.theta, jb.phi, &yr, &yi);
        if ((l + kp) & 1) {
            yr = -yr;
            yi = -yi;
        }
    }
    jb.ybuf[e] = make_double2(yr, yi);
}

// Fold the l-sum for one (interval, term) pair:
//   C_term = scale * sum_e Y_e * (A_k or conj(A_k)),
// rescaled to u = x / h_i (coefficient p times h_i^p).
template <typename Real>
__device__ void fold_pair(const PrepJob &jb, int i, int term) {
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    auto add = [&](double2 w, int2 src, const double *a) {
        const double sgn = ((src.y >> 16) & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double ar = a[2 * q], ai = sgn * a[2 * q + 1];
            acc[2 * q] += w.x * ar - w.y * ai;
            acc[2 * q + 1] += w.x * ai + w.y * ar;
        }
    };
    // acoef [K-1][M][4][2] (vector-path requests): the 8 values of mode k on
    // interval i are contiguous, one 64-byte segment per contributor
    const double *arow = jb.acoef + (size_t)i * 8 * jb.M;
    auto load8 = [&](int k, double *a) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const double2 v = *(const double2 *)(arow + 8 * (size_t)k + 2 * p);
            a[2 * p] = v.x;
            a[2 * p + 1] = v.y;
        }
    };
    const int ea = jb.term_ptr[term], eb = jb.term_ptr[term + 1];
    int e = ea;
    // four contributors at a time: their weights, indices and coefficient rows
    // are all loaded before any is added (in contributor order, as one by one)
    for (; e + 4 <= eb; e += 4) {
        double2 w[4];
        int2 src[4];
        double av[4][8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w[j] = jb.ybuf[e + j];
            src[j] = jb.term_src[e + j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) load8(src[j].x, av[j]);
#pragma unroll
        for (int j = 0; j < 4; ++j) add(w[j], src[j], av[j]);
    }
    for (; e < eb; ++e) {
        double a[8];
        load8(jb.term_src[e].x, a);
        add(jb.ybuf[e], jb.term_src[e], a);
    }
    const double h = jb.t[i + 1] - jb.t[i];
    double f = jb.scale;
    // terms are stored in reverse order (position n_terms - 1 - term), so the
    // summation walks each segment from its highest n upwards in memory
    Real *dst = (Real *)jb.table + ((size_t)i * jb.n_terms + (jb.n_terms - 1 - term)) * 8;
    if (jb.scale_im == 0.0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dst[2 * q] = (Real)(acc[2 * q] * f);
            dst[2 * q + 1] = (Real)(acc[2 * q + 1] * f);
            f *= h;
        }
    } else {
        // complex overall factor (scale, scale_im) (the detector-frame rotation)
        double g = jb.scale_im;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dst[2 * q] = (Real)(acc[2 * q] * f - acc[2 * q + 1] * g);
            dst[2 * q + 1] = (Real)(acc[2 * q] * g + acc[2 * q + 1] * f);
            f *= h;
            g *= h;
        }
    }
}

// Prepare and fold in one launch.  Workgroup 0 computes the interval starts
// and the per-part tile prefixes; workgroup 1 + g folds the group of
// fold_terms consecutive terms starting at g fold_terms over every interval
// (fold_terms is chosen so that a group is about one (interval, term) pair per
// lane).
// The group first forms the harmonic weight of each of its contributors (each
// contributor belongs to one term, so each weight is formed once, by the one
// workgroup that reads it), then folds.  Consecutive lanes take consecutive
// terms of one interval, so table stores are contiguous.
template <typename Real>
__device__ void prepare_body(const PrepJob &jb, int b) {
    if (b == 0) {
        prep_intervals(jb);
        return;
    }
    const int t0 = (b - 1) * jb.fold_terms;
    if (t0 >= jb.n_terms) return;                   // uniform per workgroup
    const int nt = min(jb.fold_terms, jb.n_terms - t0);
    const int e0 = jb.term_ptr[t0], e1 = jb.term_ptr[t0 + nt];
    for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) prep_harmonic(jb, e);
    __syncthreads();                                // weights visible to the workgroup
    const int pairs = (jb.K - 1) * nt;
    for (int q = threadIdx.x; q < pairs; q += blockDim.x)
        fold_pair<Real>(jb, q / nt, t0 + q % nt);
}

template <typename Real>
__global__ __launch_bounds__(256) void prepare_kernel(PrepJob jb) {
    prepare_body<Real>(jb, blockIdx.x);
}

template <typename Real>
__global__ __launch_bounds__(256) void prepare_batch_kernel(const PrepJob *jobs) {
    const PrepJob jb = jobs[blockIdx.y];
    prepare_body<Real>(jb, blockIdx.x);
}

// ===========================================================================
// Summation stage.  No contraction: every sample goes through the same rounded
// operations whatever the tile shape, so results do not depend on tiling.
// ===========================================================================
#pragma clang fp contract(off)

// One reduced phase at one sample (in [-pi, pi]).  c: the interval's [4][2]
// double-double cubic of that phase.
template <bool DD>
__device__ __forceinline__ double phase_eval(const FEW_AS4 double *c, dd x) {
    if (DD) {
        dd v = dd_make(c[6], c[7]);
        v = dd_add(dd_mul(v, x), dd_make(c[4], c[5]));
        v = dd_add(dd_mul(v, x), dd_make(c[2], c[3]));
        v = dd_mul(v, x);
        v = dd_add(v, dd_make(c[0], c[1]));
        return dd_reduce_2pi(v).hi;
    }
    const double xx = x.hi;
    const double v = fma(fma(fma(c[6], xx, c[4]), xx, c[2]), xx, c[0]);
    return d_reduce_2pi(v);
}

// One phase at one sample, not reduced: the interval's binary64 cubic (the
// leading parts of the double-double coefficients) at offset x.
__device__ __forceinline__ double phase_raw(const FEW_AS4 double *c, double x) {
    return fma(fma(fma(c[6], x, c[4]), x, c[2]), x, c[0]);
}

// e^{-i a} for a reduced phase a in [-pi, pi] (binary64): the binary32 path
// rounds a to binary32 and takes the binary32 sincos (harmonics are binary32
// there), the binary64 path the binary64 one.
template <typename Real>
__device__ __forceinline__ void unit_phasor(double a, Real *re, Real *im) {
    if constexpr (sizeof(Real) == 4) {
        float sn, cs;
        sincosf((float)a, &sn, &cs);
        *re = cs;
        *im = -sn;
    } else {
        double sn, cs;
        sincos(a, &sn, &cs);
        *re = cs;
        *im = -sn;
    }
}

// Per-lane state of SL samples of one tile.  NP = 3 (generic Kerr) adds the
// polar phase and e^{-i Phi_theta}.
template <typename Real, int SL, int NP>
struct LaneState {
    static constexpr int ST = NP == 3 ? SL : 1;
    Real u[SL], fr[SL], fi[SL], er[SL], ei[SL], tr[ST], ti[ST];
    double pf[SL], pr[SL], pt[ST];
    long long jj[SL];
    Real hr[SL], hq[SL], cr[SL], cq[SL], zr[SL], zi[SL];
    Real gr[SL], gi[SL];    // binary32: sum of the closed term groups
    int pm, pk, pn;
};

// Segment record x = m + 256 k (k = 0 in Schwarzschild).
__device__ __forceinline__ int seg_k(int x) { return (x + 128) >> 8; }

// Knot interval of tile `local` (tp: tiles before each interval of one part).
__device__ __forceinline__ int tile_interval(const FEW_AS4 int *tp, int K, int local) {
    int lo = 0, hi = K - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tp[mid] <= local) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Per-sample setup: samples j0 + s * 64 + lane (s < SL), valid below j1.
template <typename Real, int SL, bool DD, int NP>
__device__ __forceinline__ void lane_setup(LaneState<Real, SL, NP> &L, const SumJob &jb, int iv,
                                           long long j0, long long j1) {
    const int lane = threadIdx.x & (kWave - 1);
    const FEW_AS4 double *tk = cptr(jb.t);
    const double ti = tk[iv];
    const double inv_h = 1.0 / (tk[iv + 1] - ti);
    const FEW_AS4 double *pc = cptr(jb.pcoef) + (size_t)iv * 8 * NP;   // Phi_phi, Phi_r (, Phi_theta)
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        long long j = j0 + s * kWave + lane;
        L.jj[s] = j;
        if (j >= j1) j = j1 - 1;
        const double tj = dev_sample_time(jb.t_start, jb.dt, j);
        const dd x = two_sum(tj, -ti);
        L.pf[s] = phase_eval<DD>(pc, x);
        L.pr[s] = phase_eval<DD>(pc + 8, x);
        L.u[s] = (Real)(x.hi * inv_h);
        unit_phasor<Real>(L.pf[s], &L.er[s], &L.ei[s]);
        unit_phasor<Real>(L.pr[s], &L.fr[s], &L.fi[s]);
        if constexpr (NP == 3) {
            L.pt[s] = phase_eval<DD>(pc + 16, x);
            unit_phasor<Real>(L.pt[s], &L.tr[s], &L.ti[s]);
        }
        L.hr[s] = L.hq[s] = L.cr[s] = L.cq[s] = (Real)0;
        L.zr[s] = L.zi[s] = (Real)0;
        L.gr[s] = L.gi[s] = (Real)0;
    }
    L.pm = INT_MIN / 2;
    L.pk = INT_MIN / 2;
    L.pn = INT_MIN / 2;
}

// The 8 coefficients of one term: scalar loads from the constant address space,
// or two 16-byte LDS reads (every lane of a wave reads the same address, so the
// LDS broadcasts).
template <typename Real>
__device__ __forceinline__ void load_term(const FEW_AS4 Real *cp, Real *c) {
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = cp[i];
}

__device__ __forceinline__ void load_term(const float *cp, float *c) {
    const float4 a = *(const float4 *)cp;
    const float4 b = *(const float4 *)(cp + 4);
    c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w;
    c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
}

// One Horner step over n for every sample of the lane: S <- S f + C_n(u),
// with C_n's eight coefficients (c0r, c0i, ..., c3i) in c.  Binary32
// (coefficients in VGPRs) evaluates C_n(u) by Horner in u apart from the
// recurrence, leaving two dependent FMAs per term on it; binary64
// (coefficients in SGPRs, one scalar operand per instruction) chains all five
// FMAs of each component into the recurrence.
template <typename Real, int SL, int NP>
__device__ __forceinline__ void term_step(const LaneState<Real, SL, NP> &L, Real *sr, Real *si,
                                          const Real *c) {
    const Real c0r = c[0], c0i = c[1], c1r = c[2], c1i = c[3];
    const Real c2r = c[4], c2i = c[5], c3r = c[6], c3i = c[7];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const Real u = L.u[s];
        Real nr, ni;
        if constexpr (sizeof(Real) == 4) {
            // coefficients in VGPRs: cubic first, two FMAs on the recurrence
            const Real pr = fmar(fmar(fmar(c3r, u, c2r), u, c1r), u, c0r);
            const Real pi = fmar(fmar(fmar(c3i, u, c2i), u, c1i), u, c0i);
            nr = fmar(sr[s], L.fr[s], fmar(-si[s], L.fi[s], pr));
            ni = fmar(sr[s], L.fi[s], fmar(si[s], L.fr[s], pi));
        } else {
            // coefficients in SGPRs: one scalar operand per FMA
            const Real u2 = u * u, u3 = u2 * u;
            nr = fmar(sr[s], L.fr[s], c0r);
            nr = fmar(-si[s], L.fi[s], nr);
            nr = fmar(u, c1r, nr);
            nr = fmar(u2, c2r, nr);
            nr = fmar(u3, c3r, nr);
            ni = fmar(sr[s], L.fi[s], c0i);
            ni = fmar(si[s], L.fr[s], ni);
            ni = fmar(u, c1i, ni);
            ni = fmar(u2, c2i, ni);
            ni = fmar(u3, c3i, ni);
        }
        sr[s] = nr;
        si[s] = ni;
    }
}

// One segment: seed e^{-i(m Phi_phi + k Phi_theta + n_lo Phi_r)} (chained
// from the previous segment's by e^{-i Phi_phi} when only m steps by one, or by
// e^{-i Phi_theta} when only k does, at the same n_lo; else one sincos),
// Horner over its terms in f = e^{-i Phi_r} from the highest n down,
//   S <- S f + C_n(u),  C_n(u) = c0 + c1 u + c2 u^2 + c3 u^3,
// then h += seed * S (Kahan-compensated when COMP).  `last` points at the 8
// values (c0r, c0i, ..., c3i) of the segment's highest-n term; the lower-n
// terms follow it at a stride of 8 (the table stores terms in reverse order,
// so the walk runs upward in memory and the loads of two unrolled terms share
// one base register with immediate offsets).
template <typename Real, int SL, bool COMP, int NP, typename Ptr>
__device__ __forceinline__ void seg_step(LaneState<Real, SL, NP> &L, const int4 S, Ptr last) {
    const int k = NP == 3 ? seg_k(S.x) : 0;
    const int m = S.x - 256 * k;
    const bool step_m = m == L.pm + 1 && k == L.pk && S.y == L.pn;
    const bool step_k = NP == 3 && m == L.pm && k == L.pk + 1 && S.y == L.pn;
    if (step_m || step_k) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            Real gr, gi;
            if constexpr (NP == 3) {
                gr = step_k ? L.tr[s] : L.er[s];
                gi = step_k ? L.ti[s] : L.ei[s];
            } else {
                gr = L.er[s];
                gi = L.ei[s];
            }
            const Real a = L.zr[s] * gr - L.zi[s] * gi;
            const Real b = L.zr[s] * gi + L.zi[s] * gr;
            L.zr[s] = a;
            L.zi[s] = b;
        }
    } else {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            double ph = (double)m * L.pf[s] + (double)S.y * L.pr[s];
            if constexpr (NP == 3) ph = ph + (double)k * L.pt[s];
            unit_phasor<Real>(d_reduce_2pi(ph), &L.zr[s], &L.zi[s]);
        }
    }
    L.pm = m;
    L.pk = k;
    L.pn = S.y;
    Real sr[SL], si[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) sr[s] = si[s] = (Real)0;
    const int len = S.z;
    if constexpr (sizeof(Real) == 4) {
        // LDS operands: each pair of unrolled terms is read by four 16-byte
        // loads at immediate offsets from one base, waited on at once; the
        // other waves of the SIMD cover the latency.
#pragma unroll FEW_SEG_UNROLL
        for (int q = 0; q < len; ++q) {
            Real c[8];
            load_term(last + 8 * q, c);
            term_step<Real, SL, NP>(L, sr, si, c);
        }
    } else {
        // scalar-load operands: the next term is loaded into a second register
        // set while the current one is used, so each load has a term's FMAs
        // to return in (scalar loads may return out of order, so every wait is
        // for all of them); the last prefetch re-reads the last term, so it
        // stays in bounds.
        Ptr cp = last;
        Real c[8];
        load_term(cp, c);
#pragma unroll FEW_SEG_UNROLL
        for (int q = 0; q < len; ++q) {
            const Ptr np = (q + 1 < len) ? cp + 8 : cp;
            Real cn[8];
            load_term(np, cn);
            term_step<Real, SL, NP>(L, sr, si, c);
#pragma unroll
            for (int i = 0; i < 8; ++i) c[i] = cn[i];
            cp = np;
        }
    }
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const Real vr = L.zr[s] * sr[s] - L.zi[s] * si[s];
        const Real vi = L.zr[s] * si[s] + L.zi[s] * sr[s];
        if (COMP) {
            const Real yr = vr - L.cr[s];
            const Real tr = L.hr[s] + yr;
            L.cr[s] = (tr - L.hr[s]) - yr;
            L.hr[s] = tr;
            const Real yi = vi - L.cq[s];
            const Real ti2 = L.hq[s] + yi;
            L.cq[s] = (ti2 - L.hq[s]) - yi;
            L.hq[s] = ti2;
        } else {
            L.hr[s] += vr;
            L.hq[s] += vi;
        }
    }
}

// Value of the current (compensated) sum of sample s.
template <typename Real, int SL, bool COMP, int NP>
__device__ __forceinline__ void acc_value(const LaneState<Real, SL, NP> &L, int s, Real *re,
                                          Real *im) {
    *re = COMP ? L.hr[s] - L.cr[s] : L.hr[s];
    *im = COMP ? L.hq[s] - L.cq[s] : L.hq[s];
}

// Close a term group (binary32): add its value to the group total, restart
// the compensated sum, and make the next segment seed by sincos.
template <typename Real, int SL, bool COMP, int NP>
__device__ __forceinline__ void group_close(LaneState<Real, SL, NP> &L) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        Real vr, vi;
        acc_value<Real, SL, COMP, NP>(L, s, &vr, &vi);
        L.gr[s] = L.gr[s] + vr;
        L.gi[s] = L.gi[s] + vi;
        L.hr[s] = L.hq[s] = L.cr[s] = L.cq[s] = (Real)0;
    }
    L.pm = INT_MIN / 2;
    L.pk = INT_MIN / 2;
    L.pn = INT_MIN / 2;
}

// Final value of sample s: the group total (binary32, after the last group is
// closed) or the running sum (binary64).
template <typename Real, int SL, bool COMP, int NP>
__device__ __forceinline__ void lane_value(const LaneState<Real, SL, NP> &L, int s, Real *re,
                                           Real *im) {
    if constexpr (sizeof(Real) == 4) {
        *re = L.gr[s];
        *im = L.gi[s];
    } else {
        acc_value<Real, SL, COMP, NP>(L, s, re, im);
    }
}

template <typename Real, int SL, bool COMP, int NP>
__device__ __forceinline__ void lane_store(const LaneState<Real, SL, NP> &L, const SumJob &jb,
                                           long long j1) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        if (L.jj[s] < j1) {
            Real *o = (Real *)jb.out + 2 * L.jj[s];
            lane_value<Real, SL, COMP, NP>(L, s, &o[0], &o[1]);
        }
    }
}

// Inner-product epilogue: this lane's sums of Re(conj(d_j) h_j) and |h_j|^2
// over its valid samples, in binary64, with h_j exactly the value a store
// launch would write.
template <typename Real, int SL, bool COMP, int NP>
__device__ __forceinline__ double2 lane_inner(const LaneState<Real, SL, NP> &L,
                                              const SumJob &jb, long long j1) {
    double dh = 0.0, hh = 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        if (L.jj[s] < j1) {
            Real re, im;
            lane_value<Real, SL, COMP, NP>(L, s, &re, &im);
            const Real *d = (const Real *)jb.data + 2 * L.jj[s];
            const double hr = re, hi = im, dr = d[0], di = d[1];
            dh = dh + (dr * hr + di * hi);
            hh = hh + (hr * hr + hi * hi);
        }
    }
    return make_double2(dh, hh);
}

// Sum over the 64 lanes of a wave by a fixed butterfly (every lane ends with
// the same bits: each step adds the same two values in either lane).
__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        v.x = v.x + __shfl_xor(v.x, off);
        v.y = v.y + __shfl_xor(v.y, off);
    }
    return v;
}

// Wave tile (binary64 path): 64 x SL consecutive samples [j0, j1) of interval
// iv, coefficients read by scalar loads straight into SGPR operands.
template <typename Real, int SL, bool COMP, bool DD, int NP, bool INNER>
__device__ __forceinline__ double2 sum_wave_run(const SumJob &jb, int iv, long long j0,
                                                long long j1) {
    static_assert(sizeof(Real) == 8, "binary32 terms are read from LDS only");
    LaneState<Real, SL, NP> L;
    lane_setup<Real, SL, DD, NP>(L, jb, iv, j0, j1);
    const FEW_AS4 Real *tab = cptr((const Real *)jb.table) + (size_t)iv * jb.n_terms * 8;
    for (int g = 0; g < jb.n_segs; ++g) {
        const int4 S = load_uniform(jb.segs + g);
        seg_step<Real, SL, COMP, NP>(L, S, tab + (size_t)(jb.n_terms - S.w - S.z) * 8);
    }
    if constexpr (INNER) {
        return lane_inner<Real, SL, COMP, NP>(L, jb, j1);
    } else {
        lane_store<Real, SL, COMP, NP>(L, jb, j1);
        return make_double2(0.0, 0.0);
    }
}

// Wave tile `local` of part `pt` of a request (binary64 launches use long
// tiles only).
template <typename Real, bool COMP, bool DD, int NP, bool INNER>
__device__ __forceinline__ double2 sum_tile(const SumJob &jb, int pt, int local) {
    const FEW_AS4 int *tp = cptr(jb.tile_pref) + (size_t)pt * jb.K;
    if (local >= tp[jb.K - 1]) return make_double2(0.0, 0.0);
    const int iv = tile_interval(tp, jb.K, local);
    const FEW_AS4 long long *st = cptr(jb.starts);
    const PieceRange pr = piece_range(st[iv], st[iv + 1], jb.n, jb.parts, pt, 0);
    constexpr int LT = kWave * kSamplesPerLaneF64;
    const long long j0 = pr.lo + (long long)(local - tp[iv]) * LT;
    return sum_wave_run<Real, kSamplesPerLaneF64, COMP, DD, NP, INNER>(jb, iv, j0,
                                                                       min(j0 + LT, pr.hi));
}

// Workgroup tile (binary32 path): 4 waves x 64 x SL consecutive samples
// [base, j1) of interval iv.  The workgroup stages the interval's coefficients
// in LDS, one chunk of whole segments (at most kChunkTerms terms) at a time, and
// every wave reads each term with broadcast LDS loads into VGPRs: FMAs without
// scalar operands issue at twice the rate on gfx950.  Every lane of the
// workgroup reaches every barrier.
template <typename Real, int SL, bool COMP, bool DD, int NP, bool INNER>
__device__ __forceinline__ double2 sum_wg_run(const SumJob &jb, int iv, long long base,
                                              long long j1, Real *buf) {
    static_assert(sizeof(Real) == 4, "binary64 terms are read by scalar loads");
    constexpr int WT = kWave * SL;                  // samples per wave
    const int wave = threadIdx.x / kWave;
    // a wave past the end of a partial tile only helps stage coefficients
    const bool busy = base + (long long)wave * WT < j1;
    LaneState<Real, SL, NP> L;
    if (busy) lane_setup<Real, SL, DD, NP>(L, jb, iv, base + (long long)wave * WT, j1);
    const Real *tab = (const Real *)jb.table + (size_t)iv * jb.n_terms * 8;
    const FEW_AS4 int *ch = cptr(jb.chunks);
    for (int c = 0; c < jb.n_chunks; ++c) {
        const int g0 = ch[c], g1 = ch[c + 1];
        const int t0 = load_uniform(jb.segs + g0).w;
        const int4 Sl = load_uniform(jb.segs + g1 - 1);
        const int t1 = Sl.w + Sl.z;                 // terms [t0, t1), stored reversed
        const int nv = (t1 - t0) * 8 * (int)sizeof(Real) / 16;
        __syncthreads();                            // previous chunk fully consumed
        const float4 *src = (const float4 *)(tab + (size_t)(jb.n_terms - t1) * 8);
        float4 *dst = (float4 *)buf;
        for (int v = threadIdx.x; v < nv; v += blockDim.x) dst[v] = src[v];
        __syncthreads();
        if (busy) {
            for (int g = g0; g < g1; ++g) {
#pragma unroll
                for (int q = 0; q < kTermGroups - 1; ++q)
                    if (g == jb.grp[q]) group_close<Real, SL, COMP, NP>(L);
                const int4 S = load_uniform(jb.segs + g);
                seg_step<Real, SL, COMP, NP>(L, S, buf + (t1 - S.w - S.z) * 8);
            }
        }
    }
    if (!busy) return make_double2(0.0, 0.0);
    // close the last group, then any empty groups after it (each adds zero,
    // as in a term-split tile)
    group_close<Real, SL, COMP, NP>(L);
#pragma unroll
    for (int q = 0; q < kTermGroups - 1; ++q)
        if (jb.grp[q] == jb.n_segs) group_close<Real, SL, COMP, NP>(L);
    if constexpr (INNER) {
        return lane_inner<Real, SL, COMP, NP>(L, jb, j1);
    } else {
        lane_store<Real, SL, COMP, NP>(L, jb, j1);
        return make_double2(0.0, 0.0);
    }
}

// Term-split tile (binary32): 64 x SL samples [base, j1) of interval iv, taken
// by all four waves; wave w sums term group w (segments [grp[w-1], grp[w])),
// staging it kSplitTerms terms (whole segments) at a time in its own quarter
// of the LDS buffer, so the waves need no barrier until they combine.  Each
// wave leaves its group value in its quarter; wave 0 adds the four in group
// order, starting from zero, exactly as a long tile closes its groups.  Needs
// every segment to fit a quarter (checked on the host).
template <typename Real, int SL, bool COMP, bool DD, int NP, bool INNER>
__device__ __forceinline__ double2 sum_wg_split(const SumJob &jb, int iv, long long base,
                                                long long j1, Real *buf) {
    static_assert(sizeof(Real) == 4, "term-split tiles are binary32 tiles");
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    LaneState<Real, SL, NP> L;
    lane_setup<Real, SL, DD, NP>(L, jb, iv, base, j1);
    const int gb = wave == 0 ? 0 : jb.grp[wave - 1];
    const int ge = wave == kTermGroups - 1 ? jb.n_segs : jb.grp[wave];
    Real *wb = buf + (size_t)wave * kSplitTerms * 8;
    const Real *tab = (const Real *)jb.table + (size_t)iv * jb.n_terms * 8;
    for (int g = gb; g < ge;) {
        // whole segments [g, h) with at most kSplitTerms terms
        const int t0 = load_uniform(jb.segs + g).w;
        int h = g, t1 = t0;
        while (h < ge) {
            const int4 S = load_uniform(jb.segs + h);
            if (S.w + S.z - t0 > kSplitTerms) break;
            t1 = S.w + S.z;
            ++h;
        }
        // terms [t0, t1) are stored reversed: one contiguous run
        const int nv = (t1 - t0) * 8 * (int)sizeof(Real) / 16;
        const float4 *src = (const float4 *)(tab + (size_t)(jb.n_terms - t1) * 8);
        float4 *dst = (float4 *)wb;
        for (int v = lane; v < nv; v += kWave) dst[v] = src[v];
        __builtin_amdgcn_wave_barrier();
        for (; g < h; ++g) {
            const int4 S = load_uniform(jb.segs + g);
            seg_step<Real, SL, COMP, NP>(L, S, wb + (t1 - S.w - S.z) * 8);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // this wave's group value, next to its staging area
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        Real vr, vi;
        acc_value<Real, SL, COMP, NP>(L, s, &vr, &vi);
        wb[(s * kWave + lane) * 2] = vr;
        wb[(s * kWave + lane) * 2 + 1] = vi;
    }
    __syncthreads();
    if (wave != 0) return make_double2(0.0, 0.0);
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        Real gr = (Real)0, gi = (Real)0;
#pragma unroll
        for (int w = 0; w < kTermGroups; ++w) {
            const Real *v = buf + (size_t)w * kSplitTerms * 8 + (s * kWave + lane) * 2;
            gr = gr + v[0];
            gi = gi + v[1];
        }
        L.gr[s] = gr;
        L.gi[s] = gi;
    }
    if constexpr (INNER) {
        return lane_inner<Real, SL, COMP, NP>(L, jb, j1);
    } else {
        lane_store<Real, SL, COMP, NP>(L, jb, j1);
        return make_double2(0.0, 0.0);
    }
}

// Tile `local` of part `pt` of a request: the part's samples in its interval,
// [lo, hi), are covered by long tiles up to `split` and short tiles after it.
// The branch is uniform per workgroup.
template <typename Real, bool COMP, bool DD, int NP, bool INNER, bool SPLIT>
__device__ __forceinline__ double2 sum_wg_tile(const SumJob &jb, int pt, int local, Real *buf) {
    const FEW_AS4 int *tp = cptr(jb.tile_pref) + (size_t)pt * jb.K;
    if (local >= tp[jb.K - 1]) return make_double2(0.0, 0.0);
    const int iv = tile_interval(tp, jb.K, local);
    const FEW_AS4 long long *st = cptr(jb.starts);
    const PieceRange pr = piece_range(st[iv], st[iv + 1], jb.n, jb.parts, pt, jb.short_len);
    constexpr int LT = 4 * kWave * kSamplesPerLaneF32;
    constexpr int ST = 4 * kWave * kSamplesPerLaneShort;
    constexpr int XT = kWave * kSamplesPerLaneF32;   // term-split tile
    const int n_long = (int)((pr.split - pr.lo + LT - 1) / LT);
    const int r = local - tp[iv];
    if (r < n_long) {
        const long long base = pr.lo + (long long)r * LT;
        return sum_wg_run<Real, kSamplesPerLaneF32, COMP, DD, NP, INNER>(
            jb, iv, base, min(base + LT, pr.split), buf);
    } else if (SPLIT && jb.split) {
        const long long base = pr.split + (long long)(r - n_long) * XT;
        return sum_wg_split<Real, kSamplesPerLaneF32, COMP, DD, NP, INNER>(
            jb, iv, base, min(base + XT, pr.hi), buf);
    } else {
        const long long base = pr.split + (long long)(r - n_long) * ST;
        return sum_wg_run<Real, kSamplesPerLaneShort, COMP, DD, NP, INNER>(
            jb, iv, base, min(base + ST, pr.hi), buf);
    }
}

// Workgroups are numbered so that each of the 8 XCDs (which receive workgroups
// round-robin) works on one contiguous eighth of the range, i.e. on a few knot
// intervals whose coefficient tables stay in its own L2.
__device__ __forceinline__ int xcd_block_id() {
    const int nb = gridDim.x;                       // multiple of 8
    const int b = blockIdx.x;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

__device__ __forceinline__ int xcd_wave_id() {
    return xcd_block_id() * (blockDim.x / kWave) + (threadIdx.x / kWave);
}

// Batched launch: job j owns slots [wave_base_j, wave_base_{j+1}).
__device__ __forceinline__ int find_job(const SumJob *jobs, int n_jobs, int w) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int base = *cptr(&jobs[mid].wave_base);
        if (base <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---- binary64: one wave per tile -------------------------------------------
// One request: workgroup b runs on XCD b mod 8 (workgroups are dealt to the
// XCDs in turn), so part b mod parts is that XCD's; its waves take the part's
// tiles in dispatch order.  `slots`: wave tiles per part.
// INNER: every wave writes its tile's partial sums (zero without a tile) to
// partial[b * 4 + wave].
template <typename Real, bool COMP, bool DD, int NP, bool INNER>
__global__ __launch_bounds__(256) FEW_F64_ATTR void sum_kernel(SumJob jb, int slots) {
    const int b = blockIdx.x;
    const int pt = b % jb.parts;
    const int w = __builtin_amdgcn_readfirstlane(
        (int)((b / jb.parts) * (blockDim.x / kWave) + threadIdx.x / kWave));
    double2 v = make_double2(0.0, 0.0);
    if (w < slots) v = sum_tile<Real, COMP, DD, NP, INNER>(jb, pt, w);
    if constexpr (INNER) {
        v = wave_sum(v);
        if ((threadIdx.x & (kWave - 1)) == 0)
            jb.partial[(size_t)b * (blockDim.x / kWave) + threadIdx.x / kWave] = v;
    }
}

template <typename Real, bool COMP, bool DD>
__device__ __forceinline__ void sum_slot(const SumJob *jobs, int n_jobs, int w) {
    const int jx = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, w));
    const SumJob jb = load_uniform(jobs + jx);
    sum_tile<Real, COMP, DD, 2, false>(jb, 0, w - jb.wave_base);
}

template <typename Real, bool COMP, bool DD>
__global__ __launch_bounds__(256) FEW_F64_ATTR void sum_batch_kernel(const SumJob *jobs, int n_jobs,
                                                        int slots) {
    const int w = __builtin_amdgcn_readfirstlane(xcd_wave_id());
    if (w >= slots) return;
    sum_slot<Real, COMP, DD>(jobs, n_jobs, w);
}

// Persistent variant: a fixed grid of waves pulls wave slots from one atomic
// counter until all `slots` are handed out; every wave then exits.
template <typename Real, bool COMP, bool DD>
__global__ __launch_bounds__(256) FEW_F64_ATTR void sum_persistent_kernel(const SumJob *jobs, int n_jobs,
                                                             int slots, unsigned *counter) {
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        unsigned v = 0;
        if (lane == 0) v = atomicAdd(counter, 1u);
        const int w = __builtin_amdgcn_readfirstlane((int)v);
        if (w >= slots) break;
        sum_slot<Real, COMP, DD>(jobs, n_jobs, w);
    }
}

// ---- binary32: one workgroup per tile ---------------------------------------
// One request: workgroup b runs on XCD b mod 8, takes part b mod parts and
// that part's tiles in dispatch order, so each XCD reads the coefficients of its
// own intervals and ends on its short tiles while its last long tiles finish.
// `slots`: tiles per part.
// INNER: every workgroup writes its tile's partial sums (zero without a tile)
// to partial[b], adding its four waves in order.
template <typename Real, bool COMP, bool DD, int NP, bool INNER>
__global__ __launch_bounds__(256) FEW_SUM_ATTR void sum_wg_kernel(SumJob jb, int slots) {
    extern __shared__ float4 sum_lds[];
    const int b = blockIdx.x;
    const int local = b / jb.parts;     // < slots: the grid is parts x slots
    double2 v = sum_wg_tile<Real, COMP, DD, NP, INNER, true>(jb, b % jb.parts, local,
                                                       (Real *)sum_lds);
    if constexpr (INNER) {
        __shared__ double2 red[4];
        v = wave_sum(v);
        if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double2 t = red[0];
            for (int w = 1; w < (int)(blockDim.x / kWave); ++w) {
                t.x = t.x + red[w].x;
                t.y = t.y + red[w].y;
            }
            jb.partial[b] = t;
        }
    }
    (void)slots;
}

template <typename Real, bool COMP, bool DD>
__device__ __forceinline__ void sum_wg_slot(const SumJob *jobs, int n_jobs, int b, Real *buf) {
    const int jx = __builtin_amdgcn_readfirstlane(find_job(jobs, n_jobs, b));
    const SumJob jb = load_uniform(jobs + jx);
    sum_wg_tile<Real, COMP, DD, 2, false, false>(jb, 0, b - jb.wave_base, buf);
}

template <typename Real, bool COMP, bool DD>
__global__ __launch_bounds__(256) void sum_wg_batch_kernel(const SumJob *jobs, int n_jobs,
                                                           int slots) {
    extern __shared__ float4 sum_lds[];
    const int b = xcd_block_id();
    if (b >= slots) return;
    sum_wg_slot<Real, COMP, DD>(jobs, n_jobs, b, (Real *)sum_lds);
}

// Persistent variant: workgroups pull tile slots from one atomic counter
// (lane 0 draws, the slot is broadcast through LDS) until all are handed out.
template <typename Real, bool COMP, bool DD>
__global__ __launch_bounds__(256) void sum_wg_persistent_kernel(const SumJob *jobs,
                                                                int n_jobs, int slots,
                                                                unsigned *counter) {
    extern __shared__ float4 sum_lds[];
    __shared__ int slot;
    for (;;) {
        if (threadIdx.x == 0) slot = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int b = slot;
        __syncthreads();
        if (b >= slots) break;
        sum_wg_slot<Real, COMP, DD>(jobs, n_jobs, b, (Real *)sum_lds);
    }
}

// ===========================================================================
// Matrix-core summation (binary32 output).  See the shape constants in
// few_internal.h: per knot interval and power p of u, the product of the
// coefficient matrix (rows: the real and imaginary part of each signed m;
// columns: (n, re/im)) with the matrix of harmonics (Re f^|n|, Im f^|n|) over
// the samples, f = e^{-i Phi_r}, on fp16 hi/lo operands with fp32
// accumulation; the sum over p is a Horner recurrence in u on the
// accumulators, and the rows are combined with e^{-i m Phi_phi}.
// ===========================================================================
typedef _Float16 mf_half8 __attribute__((ext_vector_type(8)));
typedef float mf_float4 __attribute__((ext_vector_type(4)));

// Fold and pack for the matrix-core path: workgroup 0 computes the interval
// starts and tile prefixes; each other workgroup folds one interval iv for
// one row tile mt (rows 8 mt .. 8 mt + 7, the signed m values m_r; numbering
// below) and writes its part of the fp16 operand table.
//
// Fold (Eqs. (9)-(10) for fixed viewing angles, Sec. IV): every term (m_r, n)
// is C = scale sum_contributors w A, with w = -2Y_{l, m_r} for a listed mode
// and (-1)^l -2Y_{l, m_r} for the mirror of a listed mode (m_r = -m, the
// amplitude conjugated), and coefficient p rescaled to u = x / h_i by h_i^p.
// The weights depend on (l, m_r) only, so the workgroup forms them once per
// row and l.  The folded values stay in LDS.
//
// Pack.  Row r is the pair of matrix rows 2r (real part) and 2r + 1
// (imaginary part).  For power p, column (a, c) multiplies Re w (c = 0) or
// Im w (c = 1), w = f^a, a = |n|.  The terms n = a and n = -a of the row
// (coefficients P and Q) contribute P w + Q conj(w) =
// ((Re P + Re Q) Re w + (Im Q - Im P) Im w) +
// i ((Im P + Im Q) Re w + (Re P - Re Q) Im w),
// so row 2r holds (Re P + Re Q, Im Q - Im P) and row 2r + 1 holds
// (Im P + Im Q, Re P - Re Q) (Q = 0 for a = 0).  Each pair of rows (signed m
// rows 2j and 2j + 1, which one lane of the product holds) is scaled by
// 2^-E, E the exponent of the pair's largest |coefficient| on the interval
// (so scaled values stay below 2), and split into hi = fp16(v) and
// lo = fp16(v - hi), both from binary64.  Table layout, per interval:
// [3 - p][mt][t][hi, lo][lane 64][8 values] (p descending, the order of the
// Horner recurrence that reads it), lane l's operand fragment of
// v_mfma_f32_16x16x32_f16: matrix row l % 16 of the tile, columns
// a = 16 t + 4 (l / 16) + i / 2 and c = i % 2 for value i.
constexpr int kFoldSegs = 64;                       // segments of a row tile kept in LDS

__device__ void fold_pack_body(const PrepJob &jb, int b) {
    if (b == 0) {
        prep_intervals(jb);
        return;
    }
    // workgroup 1 + 8 (kMfMT (iv / 8) + mt) + iv % 8 folds row tile mt of
    // interval iv: the tiles of one interval are 8 workgroups apart and so run
    // on one XCD (workgroup b runs on XCD b mod 8), whose L2 then serves the
    // coefficient rows that several tiles read (a mode's own and mirror terms)
    const int c = b - 1, q = c >> 3;
    const int mt = q % kMfMT, iv = 8 * (q / kMfMT) + (c & 7);
    if (iv >= jb.K - 1) return;                     // uniform per workgroup
    constexpr int NL = kMaxL + 1, NN = 2 * kMfA;    // l = 0..30; n + kMfA - 1 in [0, NN - 1)
    __shared__ double2 yw[8][NL];
    __shared__ double cf[8][NN][8];
    __shared__ double rsc[8];
    __shared__ int rowm[9];
    __shared__ int rowmv[8];                        // m_r of the tile's rows
    __shared__ double2 trig[9];                     // (cos, sin) of theta / 2 and of m_r phi
    __shared__ int2 segv[kFoldSegs];
    const int tid = threadIdx.x;
    const int r0 = 8 * mt;
    // the tile's segments [g0, g1); its terms are one contiguous run [t0, t1)
    // (uniform values: scalar loads)
    const int g0 = jb.mrows[min(r0, jb.n_mrows)].y, g1 = jb.mrows[min(r0 + 8, jb.n_mrows)].y;
    const int t0 = g0 < jb.n_segs ? jb.segs[g0].w : jb.n_terms;
    const int t1 = g1 < jb.n_segs ? jb.segs[g1].w : jb.n_terms;
    // This lane's first term: its contributor range is requested first, its
    // first three contributor indices once that has arrived (after the first
    // barrier) and before the weights are formed (from LDS only), so that the
    // rows can be requested as soon as the weights are in place.
    int tt = t0 + tid;
    int ea = 0, eb = 0;
    if (tt < t1) {
        ea = jb.term_ptr[tt];
        eb = jb.term_ptr[tt + 1];
    }
    // the tile's segments and its rows' (m, first segment), both requested
    // before either is used (every lane loads, at clamped indices, so that
    // no load sits under a branch)
    const int4 S = jb.segs[min(g0 + tid, max(g1 - 1, 0))];
    const int2 R = jb.mrows[min(r0 + min(tid, 8), jb.n_mrows)];
    if (tid < g1 - g0 && tid < kFoldSegs) segv[tid] = make_int2(S.w, S.y);
    if (tid < 9) {
        const int r = r0 + tid;
        rowm[tid] = R.y;                            // first segment
        const int m = r < jb.n_mrows ? R.x : 0;
        if (tid < 8) rowmv[tid] = m;
        double sv, cv;
        if (tid == 8)
            sincos(0.5 * jb.theta, &sv, &cv);
        else
            sincos((double)m * jb.phi, &sv, &cv);
        trig[tid] = make_double2(cv, sv);
    }
    for (int x = tid; x < 8 * NN * 8; x += blockDim.x) (&cf[0][0][0])[x] = 0.0;
    __syncthreads();
    // (clamped, unconditional loads; indices past eb are never used)
    int2 src[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) src[j] = jb.term_src[min(ea + j, max(eb - 1, 0))];
    for (int x = tid; x < 8 * NL; x += blockDim.x) {
        const int k = x / NL, l = x % NL, r = r0 + k;
        double yr = 0.0, yi = 0.0;
        if (r < jb.n_mrows) {
            const int m = rowmv[k];
            if (l >= 2 && l >= abs(m) && l <= jb.l_max)
                few_swsh_m2_cs(l, m, trig[8].x, trig[8].y, trig[k].x, trig[k].y, &yr, &yi);
        }
        yw[k][l] = make_double2(yr, yi);
    }
    __syncthreads();
    // the tile's segments (first term, n of the first term) in LDS when few
    const bool seg_lds = g1 - g0 <= kFoldSegs;
    auto seg_of = [&](int g) {
        if (seg_lds) return make_int2(segv[g - g0].x, segv[g - g0].y);
        const int4 S = jb.segs[g];
        return make_int2(S.w, S.y);
    };
    const double h = jb.t[iv + 1] - jb.t[iv];
    // acoef [K-1][4][2M] (matrix-core requests): coefficient p of mode k at
    // arow[p * 2M + 2k + {0, 1}], so lanes taking consecutive modes read
    // contiguous memory in each of the four planes
    const size_t ps = 2 * (size_t)jb.M;
    const double *arow = jb.acoef + (size_t)iv * 4 * ps;
    auto load8 = [&](int mode, double *a) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const double2 v = *(const double2 *)(arow + p * ps + 2 * (size_t)mode);
            a[2 * p] = v.x;
            a[2 * p + 1] = v.y;
        }
    };
    for (; tt < t1; tt += blockDim.x) {
        if (tt != t0 + tid) {
            ea = jb.term_ptr[tt];
            eb = jb.term_ptr[tt + 1];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                src[j] = ea + j < eb ? jb.term_src[ea + j] : make_int2(0, 0);
        }
        int g = g0;
        while (g + 1 < g1 && seg_of(g + 1).x <= tt) ++g;
        const int2 S = seg_of(g);
        int k = 0;
        while (k + 1 < 8 && rowm[k + 1] <= g) ++k;
        const int n = S.y + (tt - S.x);
        double acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = 0.0;
        auto add = [&](int2 cs, const double *a) {
            const int l = cs.y & 255, mir = (cs.y >> 16) & 1;
            double2 w = yw[k][l];
            if (mir && (l & 1)) w = make_double2(-w.x, -w.y);
            const double sgn = mir ? -1.0 : 1.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double ar = a[2 * q], ai = sgn * a[2 * q + 1];
                acc[2 * q] += w.x * ar - w.y * ai;
                acc[2 * q + 1] += w.x * ai + w.y * ar;
            }
        };
        // three contributors at a time, added in contributor order: their
        // coefficient rows are requested, then the next three indices (so
        // that those arrive while these rows do), then the rows are added
        for (int e = ea; e < eb; e += 3) {
            double av[3][8];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (e + j < eb) load8(src[j].x, av[j]);
            int2 nsrc[3];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                nsrc[j] = e + 3 + j < eb ? jb.term_src[e + 3 + j] : make_int2(0, 0);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (e + j < eb) add(src[j], av[j]);
#pragma unroll
            for (int j = 0; j < 3; ++j) src[j] = nsrc[j];
        }
        double f = jb.scale, fi = jb.scale_im;
        double *dst = cf[k][n + kMfA - 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dst[2 * q] = acc[2 * q] * f - acc[2 * q + 1] * fi;
            dst[2 * q + 1] = acc[2 * q] * fi + acc[2 * q + 1] * f;
            f *= h;
            fi *= h;
        }
    }
    __syncthreads();
    {
        const int k = tid >> 5, sub = tid & 31;     // 8 rows x 32 lanes
        double mx = 0.0;
        if (k < 8)
            for (int x = sub; x < NN * 8; x += 32) mx = fmax(mx, fabs((&cf[k][0][0])[x]));
        for (int off = 16; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 32));
        // one scale for the row pair 2j, 2j + 1 (rows k and k ^ 1, the two
        // rows one lane of the product holds): the epilogue applies it once
        mx = fmax(mx, __shfl_xor(mx, 32));
        if (k < 8 && sub == 0) {
            int e = 0;
            double sc = 0.0;
            float ms = 0.0f;
            if (mx > 0.0) {
                frexp(mx, &e);
                sc = ldexp(1.0, -e);
                ms = (float)ldexp(1.0, e);
            }
            rsc[k] = sc;
            jb.mscale[(size_t)iv * kMfRows + r0 + k] = ms;
        }
    }
    __syncthreads();
    _Float16 *dst = (_Float16 *)jb.mtab + (size_t)iv * kMfIntervalHalves;
    for (int it = tid; it < 4 * kMfT * 64; it += blockDim.x) {
        const int ln = it & 63, t = (it >> 6) % kMfT, p = (it >> 6) / kMfT;
        const int kk = (ln & 15) >> 1, comp = ln & 1, g = ln >> 4;
        const double sc = rsc[kk];
        mf_half8 hi, lo;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = 16 * t + 4 * g + j;
            const double pr = cf[kk][a + kMfA - 1][2 * p], pi = cf[kk][a + kMfA - 1][2 * p + 1];
            double qr = 0.0, qi = 0.0;
            if (a > 0) {
                qr = cf[kk][-a + kMfA - 1][2 * p];
                qi = cf[kk][-a + kMfA - 1][2 * p + 1];
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double v;
                if (comp == 0)
                    v = c == 0 ? pr + qr : qi - pi;
                else
                    v = c == 0 ? pi + qi : pr - qr;
                v = v * sc;
                // through binary32 (one instruction each way; the pair still
                // carries about 22 bits: lo takes the exact binary64 residual)
                const _Float16 hv = (_Float16)(float)v;
                hi[2 * j + c] = hv;
                lo[2 * j + c] = (_Float16)(float)(v - (double)hv);
            }
        }
        const size_t at =
            ((((size_t)(3 - p) * kMfMT + mt) * kMfT + t) * 2) * 512 + (size_t)ln * 8;
        *(mf_half8 *)(dst + at) = hi;
        *(mf_half8 *)(dst + at + 512) = lo;
    }
}

// 512 lanes: about one folded term per lane (the fold's dependent loads
// dominate), two operand items per lane in the pack; at most 128 registers,
// so two workgroups fit a compute unit (the grid is slightly larger than the
// number of compute units).
constexpr int kFoldPackThreads = 512;

__global__ __launch_bounds__(kFoldPackThreads) __attribute__((amdgpu_waves_per_eu(4)))
void fold_pack_kernel(PrepJob jb) {
    fold_pack_body(jb, blockIdx.x);
}

__global__ __launch_bounds__(kFoldPackThreads) __attribute__((amdgpu_waves_per_eu(4)))
void fold_pack_batch_kernel(const PrepJob *jobs) {
    const PrepJob jb = jobs[blockIdx.y];
    fold_pack_body(jb, blockIdx.x);
}

// Complex product with one rounding per component (fused multiply-add).
__device__ __forceinline__ void cmulf(float ar, float ai, float br, float bi, float *cr,
                                      float *ci) {
    *cr = __builtin_fmaf(ar, br, -(ai * bi));
    *ci = __builtin_fmaf(ar, bi, ai * br);
}

// e^{-i v} in binary32 for a binary64 phase v, |v| < 2^50: v = q pi/2 + r, q
// the nearest integer of v 2/pi and r = v - q pi/2 with pi/2 = 2pi_hi/4 +
// 2pi_lo/4 (both quarters exact), so |r| <= pi/4 up to rounding; sin r and
// cos r from their Taylor series in binary32 (terms to r^9 and r^10: the first
// omitted term is below 2e-9 for |r| <= pi/4), then the quadrant: e^{-iv} is
// (cos r, -sin r) times (-i)^q.  q comes from adding 1.5 2^52 to v 2/pi in
// one rounding (the sum's unit in the last place is 1, so its low mantissa
// bits hold q, and q mod 4 is its two lowest).  No branch.
__device__ __forceinline__ void phasor_f32(double v, float *re, float *im) {
    constexpr double kRound = 6755399441055744.0;           // 1.5 * 2^52
    const double qs = fma(v, FEW_TWO_OVER_PI, kRound);
    const double q = qs - kRound;
    const double rd = fma(-q, 0.25 * FEW_TWO_PI_LO, fma(-q, 0.25 * FEW_TWO_PI_HI, v));
    const int qm = (int)(__builtin_bit_cast(unsigned long long, qs) & 3);   // q mod 4
    const float r = (float)rd, r2 = r * r;
    float ps = __builtin_fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
    ps = __builtin_fmaf(ps, r2, 1.0f / 120.0f);
    ps = __builtin_fmaf(ps, r2, -1.0f / 6.0f);
    const float sn = __builtin_fmaf(r * r2, ps, r);
    float pc = __builtin_fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    pc = __builtin_fmaf(pc, r2, -1.0f / 720.0f);
    pc = __builtin_fmaf(pc, r2, 1.0f / 24.0f);
    pc = __builtin_fmaf(pc, r2, -0.5f);
    const float cs = __builtin_fmaf(pc, r2, 1.0f);
    // cos v, sin v for q mod 4 = 0, 1, 2, 3: (c, s), (-s, c), (-c, -s), (s, -c)
    const bool swap = qm & 1;
    const float a = swap ? sn : cs, b = swap ? cs : sn;
    const float cv = (qm == 1 || qm == 2) ? -a : a;
    const float sv = (qm >= 2) ? -b : b;
    *re = cv;
    *im = -sv;
}

// fp16 hi/lo parts of binary32 values, hi = fp16(a), lo = fp16(a - hi) (the
// difference is exact in binary32): about 22 significant bits together.
// Here for a pair, packed as two fp16 values per 32-bit word: both hi
// parts by one packed conversion (round to nearest even), each lo part by one
// mixed-precision multiply-add a * 1 - hi that reads hi as fp16 and writes its
// fp16 result into one half of the lo word (written out because the compiler
// otherwise forms each lo in binary32 and packs the pair again).
typedef _Float16 mf_half2 __attribute__((ext_vector_type(2)));
typedef float mf_f2 __attribute__((ext_vector_type(2)));
typedef unsigned mf_u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void split_pair(float a0, float a1, unsigned &hi, unsigned &lo) {
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector((mf_f2){a0, a1}, mf_half2));
    unsigned l;
    asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]" : "=v"(l) : "v"(a0), "v"(hi));
    asm("v_fma_mixhi_f16 %0, %1, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "+v"(l)
        : "v"(a1), "v"(hi));
    lo = l;
}


// The value v of the lane whose byte address (4 x lane index) is addr.
__device__ __forceinline__ float lane_xchg(int addr, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}

// Per-wave LDS area of the per-sample values of one round (SoA, SPW samples):
// f, f^16, f^{4g} (g = 0..3), e^{-i Phi_phi}, its 8th power, the row
// harmonic z_0 e^{-2ig Phi_phi} (g = 0..3), u, and the reduced Phi_phi.
constexpr int kMfSPW = kMfNT * 16;                  // samples per wave and round
static_assert(kMfNT <= 4, "one sample tile per lane group in the epilogue");
struct MfSampleArea {
    float2 f[kMfSPW], f16[kMfSPW], c[kMfSPW][4];
    float2 e[kMfSPW], e8[kMfSPW], zg[kMfSPW][4];
    float u[kMfSPW];
    double pf[kMfSPW];
};

// One round of a workgroup: wave w takes the kMfNT * 16 samples
// base + w kMfNT 16 + s, s = 16 nt + c (tiles nt of 16, valid below e).  The
// lanes first form the per-sample values of sample s = lane + 64 k (phases,
// harmonics and their powers) into the wave's LDS area; in tile nt the four
// lane groups g = l / 16 of column c read what they need of sample 16 nt + c
// from there.  Group g holds the operand columns |n| = 16 t + 4 g + j, j < 4,
// of step t: f^{16 t + 4 g} times f^j (the same fragment serves n and -n).
// The accumulators run a Horner recurrence in u over p = 3 .. 0.  Returns this
// lane's binary64 inner-product sums (INNER) or stores h.  The LDS accesses of
// one wave complete in order, so its area needs no barrier.
template <bool INNER>
__device__ __forceinline__ double2 mf_round(const SumJob &jb, int iv, double ti, double inv_h,
                                            long long base, long long e, const float4 *lds,
                                            const float *msc, const int *mm, bool consec,
                                            MfSampleArea *sa) {
    constexpr int SPW = kMfSPW;
    constexpr int OWN = (SPW + kWave - 1) / kWave;  // samples formed per lane
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int g = lane >> 4, col = lane & 15;
    const FEW_AS4 double *pc = cptr(jb.pcoef) + (size_t)iv * 16;
    const long long wbase = base + (long long)w * SPW;
    const int m0 = mm[0], am0 = m0 < 0 ? -m0 : m0;
    // After the row combination every lane holds h of its column's sample in
    // each tile; lane group g < kMfNT then stores (or takes into the inner
    // products) the sample of tile g, so a wave issues one store per round.
    const long long jo = wbase + 16 * g + col;
    const bool own = g < kMfNT && jo < e;
    // INNER: that sample's data, requested first so that its latency passes
    // under the round's products
    // (every lane loads, at a clamped index, so that the load is not under a
    // branch, which would make the compiler wait for it at the join)
    float2 dv = make_float2(0.0f, 0.0f);
    if constexpr (INNER) dv = ((const float2 *)jb.data)[min(jo, e - 1)];
    // this lane's samples -> the wave's area
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
        const int sl = lane + kWave * k;
        if (sl >= SPW) break;
        long long j = wbase + sl;
        if (j >= e) j = e - 1;
        const double tj = dev_sample_time(jb.t_start, jb.dt, j);
        const dd x = two_sum(tj, -ti);
        const double pf = phase_raw(pc, x.hi);
        const double pr = phase_raw(pc + 8, x.hi);
        float er, ei, fr, fi;
        phasor_f32(pf, &er, &ei);
        phasor_f32(pr, &fr, &fi);
        float f2r, f2i, f4r, f4i, f8r, f8i, f12r, f12i, f16r, f16i;
        cmulf(fr, fi, fr, fi, &f2r, &f2i);
        cmulf(f2r, f2i, f2r, f2i, &f4r, &f4i);
        cmulf(f4r, f4i, f4r, f4i, &f8r, &f8i);
        cmulf(f8r, f8i, f4r, f4i, &f12r, &f12i);
        cmulf(f8r, f8i, f8r, f8i, &f16r, &f16i);
        sa->u[sl] = (float)(x.hi * inv_h);
        sa->f[sl] = make_float2(fr, fi);
        sa->f16[sl] = make_float2(f16r, f16i);
        sa->c[sl][0] = make_float2(1.0f, 0.0f);
        sa->c[sl][1] = make_float2(f4r, f4i);
        sa->c[sl][2] = make_float2(f8r, f8i);
        sa->c[sl][3] = make_float2(f12r, f12i);
        sa->e[sl] = make_float2(er, ei);
        if (consec) {
            // Rows of consecutive m (m_r = m_0 + r): every z_r is a power of
            // E = e^{-i Phi_phi}.  z_0 = E^{m_0} by binary powering (E^{-1} =
            // conj E), so each z_r carries m_r times the phase error of E, at
            // most max |m| of it.  Lane group g starts from z_0 E^{2g}.
            float e2r, e2i, e4r, e4i, e6r, e6i, e8r, e8i;
            cmulf(er, ei, er, ei, &e2r, &e2i);
            cmulf(e2r, e2i, e2r, e2i, &e4r, &e4i);
            cmulf(e4r, e4i, e2r, e2i, &e6r, &e6i);
            cmulf(e4r, e4i, e4r, e4i, &e8r, &e8i);
            float zr = 1.0f, zi = 0.0f, br = e8r, bi = e8i;
            auto take = [&](float qr, float qi) {
                float nr, ni;
                cmulf(zr, zi, qr, qi, &nr, &ni);
                zr = nr;
                zi = ni;
            };
            if (am0 & 1) take(er, ei);
            if (am0 & 2) take(e2r, e2i);
            if (am0 & 4) take(e4r, e4i);
            for (int bit = 8; bit <= am0; bit <<= 1) {
                if (am0 & bit) take(br, bi);
                float nr, ni;
                cmulf(br, bi, br, bi, &nr, &ni);
                br = nr;
                bi = ni;
            }
            if (m0 < 0) zi = -zi;
            sa->e8[sl] = make_float2(e8r, e8i);
            sa->zg[sl][0] = make_float2(zr, zi);
            float qr, qi;
            cmulf(zr, zi, e2r, e2i, &qr, &qi);
            sa->zg[sl][1] = make_float2(qr, qi);
            cmulf(zr, zi, e4r, e4i, &qr, &qi);
            sa->zg[sl][2] = make_float2(qr, qi);
            cmulf(zr, zi, e6r, e6i, &qr, &qi);
            sa->zg[sl][3] = make_float2(qr, qi);
        } else {
            sa->pf[sl] = d_reduce_2pi(pf);
        }
    }
    __builtin_amdgcn_wave_barrier();
    // operands: powers of f for every tile and step (fp16 pairs per word)
    mf_u4 bh[kMfNT][kMfT], bl[kMfNT][kMfT];
    float uu[kMfNT];
#pragma unroll
    for (int nt = 0; nt < kMfNT; ++nt) {
        const int sl = 16 * nt + col;
        uu[nt] = sa->u[sl];
        const float2 fa = sa->f[sl], fs = sa->f16[sl], c0 = sa->c[sl][g];
        const float ar = fa.x, ai = fa.y, sr = fs.x, si = fs.y;
        float cr = c0.x, ci = c0.y;
#pragma unroll
        for (int t = 0; t < kMfT; ++t) {
            float v[8];
            v[0] = cr;
            v[1] = ci;
            cmulf(v[0], v[1], ar, ai, &v[2], &v[3]);
            cmulf(v[2], v[3], ar, ai, &v[4], &v[5]);
            cmulf(v[4], v[5], ar, ai, &v[6], &v[7]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                unsigned h, l;
                split_pair(v[2 * i], v[2 * i + 1], h, l);
                bh[nt][t][i] = h;
                bl[nt][t][i] = l;
            }
            if (t + 1 < kMfT) {
                float nr, ni;
                cmulf(cr, ci, sr, si, &nr, &ni);
                cr = nr;
                ci = ni;
            }
        }
    }
    mf_float4 acc[kMfMT][kMfNT];
    // the products of power p, (mt, t) in order, each fragment read one
    // fragment ahead of its products (constant offsets from fp).  FIRST: the
    // first power, whose first product of each (mt, t = 0) starts from zero
    // (no accumulator to clear).
    auto power = [&](int p, auto first) {
        constexpr bool FIRST = decltype(first)::value;
        const float4 *fp = lds + (size_t)(3 - p) * kMfMT * kMfT * 2 * 64 + lane;
        constexpr int NF = kMfMT * kMfT;
        float4 ch = fp[0], cl = fp[64];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const int t = k % kMfT, mt = k / kMfT;
            float4 nh = ch, nl = cl;
            if (k + 1 < NF) {
                nh = fp[((k + 1) * 2) * 64];
                nl = fp[((k + 1) * 2 + 1) * 64];
            }
            // keep the next fragment's reads ahead of this fragment's products
            __builtin_amdgcn_sched_barrier(0);
            const mf_half8 ah = __builtin_bit_cast(mf_half8, ch);
            const mf_half8 al = __builtin_bit_cast(mf_half8, cl);
#pragma unroll
            for (int nt = 0; nt < kMfNT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                    al, __builtin_bit_cast(mf_half8, bh[nt][t]),
                    (FIRST && t == 0) ? mf_float4{0.0f, 0.0f, 0.0f, 0.0f} : acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < kMfNT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                    ah, __builtin_bit_cast(mf_half8, bl[nt][t]), acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < kMfNT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                    ah, __builtin_bit_cast(mf_half8, bh[nt][t]), acc[mt][nt], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            ch = nh;
            cl = nl;
        }
    };
    power(3, std::true_type{});
#pragma unroll 1
    for (int p = 2; p >= 0; --p) {
        // Horner step: every accumulator element of column nt times u
#pragma unroll
        for (int mt = 0; mt < kMfMT; ++mt)
#pragma unroll
            for (int nt = 0; nt < kMfNT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[mt][nt][i] = acc[mt][nt][i] * uu[nt];
        power(p, std::false_type{});
    }
    // Rows -> h.  The lane holds rows r = 8 mt + 2g (a0 + i b0) and r + 1
    // (a1 + i b1) of tile mt, each to be scaled by 2^{E_r} and multiplied by
    // its harmonic z_r = e^{-i m_r Phi_phi}.
    float se[kMfMT], so[kMfMT];
    int me[kMfMT], mo[kMfMT];
#pragma unroll
    for (int mt = 0; mt < kMfMT; ++mt) {
        const int r0 = 8 * mt + 2 * g;
        se[mt] = msc[r0];
        so[mt] = msc[r0 + 1];
        me[mt] = mm[r0];
        mo[mt] = mm[r0 + 1];
    }
    double dh = 0.0, hh = 0.0;
    float hro = 0.0f, hqo = 0.0f;                   // h of this lane group's sample
    // byte addresses of lanes l ^ 16 and l ^ 32 for ds_bpermute
    const int bp16 = (lane ^ 16) << 2, bp32 = (lane ^ 32) << 2;
#pragma unroll
    for (int nt = 0; nt < kMfNT; ++nt) {
        const int sl = 16 * nt + col;
        const float2 E = sa->e[sl];
        float hr, hq;
        if (consec) {
            // z_r = z_0 E^{2g} E^{8 mt} (E for the odd row): Horner in E^8
            // over the tiles of W_mt = s (a0 + i b0 + E (a1 + i b1)), s the
            // scale the two rows share
            const float2 E8 = sa->e8[sl], Z = sa->zg[sl][g];
            float qr = 0.0f, qi = 0.0f;
#pragma unroll
            for (int mt = kMfMT - 1; mt >= 0; --mt) {
                // the two rows share their scale (fold_pack_body)
                const float a0 = acc[mt][nt][0], b0 = acc[mt][nt][1];
                const float a1 = acc[mt][nt][2], b1 = acc[mt][nt][3];
                const float wr = se[mt] * __builtin_fmaf(E.x, a1, __builtin_fmaf(-E.y, b1, a0));
                const float wi = se[mt] * __builtin_fmaf(E.x, b1, __builtin_fmaf(E.y, a1, b0));
                if (mt == kMfMT - 1) {
                    qr = wr;
                    qi = wi;
                } else {
                    const float nr = __builtin_fmaf(qr, E8.x, __builtin_fmaf(-qi, E8.y, wr));
                    const float ni = __builtin_fmaf(qr, E8.y, __builtin_fmaf(qi, E8.x, wi));
                    qr = nr;
                    qi = ni;
                }
            }
            cmulf(qr, qi, Z.x, Z.y, &hr, &hq);
        } else {
            // rows of arbitrary m: one phasor per row (the odd row from the
            // even one when its m is the next integer)
            const double spf = sa->pf[sl];
            hr = 0.0f;
            hq = 0.0f;
#pragma unroll
            for (int mt = 0; mt < kMfMT; ++mt) {
                float zr, zi, yr, yi;
                phasor_f32((double)me[mt] * spf, &zr, &zi);
                if (mo[mt] == me[mt] + 1)
                    cmulf(zr, zi, E.x, E.y, &yr, &yi);
                else
                    phasor_f32((double)mo[mt] * spf, &yr, &yi);
                const float zsr = zr * se[mt], zsi = zi * se[mt];
                const float ysr = yr * so[mt], ysi = yi * so[mt];
                const float a0 = acc[mt][nt][0], b0 = acc[mt][nt][1];
                const float a1 = acc[mt][nt][2], b1 = acc[mt][nt][3];
                hr = __builtin_fmaf(zsr, a0, __builtin_fmaf(-zsi, b0, hr));
                hq = __builtin_fmaf(zsr, b0, __builtin_fmaf(zsi, a0, hq));
                hr = __builtin_fmaf(ysr, a1, __builtin_fmaf(-ysi, b1, hr));
                hq = __builtin_fmaf(ysr, b1, __builtin_fmaf(ysi, a1, hq));
            }
        }
        // the four lane groups hold the other rows of the same sample
        hr = hr + lane_xchg(bp16, hr);
        hq = hq + lane_xchg(bp16, hq);
        hr = hr + lane_xchg(bp32, hr);
        hq = hq + lane_xchg(bp32, hq);
        if (g == nt) {
            hro = hr;
            hqo = hq;
        }
    }
    if (own) {
        if constexpr (INNER) {
            const double xr = hro, xi = hqo, dr = dv.x, di = dv.y;
            dh = dr * xr + di * xi;
            hh = xr * xr + xi * xi;
        } else {
            float2 *o = (float2 *)jb.out + jo;
            *o = make_float2(hro, hqo);
        }
    }
    // the area is rewritten by the next round only after these reads
    __builtin_amdgcn_wave_barrier();
    return make_double2(dh, hh);
}

// Samples [lo, hi) of one job (matrix-core path), interval by interval; each
// interval's operand table and row scales are staged in LDS first.  Every
// lane of the workgroup runs the same loop (lo, hi uniform).  INNER: each
// lane's binary64 sums accumulate in its LDS slot iacc[threadIdx.x] (zeroed by
// the caller), which keeps them out of the registers of the product loop.
template <bool INNER>
__device__ void mf_range(const SumJob &jb, long long lo, long long hi, float4 *lds,
                         float *msc, int *mm, double2 *iacc) {
    if (lo >= hi) return;
    // the waves' sample areas follow the operand table in LDS
    MfSampleArea *sa = (MfSampleArea *)((char *)lds + kMfIntervalHalves * sizeof(_Float16)) +
                       threadIdx.x / kWave;
    __syncthreads();                                // rows of a previous job no longer read
    if ((int)threadIdx.x < kMfRows) {
        const int r = threadIdx.x;
        const FEW_AS4 int2 *mr = cptr(jb.mrows);
        mm[r] = r < jb.n_mrows ? mr[r].x : mr[jb.n_mrows - 1].x + (r - jb.n_mrows + 1);
    }
    // consecutive signed m values (padding rows continue the run)
    bool consec = true;
    {
        const FEW_AS4 int2 *mr = cptr(jb.mrows);
        for (int r = 1; r < jb.n_mrows; ++r) consec = consec && mr[r].x == mr[r - 1].x + 1;
    }
    const FEW_AS4 long long *st = cptr(jb.starts);
    int iv = 0, top = jb.K - 2;
    while (iv < top) {
        const int mid = (iv + top + 1) >> 1;
        if (st[mid] <= lo) iv = mid; else top = mid - 1;
    }
    for (; iv <= jb.K - 2 && lo < hi; ++iv) {
        const long long e = min(hi, (long long)st[iv + 1]);
        if (e <= lo) continue;
        __syncthreads();                            // previous interval no longer read
        const float4 *src = (const float4 *)((const _Float16 *)jb.mtab +
                                             (size_t)iv * kMfIntervalHalves);
        constexpr int n4 = (int)(kMfIntervalHalves * sizeof(_Float16) / 16);
        for (int v = threadIdx.x; v < n4; v += blockDim.x) lds[v] = src[v];
        if ((int)threadIdx.x < kMfRows)
            msc[threadIdx.x] = jb.mscale[(size_t)iv * kMfRows + threadIdx.x];
        __syncthreads();
        // a wave whose samples of a round all lie past the interval's end (the
        // last round of an interval) skips that round
        const long long wfirst = (long long)(threadIdx.x / kWave) * kMfSPW;
        const double ti = jb.t[iv], inv_h = 1.0 / (jb.t[iv + 1] - ti);
        for (long long base = lo; base < e; base += kMfRound) {
            if (base + wfirst >= e) continue;           // uniform per wave
            const double2 v =
                mf_round<INNER>(jb, iv, ti, inv_h, base, e, lds, msc, mm, consec, sa);
            if constexpr (INNER) {
                double2 a = iacc[threadIdx.x];
                a.x = a.x + v.x;
                a.y = a.y + v.y;
                iacc[threadIdx.x] = a;
            }
        }
        lo = e;
    }
}

// Share r of G of [0, total): workgroup b runs on XCD b mod 8 and takes share
// (b mod 8) G/8 + b/8, so each XCD works through one contiguous eighth.
__device__ __forceinline__ void mf_share(long long total, long long *lo, long long *hi) {
    const int G = gridDim.x, b = blockIdx.x;
    const int r = (G % 8 == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
    *lo = total * r / G;
    *hi = total * (r + 1) / G;
}

// Launches whose XCD split follows the weights: a multiple of 8 workgroups
// (XCD b mod 8 takes workgroup b), at most kMfBalanceWG, and weights within
// [1/4, 4].
__device__ __forceinline__ bool mf_balanced(const SumJob &jb) {
    if (jb.btime == nullptr || gridDim.x % 8 != 0 || gridDim.x > kMfBalanceWG) return false;
    for (int x = 0; x < 8; ++x)
        if (!(jb.bw[x] >= 0.25f && jb.bw[x] <= 4.0f)) return false;
    return true;
}

// Share of workgroup b with the weights wl: XCD x takes the samples
// [X_x, X_{x+1}), X_x = floor(total W_x / W_8) with W the running sum of the
// weights (X_0 = 0, X_8 = total), in equal contiguous slots of its G/8
// workgroups.
__device__ __forceinline__ void mf_share_w(const float *wl, long long total, long long *lo,
                                           long long *hi) {
    const int G = gridDim.x, b = blockIdx.x;
    const int x = b & 7, j = b >> 3, S = G >> 3;
    double cw = 0.0, all = 0.0;
    for (int i = 0; i < 8; ++i) {
        const double w = wl[i];
        if (i < x) cw += w;
        all += w;
    }
    const long long a = x == 0 ? 0 : (long long)((double)total * (cw / all));
    const long long e = x == 7 ? total : (long long)((double)total * ((cw + (double)wl[x]) / all));
    *lo = a + (e - a) * j / S;
    *hi = a + (e - a) * (j + 1) / S;
}

template <bool INNER>
__global__ __launch_bounds__(64 * kMfWaves) void sum_mfma_kernel(SumJob jb) {
    extern __shared__ float4 mf_lds[];
    __shared__ float msc[kMfRows];
    __shared__ int mm[kMfRows];
    __shared__ double2 iacc[INNER ? 64 * kMfWaves : 1];
    if constexpr (INNER) iacc[threadIdx.x] = make_double2(0.0, 0.0);
    long long lo, hi;
    // the inner-product launch keeps the equal split (its binary64 sums
    // then do not depend on the weights)
    const unsigned long long t0 = wall_clock64();
    if (!INNER && mf_balanced(jb))
        mf_share_w(jb.bw, jb.n, &lo, &hi);
    else
        mf_share(jb.n, &lo, &hi);
    mf_range<INNER>(jb, lo, hi, mf_lds, msc, mm, iacc);
    if (!INNER && jb.btime != nullptr && (int)blockIdx.x < kMfBalanceWG) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long dt = min(wall_clock64() - t0, (1ull << kMfTagShift) - 1);
            jb.btime[blockIdx.x] = ((unsigned long long)jb.btag << kMfTagShift) | dt;
        }
    }
    if constexpr (INNER) {
        __shared__ double2 red[kMfWaves];
        double2 v = wave_sum(iacc[threadIdx.x]);
        if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double2 t = red[0];
            for (int w = 1; w < kMfWaves; ++w) {
                t.x = t.x + red[w].x;
                t.y = t.y + red[w].y;
            }
            jb.partial[blockIdx.x] = t;
        }
    }
}

// Batched launch: the jobs' samples laid end to end (job j from sample_base_j),
// split into equal shares.
__global__ __launch_bounds__(64 * kMfWaves) void sum_mfma_batch_kernel(const SumJob *jobs, int n_jobs,
                                                             long long total) {
    extern __shared__ float4 mf_lds[];
    __shared__ float msc[kMfRows];
    __shared__ int mm[kMfRows];
    long long lo, hi;
    mf_share(total, &lo, &hi);
    int j = 0, top = n_jobs - 1;
    while (j < top) {
        const int mid = (j + top + 1) >> 1;
        if (*cptr(&jobs[mid].sample_base) <= lo) j = mid; else top = mid - 1;
    }
    for (; j < n_jobs; ++j) {
        const long long b0 = *cptr(&jobs[j].sample_base);
        if (b0 >= hi) break;
        const SumJob jb = load_uniform(jobs + j);
        const long long a = max(lo, b0) - b0, e = min(hi, b0 + jb.n) - b0;
        if (a < e) mf_range<false>(jb, a, e, mf_lds, msc, mm, nullptr);
    }
}

#pragma clang fp contract(on)

// ===========================================================================
// Mode selector (Sec. III D): per knot, order the modes by decreasing power
// |A|^2 (ties by increasing index), sum the powers sequentially in that order,
// and keep the shortest prefix that reaches (1 - eps) of the knot's total (at
// least the top mode).  The selection is the union over knots.  One workgroup
// of 1024 lanes per knot, in two stages.
//
// Bounded stage.  A mode j is kept iff S_j < (1 - eps) T, S_j the sequential
// sum of the powers ranked before it and T the sequential total.  Any sum of
// n non-negative binary64 values, in any order, is within (n - 1) u of the
// exact sum times the exact sum (u = 2^-53), so sums formed in another order
// (here: block reductions and LDS atomics) decide every comparison the same
// way unless they lie within a margin, taken as 8 (M + 4) u T, of the
// threshold.  The workgroup finds the last kept mode by a most-significant-
// digit radix select on the power's bits (non-negative binary64 values order
// as their bit patterns): per level, 8 bits below the candidates' common
// prefix are bucketed with the bucket power sums, and the last bucket whose
// preceding sum is below the threshold holds the last kept mode.  Each choice
// is checked against the margin on both sides; equal powers are ranked by
// index.
//
// Sorted stage, taken only when some comparison falls inside the margin (or
// the total is 0 or not finite, or the plan asks for it): bitonic sort of
// (power, index) held in registers; one lane forms the binary64 partial sums
// in sorted order (values loaded 32 at a time, so only the chain of adds is
// serial) and every threshold decision is taken on exactly those sums.
// ===========================================================================
__device__ __forceinline__ bool sel_before(double ka, int ia, double kb, int ib) {
    return ka > kb || (ka == kb && ia < ib);
}

constexpr int kSelectThreads = 1024;

// One compare-exchange of the bitonic network from the side of the element at
// position p, whose partner (position p ^ stride) holds (kq, iq).
__device__ __forceinline__ void sel_exchange(double &kv, int &iv, double kq, int iq, int p,
                                             int stride, int size) {
    const bool lower = (p & stride) == 0;
    const int low = lower ? p : (p ^ stride);
    const bool up = (low & size) == 0;             // this run sorts in "before" order
    const bool mine_first = sel_before(kv, iv, kq, iq);
    if (mine_first != (lower == up)) {
        kv = kq;
        iv = iq;
    }
}

// N = 1024 R positions (R = 1, 2 or 4); lane t holds positions t + 1024 r in
// registers.  Partners closer than a wave are exchanged by shuffles, partners
// 1024 or more apart are in the lane's own registers, the rest go through LDS.
__device__ void select_sorted(const double *amp, int M, int N, double one_minus_eps, int *keep,
                              double *sel_lds) {
    double *key = sel_lds;
    int *idx = (int *)(sel_lds + N);
    __shared__ double total;
    __shared__ int below;
    const int tid = threadIdx.x;
    const int R = N / kSelectThreads;
    const size_t k = blockIdx.x;
    double kv[4];
    int iv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = tid + kSelectThreads * r;
        if (r < R && p < M) {
            const double re = amp[(k * M + p) * 2], im = amp[(k * M + p) * 2 + 1];
            kv[r] = __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
            iv[r] = p;
        } else {
            kv[r] = -1.0;           // below every power
            iv[r] = INT_MAX;
        }
    }
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= kSelectThreads) {
                const int rs = stride / kSelectThreads;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r < R && (r & rs) == 0) {
                        const int r2 = r | rs;
                        const int p = tid + kSelectThreads * r;
                        const bool up = (p & size) == 0;
                        const bool sw = up ? sel_before(kv[r2], iv[r2], kv[r], iv[r])
                                           : sel_before(kv[r], iv[r], kv[r2], iv[r2]);
                        if (sw) {
                            const double tk = kv[r]; kv[r] = kv[r2]; kv[r2] = tk;
                            const int ti = iv[r]; iv[r] = iv[r2]; iv[r2] = ti;
                        }
                    }
                }
            } else if (stride >= kWave) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r < R) {
                        key[tid + kSelectThreads * r] = kv[r];
                        idx[tid + kSelectThreads * r] = iv[r];
                    }
                }
                __syncthreads();
                double kq[4];
                int iq[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r < R) {
                        const int q = (tid + kSelectThreads * r) ^ stride;
                        kq[r] = key[q];
                        iq[r] = idx[q];
                    }
                }
                __syncthreads();                    // reads done before the next writes
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r < R)
                        sel_exchange(kv[r], iv[r], kq[r], iq[r], tid + kSelectThreads * r,
                                     stride, size);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r < R) {
                        const double kq = __shfl_xor(kv[r], stride);
                        const int iq = __shfl_xor(iv[r], stride);
                        sel_exchange(kv[r], iv[r], kq, iq, tid + kSelectThreads * r, stride,
                                     size);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r < R) {
            key[tid + kSelectThreads * r] = kv[r];
            idx[tid + kSelectThreads * r] = iv[r];
        }
    }
    __syncthreads();
    // sequential partial sums: key[j] becomes the sum of the powers before j.
    // One lane walks the sorted powers in blocks of 32 held in its registers,
    // so the serial part is the chain of binary64 adds alone.
    if (tid == 0) {
        constexpr int B = 32;
        double run = 0.0;
        int j = 0;
        for (; j + B <= M; j += B) {
            double v[B];
#pragma unroll
            for (int q = 0; q < B; ++q) v[q] = key[j + q];
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const double before = run;
                run = __dadd_rn(run, v[q]);
                v[q] = before;
            }
#pragma unroll
            for (int q = 0; q < B; ++q) key[j + q] = v[q];
        }
        for (; j < M; ++j) {
            const double before = run;
            run = __dadd_rn(run, key[j]);
            key[j] = before;
        }
        total = run;
        below = 0;
    }
    __syncthreads();
    // kept: the modes whose preceding sum is below (1 - eps) total, a prefix
    // since the sums do not decrease; at least the top mode
    const double thr = __dmul_rn(one_minus_eps, total);
    int local = 0;
    for (int j = tid; j < M; j += kSelectThreads) local += key[j] < thr ? 1 : 0;
    if (local) atomicAdd(&below, local);
    __syncthreads();
    const int cut = below > 0 ? below : 1;
    for (int j = tid; j < cut; j += kSelectThreads) keep[idx[j]] = 1;
}

// Bounded stage of one knot (see above).  Returns false, uniformly over the
// workgroup and before writing anything, when the sorted stage must decide.
// ties: LDS scratch for up to 4096 indices.
__device__ bool select_bounded(const double *amp, int M, double one_minus_eps, int *keep,
                               int *ties) {
    constexpr int NW = kSelectThreads / kWave;
    __shared__ double bsum[256];
    __shared__ int bcnt[256];
    __shared__ double wsum[NW];
    __shared__ unsigned long long wand[NW], wor[NW];
    __shared__ double s_total, s_above;
    __shared__ unsigned long long s_pre, s_mask;
    __shared__ int s_state, s_count, s_nties, s_bad;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const size_t k = blockIdx.x;
    double pv[4];
    unsigned long long kb[4];
    bool ok[4];
    double loc = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = tid + kSelectThreads * r;
        ok[r] = p < M;
        pv[r] = 0.0;
        if (ok[r]) {
            const double re = amp[(k * M + p) * 2], im = amp[(k * M + p) * 2 + 1];
            pv[r] = __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
        }
        kb[r] = (unsigned long long)__double_as_longlong(pv[r]);
        loc += pv[r];
    }
    for (int off = kWave / 2; off > 0; off >>= 1) loc += __shfl_xor(loc, off);
    if (lane == 0) wsum[w] = loc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < NW; ++i) t += wsum[i];
        s_total = t;
        s_above = 0.0;
        s_pre = 0ull;
        s_mask = 0ull;
        s_state = 0;
        s_bad = 0;
        s_nties = 0;
    }
    __syncthreads();
    const double T = s_total;
    if (!(T > 0.0) || !(T < INFINITY)) return false;
    const double thr = __dmul_rn(one_minus_eps, T);
    const double margin = 8.0 * (double)(M + 4) * 0x1p-53 * T;
    // levels: the candidates are the modes whose masked bits equal s_pre
    for (;;) {
        const unsigned long long pre = s_pre, hm = s_mask;
        unsigned long long a = ~0ull, o = 0ull;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (ok[r] && (kb[r] & hm) == pre) {
                a &= kb[r];
                o |= kb[r];
            }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            a &= (unsigned long long)__shfl_xor((long long)a, off);
            o |= (unsigned long long)__shfl_xor((long long)o, off);
        }
        if (lane == 0) {
            wand[w] = a;
            wor[w] = o;
        }
        if (tid < 256) {
            bsum[tid] = 0.0;
            bcnt[tid] = 0;
        }
        __syncthreads();
        a = ~0ull;
        o = 0ull;
        for (int i = 0; i < NW; ++i) {
            a &= wand[i];
            o |= wor[i];
        }
        const unsigned long long diff = a ^ o;
        if (diff == 0ull) break;                    // the candidates share one power
        const int hb = 63 - __clzll((long long)diff);
        const int sh = hb >= 7 ? hb - 7 : 0;
        const unsigned long long keepm = ~0ull << (hb + 1);   // bits common to all candidates
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (ok[r] && (kb[r] & hm) == pre) {
                const int d = (int)((kb[r] >> sh) & 255ull);
                atomicAdd(&bsum[d], pv[r]);
                atomicAdd(&bcnt[d], 1);
            }
        __syncthreads();
        if (w == 0) {
            // rank order: e = 4 lane + i takes bucket 255 - e (larger powers first)
            double sv[4];
            int cv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                sv[i] = bsum[255 - (4 * lane + i)];
                cv[i] = bcnt[255 - (4 * lane + i)];
            }
            double inc = ((sv[0] + sv[1]) + sv[2]) + sv[3];
            for (int off = 1; off < kWave; off <<= 1) {
                const double y = __shfl_up(inc, off);
                if (lane >= off) inc += y;
            }
            double run = __shfl_up(inc, 1);
            run = s_above + (lane == 0 ? 0.0 : run);
            double C[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                C[i] = run;
                run += sv[i];
            }
            int best = -1;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (cv[i] > 0 && C[i] < thr) best = 4 * lane + i;
            for (int off = kWave / 2; off > 0; off >>= 1) best = max(best, __shfl_xor(best, off));
            int nxt = 0x7fffffff;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (cv[i] > 0 && 4 * lane + i > best) nxt = min(nxt, 4 * lane + i);
            for (int off = kWave / 2; off > 0; off >>= 1) nxt = min(nxt, __shfl_xor(nxt, off));
            bool bad = best < 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = 4 * lane + i;
                if (e == best && !(C[i] < thr - margin)) bad = true;
                if (e == nxt && !(C[i] >= thr + margin)) bad = true;
            }
            bad = __any(bad);
            if (bad) {
                if (lane == 0) s_state = 2;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * lane + i == best) {
                        const unsigned long long d = (unsigned long long)(255 - best);
                        s_pre = (a & keepm) | (d << sh);
                        s_mask = sh > 0 ? (~0ull << sh) : ~0ull;
                        s_above = C[i];
                        s_count = cv[i];
                        s_state = cv[i] == 1 ? 1 : (sh == 0 ? 3 : 0);
                    }
            }
        }
        __syncthreads();
        if (s_state != 0) break;
    }
    const int state = s_state;
    if (state == 2) return false;
    const unsigned long long pre = s_pre, hm = s_mask;
    if (state != 1) {
        // the candidates have one power p: the one ranked q-th by index has q p
        // before it within the candidates
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (ok[r] && (kb[r] & hm) == pre) ties[atomicAdd(&s_nties, 1)] = tid + kSelectThreads * r;
        __syncthreads();
        const int nt = s_nties;
        const double above = s_above;
        bool bad = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (!(ok[r] && (kb[r] & hm) == pre)) continue;
            const int me = tid + kSelectThreads * r;
            int q = 0;
            for (int i = 0; i < nt; ++i) q += ties[i] < me ? 1 : 0;
            const double before = fma((double)q, pv[r], above);
            if (!(before < thr - margin) && !(before >= thr + margin)) bad = true;
            ok[r] = before < thr;                   // from here: kept among the candidates
            kb[r] = pre;
        }
        if (bad) s_bad = 1;
        __syncthreads();
        if (s_bad) return false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = tid + kSelectThreads * r;
            if (p >= M) continue;
            const unsigned long long km =
                (unsigned long long)__double_as_longlong(pv[r]) & hm;
            const bool cand = km == pre;
            if ((!cand && km > pre) || (cand && ok[r])) keep[p] = 1;
        }
        return true;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (ok[r] && (kb[r] & hm) >= pre) keep[tid + kSelectThreads * r] = 1;
    return true;
}

// One workgroup per knot; `sorted` forces the sorted stage.
__global__ __launch_bounds__(kSelectThreads) void select_kernel(const double *amp, int M, int N,
                                                                double one_minus_eps,
                                                                int sorted, int *keep) {
    extern __shared__ double sel_lds[];
    if (!sorted && select_bounded(amp, M, one_minus_eps, keep, (int *)sel_lds)) return;
    __syncthreads();                                // the bounded stage's LDS reads are done
    select_sorted(amp, M, N, one_minus_eps, keep, sel_lds);
}

__global__ void zero_u32_kernel(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ===========================================================================
// Launchers.
// ===========================================================================
static inline int round_up8(long long x) { return (int)((x + 7) / 8 * 8); }

// Upload of a request's host tables: `bytes` from pinned, host-coherent memory
// (read by the GPU over the host link) into device memory, by a kernel on the
// compute queue, so a small upload does not wait on a copy engine's signal.
// 16-byte words, then the remaining bytes one per lane.
__global__ __launch_bounds__(256) void upload_kernel(const unsigned char *src, unsigned char *dst,
                                                     long long bytes) {
    const long long n16 = bytes / 16;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = tid; i < n16; i += stride)
        ((uint4 *)dst)[i] = ((const uint4 *)src)[i];
    if (tid < bytes - n16 * 16) dst[n16 * 16 + tid] = src[n16 * 16 + tid];
}

hipError_t launch_upload(const void *src, void *dst, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    const long long n16 = (long long)(bytes / 16);
    const int blocks = (int)std::max<long long>(1, std::min<long long>((n16 + 255) / 256, 128));
    hipLaunchKernelGGL(upload_kernel, dim3(blocks), dim3(256), 0, stream,
                       (const unsigned char *)src, (unsigned char *)dst, (long long)bytes);
    return hipGetLastError();
}

// Amplitude coefficients in the documented export layout: dst [K-1][M][4][2]
// from the matrix-core requests' internal [K-1][4][2M].
__global__ __launch_bounds__(256) void acoef_export_kernel(const double *src, double *dst,
                                                           long long K1, long long M) {
    const long long n = K1 * M * 8;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x) {
        const long long c = x & 1, p = (x >> 1) & 3, k = (x >> 3) % M, i = (x >> 3) / M;
        dst[x] = src[(i * 4 + p) * 2 * M + 2 * k + c];
    }
}

hipError_t launch_acoef_export(const double *src, double *dst, int K, int M,
                               hipStream_t stream) {
    const long long n = (long long)(K - 1) * M * 8;
    const int blocks = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(acoef_export_kernel, dim3(blocks), dim3(256), 0, stream, src, dst,
                       (long long)(K - 1), (long long)M);
    return hipGetLastError();
}

static inline size_t fit_lds_bytes(int K) {
    // phase workgroups: 9 arrays of K; amplitude workgroups: 5 arrays of K
    size_t n = 9 * (size_t)K;
    if (K <= kFitStageKnots)    // 4 arrays of K, the chunk values, a 2 KB slot per wave
        n = std::max(n, 4 * (size_t)K + 2 * 4 * kWave + 8 + 4 * 4 * kWave);
    return sizeof(double) * n;
}

static void fit_lds_attributes() {
    static std::once_flag once;
    std::call_once(once, [] {
        const int bytes = (int)fit_lds_bytes(kFitStageKnots);
        hipFuncSetAttribute((const void *)fit_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
        hipFuncSetAttribute((const void *)fit_batch_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    });
}

hipError_t launch_fit(const FitJob &job, const double *t_host, hipStream_t stream) {
    fit_lds_attributes();
    dim3 grid(job.n_ph + job.amp_blocks);
    FitKnots kt;
    if (job.K <= kFitStageKnots) std::memcpy(kt.t, t_host, sizeof(double) * job.K);
    hipLaunchKernelGGL(fit_kernel, grid, dim3(256), fit_lds_bytes(job.K), stream, job, kt);
    return hipGetLastError();
}

hipError_t launch_fit_batch(const FitJob *jobs_dev, int n_jobs, int max_blocks, int max_K,
                            hipStream_t stream) {
    fit_lds_attributes();
    dim3 grid(kMaxPhases + max_blocks, n_jobs);
    // jobs of up to kFitStageKnots knots stage in LDS whatever max_K is
    const size_t bytes =
        std::max(fit_lds_bytes(max_K), fit_lds_bytes(std::min(max_K, kFitStageKnots)));
    hipLaunchKernelGGL(fit_batch_kernel, grid, dim3(256), bytes, stream,
                       jobs_dev);
    return hipGetLastError();
}

hipError_t launch_prepare(const PrepJob &job, bool fp32, hipStream_t stream) {
    const dim3 grid(1 + job.fold_blocks);
    if (fp32)
        hipLaunchKernelGGL(prepare_kernel<float>, grid, dim3(256), 0, stream, job);
    else
        hipLaunchKernelGGL(prepare_kernel<double>, grid, dim3(256), 0, stream, job);
    return hipGetLastError();
}

hipError_t launch_prepare_batch(const PrepJob *jobs_dev, int n_jobs, int max_fold_blocks,
                                bool fp32, hipStream_t stream) {
    const dim3 grid(1 + max_fold_blocks, n_jobs);
    if (fp32)
        hipLaunchKernelGGL(prepare_batch_kernel<float>, grid, dim3(256), 0, stream, jobs_dev);
    else
        hipLaunchKernelGGL(prepare_batch_kernel<double>, grid, dim3(256), 0, stream, jobs_dev);
    return hipGetLastError();
}

static inline size_t sum_lds_bytes() { return sizeof(float) * 8 * (size_t)kChunkTerms; }

int sum_resident_workgroups(int n_ph) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const void *fn = n_ph == 3 ? (const void *)sum_wg_kernel<float, true, false, 3, false>
                               : (const void *)sum_wg_kernel<float, true, false, 2, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, sum_lds_bytes()) !=
        hipSuccess)
        return 0;
    return cus * per_cu;
}

hipError_t launch_sum(const SumJob &job, int slots, bool fp32, hipStream_t stream) {
    const long long parts = job.parts;
    const bool kerr = job.n_ph == 3;
    if (fp32) {
        const dim3 grid((unsigned)(parts * slots));
        if (kerr)
            hipLaunchKernelGGL((sum_wg_kernel<float, true, false, 3, false>), grid, dim3(256),
                               sum_lds_bytes(), stream, job, slots);
        else
            hipLaunchKernelGGL((sum_wg_kernel<float, true, false, 2, false>), grid, dim3(256),
                               sum_lds_bytes(), stream, job, slots);
    } else {
        const int waves_per_block = 256 / kWave;
        const long long blocks = (slots + waves_per_block - 1) / waves_per_block;
        const dim3 grid((unsigned)(parts * blocks));
        if (kerr)
            hipLaunchKernelGGL((sum_kernel<double, false, true, 3, false>), grid, dim3(256), 0,
                               stream, job, slots);
        else
            hipLaunchKernelGGL((sum_kernel<double, false, true, 2, false>), grid, dim3(256), 0,
                               stream, job, slots);
    }
    return hipGetLastError();
}

// Adds count partials in a fixed order (strided per lane, four loads in
// flight, then a tree in LDS) and writes out2 = factor * (x sum, y sum).
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void reduce_partials_kernel(const double2 *partial,
                                                                         long long count,
                                                                         double factor,
                                                                         double *out2) {
    __shared__ double2 red[kReduceThreads];
    double2 v = make_double2(0.0, 0.0);
    const long long step = blockDim.x;
    long long i = threadIdx.x;
    for (; i + 3 * step < count; i += 4 * step) {
        const double2 a = partial[i], b = partial[i + step], c = partial[i + 2 * step],
                      d = partial[i + 3 * step];
        v.x = v.x + a.x; v.y = v.y + a.y;
        v.x = v.x + b.x; v.y = v.y + b.y;
        v.x = v.x + c.x; v.y = v.y + c.y;
        v.x = v.x + d.x; v.y = v.y + d.y;
    }
    for (; i < count; i += step) {
        v.x = v.x + partial[i].x;
        v.y = v.y + partial[i].y;
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[threadIdx.x].x = red[threadIdx.x].x + red[threadIdx.x + off].x;
            red[threadIdx.x].y = red[threadIdx.x].y + red[threadIdx.x + off].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = factor * red[0].x;
        out2[1] = factor * red[0].y;
    }
}

// Partial sums of the allocation-free inner product: a file-scope device
// array, one copy per GPU, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (in host code the name is a host-side
// stand-in); it uses the device address hipGetSymbolAddress returns, looked up
// once per device by noalloc_scratch().
static __device__ __align__(256) double2 scratch[kNoAllocSlots];

hipError_t noalloc_scratch(int device, double2 **out) {
    static std::mutex mu;
    static double2 *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double2 *)p;
    }
    *out = addr[device];
    return hipSuccess;
}

long long inner_slots(int parts, int slots, bool fp32) {
    if (fp32) return (long long)parts * slots;
    const int waves_per_block = 256 / kWave;
    return (long long)parts * ((slots + waves_per_block - 1) / waves_per_block) * waves_per_block;
}

hipError_t launch_sum_inner(const SumJob &job, int slots, bool fp32, double two_dt,
                            double *out2, hipStream_t stream) {
    const long long parts = job.parts;
    const bool kerr = job.n_ph == 3;
    if (fp32) {
        const dim3 grid((unsigned)(parts * slots));
        if (kerr)
            hipLaunchKernelGGL((sum_wg_kernel<float, true, false, 3, true>), grid, dim3(256),
                               sum_lds_bytes(), stream, job, slots);
        else
            hipLaunchKernelGGL((sum_wg_kernel<float, true, false, 2, true>), grid, dim3(256),
                               sum_lds_bytes(), stream, job, slots);
    } else {
        const int waves_per_block = 256 / kWave;
        const long long blocks = (slots + waves_per_block - 1) / waves_per_block;
        const dim3 grid((unsigned)(parts * blocks));
        if (kerr)
            hipLaunchKernelGGL((sum_kernel<double, false, true, 3, true>), grid, dim3(256), 0,
                               stream, job, slots);
        else
            hipLaunchKernelGGL((sum_kernel<double, false, true, 2, true>), grid, dim3(256), 0,
                               stream, job, slots);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kReduceThreads), 0, stream,
                       job.partial, inner_slots(job.parts, slots, fp32), two_dt, out2);
    return hipGetLastError();
}

// Workgroup 0 and the (interval, row tile) workgroups of a K-knot request,
// the intervals in groups of 8 (fold_pack_body).
static int fold_pack_blocks(int K) { return 1 + 8 * kMfMT * ((K - 1 + 7) / 8); }

hipError_t launch_fold_pack(const PrepJob &job, hipStream_t stream) {
    hipLaunchKernelGGL(fold_pack_kernel, dim3(fold_pack_blocks(job.K)), dim3(kFoldPackThreads), 0,
                       stream, job);
    return hipGetLastError();
}

hipError_t launch_fold_pack_batch(const PrepJob *jobs_dev, int n_jobs, int max_K,
                                  hipStream_t stream) {
    hipLaunchKernelGGL(fold_pack_batch_kernel, dim3(fold_pack_blocks(max_K), n_jobs),
                       dim3(kFoldPackThreads), 0, stream, jobs_dev);
    return hipGetLastError();
}

static constexpr size_t mf_lds_bytes() {
    return kMfIntervalHalves * sizeof(_Float16) + kMfWaves * sizeof(MfSampleArea);
}

// One workgroup per compute unit (the operand table takes most of the LDS).
int mfma_workgroups() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    static std::once_flag once;
    std::call_once(once, [] {
        hipFuncSetAttribute((const void *)sum_mfma_kernel<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)mf_lds_bytes());
        hipFuncSetAttribute((const void *)sum_mfma_kernel<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)mf_lds_bytes());
        hipFuncSetAttribute((const void *)sum_mfma_batch_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)mf_lds_bytes());
    });
    return cus;
}

hipError_t launch_sum_mfma(const SumJob &job, int n_wg, hipStream_t stream) {
    hipLaunchKernelGGL(sum_mfma_kernel<false>, dim3(n_wg), dim3(64 * kMfWaves), mf_lds_bytes(),
                       stream, job);
    return hipGetLastError();
}

hipError_t launch_sum_mfma_inner(const SumJob &job, int n_wg, double two_dt, double *out2,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(sum_mfma_kernel<true>, dim3(n_wg), dim3(64 * kMfWaves), mf_lds_bytes(),
                       stream, job);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kReduceThreads), 0, stream,
                       job.partial, (long long)n_wg, two_dt, out2);
    return hipGetLastError();
}

hipError_t launch_sum_mfma_batch(const SumJob *jobs_dev, int n_jobs, long long total, int n_wg,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(sum_mfma_batch_kernel, dim3(n_wg), dim3(64 * kMfWaves), mf_lds_bytes(),
                       stream, jobs_dev, n_jobs, total);
    return hipGetLastError();
}

hipError_t launch_sum_batch(const SumJob *jobs_dev, int n_jobs, int total_slots, bool fp32,
                            bool persistent, unsigned *counter_dev, hipStream_t stream) {
    const int waves_per_block = 256 / kWave;
    if (!persistent) {
        if (fp32)
            hipLaunchKernelGGL((sum_wg_batch_kernel<float, true, false>),
                               dim3(round_up8(total_slots)), dim3(256), sum_lds_bytes(), stream,
                               jobs_dev, n_jobs, total_slots);
        else
            hipLaunchKernelGGL((sum_batch_kernel<double, false, true>),
                               dim3(round_up8((total_slots + waves_per_block - 1) / waves_per_block)),
                               dim3(256), 0, stream, jobs_dev, n_jobs, total_slots);
        return hipGetLastError();
    }
    // one resident grid: 256 CUs x 4 workgroups of 4 waves
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, stream, counter_dev, 1);
    if (fp32) {
        int blocks = 256 * 4;
        if (blocks > total_slots) blocks = total_slots > 0 ? total_slots : 1;
        hipLaunchKernelGGL((sum_wg_persistent_kernel<float, true, false>),
                           dim3(blocks), dim3(256), sum_lds_bytes(), stream, jobs_dev, n_jobs,
                           total_slots, counter_dev);
    } else {
        int blocks = 256 * 8;
        const int needed = (total_slots + waves_per_block - 1) / waves_per_block;
        if (blocks > needed) blocks = needed > 0 ? needed : 1;
        hipLaunchKernelGGL((sum_persistent_kernel<double, false, true>),
                           dim3(blocks), dim3(256), 0, stream, jobs_dev, n_jobs, total_slots,
                           counter_dev);
    }
    return hipGetLastError();
}

hipError_t launch_select(const double *amp, int K, int M, double eps, bool sorted, int *keep,
                         hipStream_t stream) {
    int N = kSelectThreads;                 // 1024, 2048 or 4096 sort positions
    while (N < M) N <<= 1;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((M + 255) / 256), dim3(256), 0, stream,
                       (unsigned *)keep, M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = (sizeof(double) + sizeof(int)) * (size_t)N;
    hipLaunchKernelGGL(select_kernel, dim3(K), dim3(kSelectThreads), lds, stream, amp, M, N,
                       1.0 - eps, sorted ? 1 : 0, keep);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned *p, int n, hipStream_t stream) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace few
