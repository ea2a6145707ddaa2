// Internal declarations shared by the host runtime (few_api.cpp,
// host_core.cpp) and the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace few {

constexpr int kMaxKnots = 1024;       // phase-solve LDS: eight binary64 arrays of this length (64 KiB)
constexpr int kMaxL = 30;             // Wigner-d sum stays well conditioned in binary64
constexpr int kMaxAbsN = 1000;
constexpr int kMaxAbsK = 30;          // polar index of generic-Kerr modes
constexpr int kWave = 64;
constexpr int kMaxGap = 4;            // zero terms filled inside one segment
#ifndef FEW_SEG_UNROLL
#define FEW_SEG_UNROLL 2
#endif
#ifndef FEW_CHUNK_TERMS
#define FEW_CHUNK_TERMS 1024
#endif
// Amplitude series per fit workgroup (lane = series; the four waves take a
// quarter of the rows each, or wave 0 all of them on larger grids).
constexpr int kFitSeriesPerBlock = 64;
// Grids of at most this many knots keep each lane's knot values in registers
// (a quarter of the rows per wave) and factor the grid with one wave's scan;
// larger grids stream knot values with one lane per series.
constexpr int kFitStageKnots = 128;
constexpr int kChunkTerms = FEW_CHUNK_TERMS;   // terms staged in LDS at once (binary32: 32 B each)

// Samples per lane in one wave tile of the summation kernel.
#ifndef FEW_SL_F32
#define FEW_SL_F32 4
#endif
#ifndef FEW_SL_F64
#define FEW_SL_F64 2
#endif
constexpr int kSamplesPerLaneF32 = FEW_SL_F32;
constexpr int kSamplesPerLaneF64 = FEW_SL_F64;

// Samples per tile: a workgroup of 4 waves (binary32) or one wave (binary64).
inline int tile_samples(bool fp32) {
    return fp32 ? 4 * kWave * kSamplesPerLaneF32 : kWave * kSamplesPerLaneF64;
}

// Binary32: the last samples of a single-request launch are cut into short
// tiles (half the samples per lane) so the end of the launch drains evenly.
// The short-tile region holds FEW_SHORT_QUARTERS / 4 of one round of long tiles
// over the resident workgroups.  (Binary64 tiles read their coefficients with
// scalar loads, which short tiles amortise poorly: long tiles only.)
#ifndef FEW_SL_SHORT
#define FEW_SL_SHORT 2
#endif
#ifndef FEW_SHORT_QUARTERS
#define FEW_SHORT_QUARTERS 2
#endif
constexpr int kSamplesPerLaneShort = FEW_SL_SHORT;
inline int short_tile_samples(bool fp32) {
    return fp32 ? 4 * kWave * kSamplesPerLaneShort : kWave * kSamplesPerLaneF64;
}

// Binary32 sums run over four term groups (consecutive segments with about a
// quarter of the terms each): every sample's compensated sum restarts, and its
// harmonic seed is recomputed, at each group's first segment, and the four
// group values are added in group order.  A term-split tile uses that: its four
// waves take the same 64 x kSamplesPerLaneF32 samples, one group each, staging
// their group kSplitTerms terms at a time in their own quarter of the LDS
// buffer.  Requests whose segments all fit a quarter cut their short tiles this
// way (the end of a launch then drains in pieces a quarter as long); others
// keep the 2-sample short tiles.  Either way a sample gets the same rounded
// operations.
constexpr int kTermGroups = 4;
constexpr int kSplitTerms = FEW_CHUNK_TERMS / kTermGroups;
// Requests with fewer folded terms form one group (reseeding at group starts
// costs a few sincos per sample and tile, which short sums do not repay) and
// keep the 2-sample short tiles.
constexpr int kGroupMinTerms = 1024;
inline int split_tile_samples() { return kWave * kSamplesPerLaneF32; }

// Matrix-core summation (binary32 output).  Per knot interval the folded sum
// is a contraction: with rows = the distinct signed m values (a complex row
// each, as a real re/im pair) and columns n,
//   h = sum_m e^{-i m Phi_phi} sum_p u^p sum_n C^p_{m,n} f^n,
// f = e^{-i Phi_r}.  For each p the sum over n is the product of the
// coefficient matrix [rows x (n, re/im)] with the matrix of powers f^n over
// the samples, run on v_mfma_f32_16x16x32_f16 with both operands split into
// fp16 hi + lo parts (hi*hi + hi*lo + lo*hi, about 22 significant bits) and
// fp32 accumulation; the sum over p is a Horner recurrence in u on the
// accumulators.  Only the powers f^a, a = |n| >= 0, are formed: a column of
// n < 0 multiplies conj(f^|n|), and the conjugation lives in the coefficient
// matrix, so the terms n and -n meet the same operand fragment and their
// coefficient rows are added into one (the product is linear in them).
// Fixed shape: kMfMT tiles of 16 matrix rows (8 signed m each), kMfT steps of
// 32 columns (16 values of |n| each; |n| < 16 kMfT), kMfNT tiles of 16
// samples per wave, kMfWaves waves per workgroup.  A request takes this
// path when its term layout fits the shape and is long enough to repay it.
#ifndef FEW_MF_NT
#define FEW_MF_NT 3
#endif
#ifndef FEW_MF_WAVES
#define FEW_MF_WAVES 12
#endif
constexpr int kMfMT = 3;
constexpr int kMfT = 2;
constexpr int kMfNT = FEW_MF_NT;
constexpr int kMfWaves = FEW_MF_WAVES;
constexpr int kMfRows = 8 * kMfMT;          // signed m values per request
constexpr int kMfA = 16 * kMfT;             // |n| < kMfA
constexpr int kMfRound = kMfWaves * kMfNT * 16;   // samples per workgroup round
// fp16 values of one interval: [p 4][mt][t][hi, lo][lane 64][8]
constexpr size_t kMfIntervalHalves = (size_t)4 * kMfMT * kMfT * 2 * 64 * 8;
constexpr int kMfMinTerms = 480;            // below this the vector kernel is cheaper

// ---------------------------------------------------------------------------
// Device-side job descriptors.  Pointers are device addresses in the plan
// arena (or caller memory for inputs/outputs).
// ---------------------------------------------------------------------------

// Spline stage for one request.
struct FitJob {
    const double *t;        // [K] knot times
    const double *phi_phi;  // [K]
    const double *phi_r;    // [K]
    const double *phi_theta;  // [K] (generic Kerr) or null
    const double *amp;      // [K][M][2]
    double *pcoef;          // [K-1][n_ph][4][2] double-double phase cubics
    double *acoef;          // amplitude cubics: [K-1][M][4][2], or [K-1][4][2M] if pmajor
    int acoef_pmajor;       // 1: coefficient p of series q = 2k + re/im at [i][p][q]
                            // (matrix-core requests: read by fold_pack), 0: mode-major
    int K, M;
    int n_ph;               // phases: Phi_phi, Phi_r (, Phi_theta)
    int amp_blocks;         // blocks covering the 2M amplitude series (after n_ph phase blocks)
    // Upload carried by this launch (single-request fits): up_bytes bytes
    // from the pinned, host-coherent staging slot up_src to the request's
    // arena block up_dst, copied by the amplitude workgroups' waves that do
    // not sweep; t then points at the knots in the staging slot.  0: none.
    const uint4 *up_src;
    uint4 *up_dst;
    long long up_bytes;
};

constexpr int kMaxPhases = 3;

// Knot times of a single-request fit of at most kFitStageKnots knots, passed
// by value as a launch argument.
struct FitKnots {
    double t[kFitStageKnots];
};

// Fold + interval bookkeeping for one request.
struct PrepJob {
    const double *t;
    const double *acoef;
    const int *term_ptr;    // [n_terms + 1]
    const int2 *term_src;   // [n_src]: (mode, l | m << 8 | mirror << 16)
    double2 *ybuf;          // [n_src] harmonic weight of each contributor
    void *table;            // [K-1][n_terms][8] binary32 or binary64, terms in reverse order
    long long *starts;      // [K]
    int *tile_pref;         // [parts][K]: tiles before each interval, per part
    double theta, phi, scale, t_start, dt;
    double scale_im;        // imaginary part of a complex overall factor (0: real scale)
    long long n;
    long long short_len;    // samples at the end of each part cut into short tiles
    int parts;              // contiguous sample parts (one per XCD) or 1
    int K, M, n_terms, n_src;
    int tile;               // samples per tile
    int short_tile;         // samples per short tile
    int fold_terms;         // consecutive terms folded by one workgroup
    int fold_blocks;        // term groups of the fold
    // matrix-core path: the fold writes the fp16 operand table and the
    // per-(interval, row) scales
    const int4 *segs;       // [n_segs]
    const int2 *mrows;      // [n_mrows + 1]: (m, first segment) per row, sentinel (0, n_segs)
    void *mtab;             // [K-1][kMfIntervalHalves] fp16
    float *mscale;          // [K-1][kMfRows]: 2^E with row values scaled by 2^-E
    int n_mrows, n_min, n_segs;
    int l_max;              // largest listed l
};

// Split of the matrix-core summation between the eight XCDs: the XCDs of
// one device run at different clocks under load, so a store launch may give
// XCD x a share of the samples proportional to a weight w[x], and each of its
// workgroups then reports its time (with the launch's tag) in pinned host
// memory, from which the host forms the weights of later launches.  Only
// performance depends on it: any weights give a split that covers every
// sample once.
constexpr int kMfBalanceWG = 256;       // workgroups a report array holds
constexpr int kMfTagShift = 40;         // report word: tag << 40 | s_memrealtime ticks

// Summation stage for one request.
struct SumJob {
    const double *t;
    const double *pcoef;    // [K-1][n_ph][4][2]
    const void *table;
    const int4 *segs;       // [n_segs]: (m + 256 k, n_lo, length, first term)
    const int *chunks;      // [n_chunks + 1]: first segment of each LDS chunk
    const long long *starts;
    const int *tile_pref;
    void *out;              // [n] complex output (store launches)
    const void *data;       // [n] complex data d (inner-product launches)
    double2 *partial;       // per tile slot: (sum Re(conj(d) h), sum |h|^2)
    double t_start, dt;
    long long n;
    long long short_len;    // samples at the end of each part cut into short tiles
    int parts;              // contiguous sample parts (one per XCD) or 1
    int K, n_terms, n_segs, n_chunks;
    int n_ph;               // phases in pcoef (3: generic Kerr, Phi_theta last)
    int wave_base;          // first global tile slot of this job (batched launch)
    int grp[kTermGroups - 1];   // first segment of term groups 1..3 (binary32)
    int split;              // short tiles are term-split tiles
    // matrix-core path
    const void *mtab;       // [K-1][kMfIntervalHalves] fp16 operand table
    const float *mscale;    // [K-1][kMfRows]
    const int2 *mrows;      // [n_mrows + 1]
    int n_mrows, n_min;
    long long sample_base;  // first sample of this job in a batched launch's range
    // matrix-core store launches: XCD split weights (all 0: equal split), and
    // where each workgroup reports (tag << kMfTagShift | its time), or nullptr
    float bw[8];
    unsigned long long *btime;
    unsigned btag;
};

// Launchers (kernels.hip).  All enqueue on `stream` and return the HIP status.
// Binary32 summation workgroups resident at once on the current device, for
// the two-phase (Schwarzschild) or three-phase (generic Kerr) kernel.
int sum_resident_workgroups(int n_ph);
hipError_t launch_upload(const void *src, void *dst, size_t bytes, hipStream_t stream);
// acoef [K-1][4][2M] -> dst [K-1][M][4][2] (the few_spline_coefs layout)
hipError_t launch_acoef_export(const double *src, double *dst, int K, int M,
                               hipStream_t stream);
// t_host: the K knot times in host memory (copied into the launch's arguments
// when K <= kFitStageKnots).
hipError_t launch_fit(const FitJob &job, const double *t_host, hipStream_t stream);
hipError_t launch_fit_batch(const FitJob *jobs_dev, int n_jobs, int max_blocks, int max_K,
                            hipStream_t stream);
hipError_t launch_prepare(const PrepJob &job, bool fp32, hipStream_t stream);
hipError_t launch_prepare_batch(const PrepJob *jobs_dev, int n_jobs, int max_fold_blocks,
                                bool fp32, hipStream_t stream);
hipError_t launch_sum(const SumJob &job, int slots, bool fp32, hipStream_t stream);
// Inner-product variant of launch_sum: instead of storing h, every tile slot
// writes its partial sums to job.partial (inner_slots(...) entries), then one
// workgroup adds them in a fixed order into out2 = 2 dt (<d|h> sum, <h|h> sum).
hipError_t launch_sum_inner(const SumJob &job, int slots, bool fp32, double two_dt,
                            double *out2, hipStream_t stream);
long long inner_slots(int parts, int slots, bool fp32);
// Allocation-free inner product: partial sums go to a static device array of
// kNoAllocSlots entries (2 MiB, one copy per GPU).  noalloc_scratch() returns
// its device address on `device`, which must be the current device; it looks
// the address up (hipGetSymbolAddress) on the first call per device.
constexpr long long kNoAllocSlots = 131072;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, double2 **out);
hipError_t launch_sum_batch(const SumJob *jobs_dev, int n_jobs, int total_wave_slots,
                            bool fp32, bool persistent, unsigned *counter_dev,
                            hipStream_t stream);
hipError_t launch_zero_u32(unsigned *p, int n, hipStream_t stream);
// Matrix-core path: the prepare step (interval starts, fold and the fp16
// operand table, one request or n_jobs of them with max_K knots at most), and
// the summation (every workgroup takes an equal contiguous share of the
// samples; n_wg workgroups; with INNER each writes its partial sums to
// job.partial[b] and one more launch adds them into out2 = two_dt * sums).
hipError_t launch_fold_pack(const PrepJob &job, hipStream_t stream);
hipError_t launch_fold_pack_batch(const PrepJob *jobs_dev, int n_jobs, int max_K,
                                  hipStream_t stream);
int mfma_workgroups();
hipError_t launch_sum_mfma(const SumJob &job, int n_wg, hipStream_t stream);
hipError_t launch_sum_mfma_inner(const SumJob &job, int n_wg, double two_dt, double *out2,
                                 hipStream_t stream);
hipError_t launch_sum_mfma_batch(const SumJob *jobs_dev, int n_jobs, long long total,
                                 int n_wg, hipStream_t stream);
hipError_t launch_select(const double *amp, int K, int M, double eps, bool sorted, int *keep,
                         hipStream_t stream);
constexpr int kMaxSelectModes = 4096;   // LDS: (binary64 key + int index) per padded mode

// ---------------------------------------------------------------------------
// Host core (host_core.cpp): no device work.
// ---------------------------------------------------------------------------
struct TermLayout {
    int n_segs = 0, n_terms = 0, n_src = 0, n_chunks = 0;
    int *segs = nullptr;       // 4 * n_segs
    int *term_ptr = nullptr;   // n_terms + 1
    int *term_src = nullptr;   // 2 * n_src
    int *chunks = nullptr;     // n_chunks + 1: first segment of each chunk of <= kChunkTerms terms
    int grp[kTermGroups - 1] = {0, 0, 0};   // first segment of term groups 1..3
    int max_seg_terms = 0;     // longest segment
    // matrix-core path: distinct signed m values (rows) and the n range
    int n_mrows = 0, n_min = 0, n_max = 0, l_max = 0;
    int *mrows = nullptr;      // 2 * (n_mrows + 1): (m, first segment), sentinel (0, n_segs)
    bool mfma = false;         // layout fits the matrix-core shape (Schwarzschild terms)
};

// Build the folded term layout; returns 0 or a few_status error code.
int build_term_layout(int M, const int32_t *modes, int width, int max_gap, TermLayout *out);
void free_term_layout(TermLayout *t);

// Detector frame (see few_host_frame): source viewing angles and the complex
// factor -e^{-2 i psi}; returns 0 or FEW_E_ARG.
int detector_frame(double theta_s, double phi_s, double theta_k, double phi_k,
                   double *theta_src, double *phi_src, double *rot_re, double *rot_im);

// starts[i] for i in [0, K): see few_host_interval_starts.
void interval_starts(int K, const double *t, double t_start, double dt, long long n,
                     long long *starts);

// Upper bound of the wave tiles a request needs.
inline long long tile_upper_bound(long long n, int K, int tile) {
    return (n + tile - 1) / tile + (K - 1);
}

// Single-request launches split the samples into kParts contiguous parts,
// [floor(p n / kParts), floor((p + 1) n / kParts)), one per XCD, so each XCD
// reads the coefficient tables of its own intervals only.
constexpr int kParts = 8;

__host__ __device__ inline long long part_begin(long long n, int parts, int p) {
    return n * p / parts;
}

// Tiles of one part (at most ceil(n / parts) samples) whose last short_len
// samples use short tiles: each interval adds at most one partial tile of
// each kind.
inline long long part_tile_bound(long long n, int parts, long long short_len, int K, int tile,
                                 int short_tile) {
    const long long len = (n + parts - 1) / parts;
    if (short_len <= 0) return tile_upper_bound(len, K, tile);
    const long long s = short_len < len ? short_len : len;
    return (len + tile - 1) / tile + (s + short_tile - 1) / short_tile + 2LL * (K - 1);
}

// Arena layout of one request's resident state.
struct ReqLayout {
    size_t off_t, off_segs, off_term_ptr, off_term_src, off_chunks, off_mrows,
        upload_end;   // host-staged
    size_t off_pcoef, off_acoef, off_ybuf, off_table, off_starts, off_tile_pref, off_mtab,
        off_mscale, total;
    size_t dev_begin;       // first device-produced offset (== off_pcoef)
};
// mfma: binary32 request on the matrix-core path (binary64 fold table, fp16
// operand table and row scales; n_mrows rows)
ReqLayout request_layout(bool fp32, int K, int M, int n_segs, int n_terms, int n_src,
                         int n_chunks, int n_ph, bool mfma = false, int n_mrows = 0);

// Binary64 sample time exactly as written: t_start + j * dt, no contraction.
double sample_time(double t_start, double dt, long long j);

}  // namespace few
