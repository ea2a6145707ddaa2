// Host-side bookkeeping of libfew: the folded term layout, the first sample of
// each knot interval, and the arena layout of one request.  No device work;
// the exported few_host_* helpers are usable on machines without a GPU.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/few.h"
#include "few_internal.h"

#pragma clang fp contract(off)

namespace few {

double sample_time(double t_start, double dt, long long j) {
    volatile double prod = (double)j * dt;
    return t_start + prod;
}

void interval_starts(int K, const double *t, double t_start, double dt, long long n,
                     long long *starts) {
    starts[0] = 0;
    for (int i = 1; i < K - 1; ++i) {
        double est = std::ceil((t[i] - t_start) / dt);
        long long j;
        if (!(est > 0.0)) j = 0;
        else if (est >= (double)n) j = n;
        else j = (long long)est;
        while (j > 0 && sample_time(t_start, dt, j - 1) >= t[i]) --j;
        while (j < n && sample_time(t_start, dt, j) < t[i]) ++j;
        starts[i] = j;
    }
    starts[K - 1] = n;
}

namespace {
// One signed term contribution: (m, kp, n) of the signed mode, the listed mode
// index and its (l, m), and whether it is the mirror of a listed m > 0 mode.
struct Entry {
    int m, kp, n, k, l, mode_m, mirror;
};
}  // namespace

void free_term_layout(TermLayout *t) {
    std::free(t->segs);
    std::free(t->term_ptr);
    std::free(t->term_src);
    std::free(t->chunks);
    std::free(t->mrows);
    *t = TermLayout{};
}

// Eq. (9): every listed mode (l, m >= 0, k, n) contributes A Y_lm to the
// signed term (m, k, n); for m > 0 its mirror contributes
// (-1)^{l+k} conj(A) Y_{l,-m} to the term (-m, -k, -n).  For fixed viewing
// angles the l-sum then folds into one complex cubic per signed (m, k, n).
// width 3: modes (l, m, n) with k = 0 (Schwarzschild); width 4: (l, m, k, n).
int build_term_layout(int M, const int32_t *modes, int width, int max_gap, TermLayout *out) {
    *out = TermLayout{};
    if (M < 1 || !modes || (width != 3 && width != 4)) return FEW_E_ARG;
    // order by (m, kp, n, listed index, mirror): entries are generated in
    // (index, mirror) order, then a stable radix sort on the 23-bit key
    // (m, kp, n) keeps that order inside each term
    // (scratch vectors are reused per thread: fresh large blocks would be
    // mapped and faulted in on every call)
    thread_local std::vector<Entry> gen, e;
    thread_local std::vector<uint32_t> key, idx, tmp;
    thread_local std::vector<int> segs, term_ptr, src, chunks;
    gen.clear();
    key.clear();
    auto pack = [](int m, int kp, int n) {
        return (uint32_t)((m + kMaxL) << 17 | (kp + kMaxAbsK) << 11 | (n + kMaxAbsN));
    };
    for (int k = 0; k < M; ++k) {
        const int32_t *md = modes + (size_t)width * k;
        int l = md[0], m = md[1], kp = width == 4 ? md[2] : 0, n = md[width - 1];
        if (l < 2 || l > kMaxL || m < 0 || m > l || n < -kMaxAbsN || n > kMaxAbsN ||
            kp < -kMaxAbsK || kp > kMaxAbsK)
            return FEW_E_MODES;
        gen.push_back({m, kp, n, k, l, m, 0});
        key.push_back(pack(m, kp, n));
        if (m > 0) {
            gen.push_back({-m, -kp, -n, k, l, m, 1});
            key.push_back(pack(-m, -kp, -n));
        }
    }
    const size_t ne = gen.size();
    idx.resize(ne);
    tmp.resize(ne);
    for (size_t q = 0; q < ne; ++q) idx[q] = (uint32_t)q;
    for (int pass = 0; pass < 3; ++pass) {
        const int shift = 8 * pass;
        uint32_t count[257] = {0};
        for (size_t q = 0; q < ne; ++q) ++count[((key[idx[q]] >> shift) & 255) + 1];
        for (int b = 0; b < 256; ++b) count[b + 1] += count[b];
        for (size_t q = 0; q < ne; ++q) tmp[count[(key[idx[q]] >> shift) & 255]++] = idx[q];
        idx.swap(tmp);
    }
    e.resize(ne);
    for (size_t q = 0; q < ne; ++q) e[q] = gen[idx[q]];

    // segments over distinct (m, kp, n) with contiguous n: segs
    // (m + 256 kp, n_lo, len, first), term_ptr (first contributor of each
    // term), src (contributors: listed index, l | m << 8 | mirror << 16 |
    // (kp + 64) << 17)
    segs.clear();
    term_ptr.clear();
    src.clear();
    size_t p = 0;
    int term = 0;
    while (p < e.size()) {
        int m = e[p].m, kp = e[p].kp;
        int n_lo = e[p].n, n_prev = e[p].n;
        int first = term;
        // extend while the next distinct n of this (m, kp) is within the gap
        size_t q = p;
        while (q < e.size() && e[q].m == m && e[q].kp == kp) {
            int n = e[q].n;
            if (n > n_prev + 1 + max_gap && q != p) break;
            // no segment longer than one LDS chunk
            if (q != p && (term - first) + (n - n_prev) > kChunkTerms) break;
            // fill zero terms between n_prev and n
            for (int z = n_prev + 1; z < n; ++z) {
                term_ptr.push_back((int)src.size() / 2);
                ++term;
            }
            term_ptr.push_back((int)src.size() / 2);
            ++term;
            while (q < e.size() && e[q].m == m && e[q].kp == kp && e[q].n == n) {
                src.push_back(e[q].k);
                src.push_back(e[q].l | (e[q].mode_m << 8) | (e[q].mirror << 16) |
                              ((e[q].kp + 64) << 17));
                ++q;
            }
            n_prev = n;
        }
        segs.push_back(m + 256 * kp);
        segs.push_back(n_lo);
        segs.push_back(term - first);
        segs.push_back(first);
        p = q;
    }
    term_ptr.push_back((int)src.size() / 2);
    // chunks: runs of whole segments with at most kChunkTerms terms
    chunks.clear();
    chunks.push_back(0);
    const int n_seg = (int)segs.size() / 4;
    int run = 0;
    for (int g = 0; g < n_seg; ++g) {
        const int len = segs[4 * g + 2];
        if (run > 0 && run + len > kChunkTerms) {
            chunks.push_back(g);
            run = 0;
        }
        run += len;
    }
    chunks.push_back(n_seg);
    // term groups: group q starts at the segment boundary nearest to q / 4 of
    // the terms (boundaries non-decreasing; a group may be empty); one group
    // below kGroupMinTerms terms
    {
        int g = 0, start = 0;
        for (int q = 1; q < kTermGroups; ++q) {
            if (term < kGroupMinTerms) {
                out->grp[q - 1] = n_seg;
                continue;
            }
            const double target = (double)term * q / kTermGroups;
            while (g < n_seg && start + segs[4 * g + 2] <= target) start += segs[4 * g++ + 2];
            if (g < n_seg && target - start > start + segs[4 * g + 2] - target)
                start += segs[4 * g++ + 2];
            out->grp[q - 1] = g;
        }
        out->max_seg_terms = 0;
        for (int k = 0; k < n_seg; ++k) out->max_seg_terms = std::max(out->max_seg_terms, segs[4 * k + 2]);
    }
    // matrix-core rows: the distinct signed m values (segments are in m order)
    // and the n range over all segments
    {
        std::vector<int> mr;
        int n_min = INT32_MAX, n_max = INT32_MIN;
        for (int g = 0; g < n_seg; ++g) {
            const int m = segs[4 * g];
            if (g == 0 || m != segs[4 * (g - 1)]) {
                mr.push_back(m);
                mr.push_back(g);
            }
            n_min = std::min(n_min, segs[4 * g + 1]);
            n_max = std::max(n_max, segs[4 * g + 1] + segs[4 * g + 2] - 1);
        }
        mr.push_back(0);
        mr.push_back(n_seg);
        out->n_mrows = (int)mr.size() / 2 - 1;
        int lm = 0;
        for (int k = 0; k < M; ++k) lm = std::max(lm, (int)modes[(size_t)width * k]);
        out->l_max = lm;
        out->n_min = n_min;
        out->n_max = n_max;
        out->mfma = width == 3 && n_min > -kMfA && n_max < kMfA && out->n_mrows <= kMfRows &&
                    term >= kMfMinTerms;
        out->mrows = (int *)std::malloc(sizeof(int) * mr.size());
        if (!out->mrows) {
            free_term_layout(out);
            return FEW_E_NOMEM;
        }
        std::memcpy(out->mrows, mr.data(), sizeof(int) * mr.size());
    }
    out->n_chunks = (int)chunks.size() - 1;
    out->n_segs = (int)segs.size() / 4;
    out->n_terms = term;
    out->n_src = (int)src.size() / 2;
    out->segs = (int *)std::malloc(sizeof(int) * segs.size());
    out->term_ptr = (int *)std::malloc(sizeof(int) * term_ptr.size());
    out->term_src = (int *)std::malloc(sizeof(int) * std::max<size_t>(src.size(), 2));
    out->chunks = (int *)std::malloc(sizeof(int) * chunks.size());
    if (!out->segs || !out->term_ptr || !out->term_src || !out->chunks) {
        free_term_layout(out);
        return FEW_E_NOMEM;
    }
    std::memcpy(out->segs, segs.data(), sizeof(int) * segs.size());
    std::memcpy(out->term_ptr, term_ptr.data(), sizeof(int) * term_ptr.size());
    std::memcpy(out->term_src, src.data(), sizeof(int) * src.size());
    std::memcpy(out->chunks, chunks.data(), sizeof(int) * chunks.size());
    return FEW_OK;
}

// Sec. II frame conventions.  With R (sky position) and S (spin direction) as
// unit vectors in the barycentre frame, the source frame has z = S and x along
// R x S, so the observer, at -R from the source, sits at polar angle
// arccos(-R.S) and azimuth -pi/2.  The pi/2 turn of the polarisation basis is a
// sign flip of h, and the barycentre frame follows by turning the basis through
// psi, tan psi = [cos tS sin tK cos(pS - pK) - sin tS cos tK] /
// [sin tK sin(pS - pK)], which multiplies h by e^{-2 i psi}.  e^{-2 i psi} is
// formed from the numerator a and denominator b directly:
// (b - i a)^2 / (a^2 + b^2); R parallel to S leaves psi undefined: factor 1.
int detector_frame(double theta_s, double phi_s, double theta_k, double phi_k,
                   double *theta_src, double *phi_src, double *rot_re, double *rot_im) {
    if (!std::isfinite(theta_s) || !std::isfinite(phi_s) || !std::isfinite(theta_k) ||
        !std::isfinite(phi_k))
        return FEW_E_ARG;
    const double st = std::sin(theta_s), ct = std::cos(theta_s);
    const double sk = std::sin(theta_k), ck = std::cos(theta_k);
    const double rs = st * sk * std::cos(phi_s - phi_k) + ct * ck;      // R . S
    const double c = std::max(-1.0, std::min(1.0, -rs));
    *theta_src = std::acos(c);
    *phi_src = -M_PI / 2;
    const double a = ct * sk * std::cos(phi_s - phi_k) - st * ck;
    const double b = sk * std::sin(phi_s - phi_k);
    const double q = a * a + b * b;
    double er = 1.0, ei = 0.0;                                          // e^{-2 i psi}
    if (q > 0.0) {
        er = (b * b - a * a) / q;
        ei = -2.0 * a * b / q;
    }
    *rot_re = -er;
    *rot_im = -ei;
    return FEW_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

ReqLayout request_layout(bool fp32, int K, int M, int n_segs, int n_terms, int n_src,
                         int n_chunks, int n_ph, bool mfma, int n_mrows) {
    ReqLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    // host-uploaded arrays first, contiguous, so one copy stages them
    L.off_t = take(sizeof(double) * K);
    L.off_segs = take(sizeof(int) * 4 * (size_t)n_segs);
    L.off_term_ptr = take(sizeof(int) * (size_t)(n_terms + 1));
    L.off_term_src = take(sizeof(int) * 2 * (size_t)std::max(n_src, 1));
    L.off_chunks = take(sizeof(int) * (size_t)(n_chunks + 1));
    L.off_mrows = take(sizeof(int) * 2 * (size_t)(n_mrows + 1));
    L.upload_end = L.off_mrows + sizeof(int) * 2 * (size_t)(n_mrows + 1);
    // device-produced arrays
    L.off_pcoef = take(sizeof(double) * 8 * n_ph * (size_t)(K - 1));
    L.dev_begin = L.off_pcoef;
    L.off_acoef = take(sizeof(double) * 8 * (size_t)(K - 1) * M);
    L.off_ybuf = take(sizeof(double) * 2 * (size_t)std::max(n_src, 1));
    // fold table of the vector kernels (matrix-core requests fold straight
    // into the fp16 operand table)
    L.off_table = take(mfma ? 0 : (fp32 ? 4 : 8) * 8 * (size_t)(K - 1) * n_terms);
    L.off_starts = take(sizeof(long long) * K);
    L.off_tile_pref = take(sizeof(int) * kParts * (size_t)K);
    L.off_mtab = take(mfma ? sizeof(uint16_t) * kMfIntervalHalves * (size_t)(K - 1) : 0);
    L.off_mscale = take(mfma ? sizeof(float) * kMfRows * (size_t)(K - 1) : 0);
    L.total = o;
    return L;
}

}  // namespace few

using namespace few;

static int32_t host_terms(int32_t M, const int32_t *modes, int width, int32_t max_gap,
                          int32_t cap_segs, int32_t *segs, int32_t *n_segs,
                          int32_t cap_terms, int32_t *term_ptr, int32_t *n_terms,
                          int32_t cap_src, int32_t *term_src, int32_t *n_src) {
    if (!modes || !segs || !n_segs || !term_ptr || !n_terms || !term_src || !n_src ||
        max_gap < 0)
        return FEW_E_ARG;
    TermLayout L;
    int rc = build_term_layout(M, modes, width, max_gap, &L);
    if (rc) return rc;
    *n_segs = L.n_segs;
    *n_terms = L.n_terms;
    *n_src = L.n_src;
    if (L.n_segs > cap_segs || L.n_terms + 1 > cap_terms || L.n_src > cap_src) {
        free_term_layout(&L);
        return FEW_E_ARG;
    }
    std::memcpy(segs, L.segs, sizeof(int) * 4 * L.n_segs);
    std::memcpy(term_ptr, L.term_ptr, sizeof(int) * (L.n_terms + 1));
    std::memcpy(term_src, L.term_src, sizeof(int) * 2 * L.n_src);
    free_term_layout(&L);
    return FEW_OK;
}

extern "C" int32_t few_host_terms(int32_t M, const int32_t *lmn, int32_t max_gap,
                                  int32_t cap_segs, int32_t *segs, int32_t *n_segs,
                                  int32_t cap_terms, int32_t *term_ptr, int32_t *n_terms,
                                  int32_t cap_src, int32_t *term_src, int32_t *n_src) {
    return host_terms(M, lmn, 3, max_gap, cap_segs, segs, n_segs, cap_terms, term_ptr,
                      n_terms, cap_src, term_src, n_src);
}

extern "C" int32_t few_host_terms_kerr(int32_t M, const int32_t *lmkn, int32_t max_gap,
                                       int32_t cap_segs, int32_t *segs, int32_t *n_segs,
                                       int32_t cap_terms, int32_t *term_ptr, int32_t *n_terms,
                                       int32_t cap_src, int32_t *term_src, int32_t *n_src) {
    return host_terms(M, lmkn, 4, max_gap, cap_segs, segs, n_segs, cap_terms, term_ptr,
                      n_terms, cap_src, term_src, n_src);
}

extern "C" int32_t few_host_frame(double theta_s, double phi_s, double theta_k, double phi_k,
                                  double *out4) {
    if (!out4) return FEW_E_ARG;
    return detector_frame(theta_s, phi_s, theta_k, phi_k, &out4[0], &out4[1], &out4[2],
                          &out4[3]);
}

extern "C" int32_t few_host_interval_starts(int32_t K, const double *t_knots, double t_start,
                                            double dt, int64_t n, int64_t *starts) {
    if (!t_knots || !starts || K < 4 || n < 1 || !(dt > 0.0)) return FEW_E_ARG;
    interval_starts(K, t_knots, t_start, dt, (long long)n, (long long *)starts);
    return FEW_OK;
}

extern "C" uint64_t few_host_request_bytes(int32_t precision, int32_t K, int32_t M,
                                           int32_t n_terms) {
    if (K < 4 || M < 1 || n_terms < 1) return 0;
    // n_src <= 2M, n_segs <= n_terms
    // binary32 requests long enough for the matrix-core path are sized for it
    const bool mf = precision == FEW_MIXED && n_terms >= kMfMinTerms;
    ReqLayout L = request_layout(precision == FEW_MIXED, K, M, n_terms, n_terms, 2 * M, n_terms,
                                 3, mf, mf ? kMfRows : 0);
    return (uint64_t)L.total;
}

extern "C" int32_t few_host_mfma_path(int32_t M, const int32_t *lmn) {
    TermLayout L;
    const int rc = build_term_layout(M, lmn, 3, kMaxGap, &L);
    if (rc) return rc;
    const int ok = L.mfma ? 1 : 0;
    free_term_layout(&L);
    return ok;
}

extern "C" void few_host_mfma_shape(int32_t *out8) {
    if (!out8) return;
    out8[0] = kMfWaves;
    out8[1] = kMfNT;
    out8[2] = kMfMT;
    out8[3] = kMfT;
    out8[4] = 4 * kMfMT * kMfT * 3;
    out8[5] = kMfA;
    out8[6] = kMfRows;
    out8[7] = kMfMinTerms;
}
