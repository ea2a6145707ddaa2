// libfew host runtime: the C ABI of include/few.h.
//
// Synchronous path: few_spline_fit (upload small host arrays, fit kernel) and
// few_mode_sum (prepare kernel, sum kernel) enqueue on the caller's stream.
// Served path: few_submit queues requests; one scheduler thread per plan
// admits them in arrival order while their footprint fits the device arena,
// packs the admitted ones into one batched launch (fit, prepare, persistent
// sum) on one of max_inflight streams, and retires a batch when its completion
// event fires.  Work of different requests never shares a wave, so every
// result is bitwise the same alone or in a batch.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/few.h"
#include "few_internal.h"

using namespace few;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(FEW_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));            \
    } while (0)

// ---------------------------------------------------------------------------
// XCD split of the matrix-core summation (one per stream the plan launches
// on).  The workgroups of each store launch report their times, tagged with
// the launch's number, in the pinned array rep; before a launch, the latest
// complete report (every workgroup with one tag, and the weights that launch
// used still in the history) moves each weight half way towards equal XCD
// finishing times, w_x (1 + (T / T_x - 1) / 2) with T_x the longest time of
// XCD x and T their mean, renormalised to mean 1 within [1/2, 2].  Reports
// are read while later launches may overwrite them: a mixed set is skipped.
// ---------------------------------------------------------------------------
// One step of that rule: the weights wp[8] a launch used and its XCDs'
// finishing times T[8] > 0 give the next weights w[8].
void xcd_split_step(const double *wp, const double *T, double *w) {
    double mean = 0.0;
    for (int x = 0; x < 8; ++x) mean += 0.125 * T[x];
    double s = 0.0;
    for (int x = 0; x < 8; ++x) {
        w[x] = wp[x] * (1.0 + 0.5 * (mean / T[x] - 1.0));
        s += 0.125 * w[x];
    }
    for (int x = 0; x < 8; ++x) w[x] = std::min(2.0, std::max(0.5, w[x] / s));
}

struct XcdSplit {
    unsigned long long *rep = nullptr;  // [kMfBalanceWG], pinned host memory
    double w[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    unsigned tag = 0;                   // tag of the next launch
    unsigned applied = ~0u;             // last report folded in
    struct Used {
        unsigned tag = ~0u;
        double w[8];
    } hist[8];                          // weights of the last launches, by tag mod 8
    std::mutex mu;

    void apply(SumJob *j, int G) {
        std::lock_guard<std::mutex> g(mu);
        constexpr unsigned kTagMask = (1u << (64 - kMfTagShift)) - 1;
        if (G % 8 == 0 && G <= kMfBalanceWG) {
            const volatile unsigned long long *r = rep;
            const unsigned t = (unsigned)(r[0] >> kMfTagShift);
            bool ok = t != applied;
            double T[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int i = 0; i < G && ok; ++i) {
                const unsigned long long v = r[i];
                ok = (unsigned)(v >> kMfTagShift) == t;
                T[i & 7] = std::max(T[i & 7], (double)(v & ((1ull << kMfTagShift) - 1)));
            }
            const Used &u = hist[t % 8];
            ok = ok && u.tag == t;
            for (int x = 0; x < 8; ++x) ok = ok && T[x] > 0.0;
            if (ok) {
                xcd_split_step(u.w, T, w);
                applied = t;
            }
        }
        const unsigned tg = tag & kTagMask;
        j->btime = rep;
        j->btag = tg;
        for (int x = 0; x < 8; ++x) j->bw[x] = (float)w[x];
        Used &h = hist[tg % 8];
        h.tag = tg;
        for (int x = 0; x < 8; ++x) h.w[x] = (double)j->bw[x];
        ++tag;
    }
};

// ---------------------------------------------------------------------------
// Device arena: one hipMalloc per plan, first-fit sub-allocation on the host.
// ---------------------------------------------------------------------------
class Arena {
  public:
    void init(char *base, size_t size) {
        base_ = base;
        size_ = size;
        free_.clear();
        free_[0] = size;
        used_ = 0;
    }
    // returns offset or SIZE_MAX
    size_t alloc(size_t bytes) {
        std::lock_guard<std::mutex> g(mu_);
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
                live_[off] = bytes;
                used_ += bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = live_.find(off);
        if (it == live_.end()) return;
        size_t sz = it->second;
        live_.erase(it);
        used_ -= sz;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + sz == nx->first) {
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += sz;
                return;
            }
        }
        free_[off] = sz;
    }
    // whether alloc(bytes) would succeed now
    bool alloc_probe(size_t bytes) {
        std::lock_guard<std::mutex> g(mu_);
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        for (auto &kv : free_)
            if (kv.second >= bytes) return true;
        return false;
    }
    char *ptr(size_t off) const { return base_ + off; }
    size_t size() const { return size_; }

  private:
    std::mutex mu_;
    char *base_ = nullptr;
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_, live_;
};

// Reusable pinned host buffers (hipHostMalloc is slow; keep them).
class PinnedPool {
  public:
    void *get(size_t bytes) {
        std::lock_guard<std::mutex> g(mu_);
        for (auto &b : bufs_)
            if (!b.busy && b.size >= bytes) {
                b.busy = true;
                return b.ptr;
            }
        void *p = nullptr;
        size_t sz = std::max<size_t>(bytes, 1 << 16);
        if (hipHostMalloc(&p, sz, hipHostMallocCoherent) != hipSuccess) return nullptr;
        bufs_.push_back({p, sz, true});
        return p;
    }
    void put(void *p) {
        std::lock_guard<std::mutex> g(mu_);
        for (auto &b : bufs_)
            if (b.ptr == p) b.busy = false;
    }
    void clear() {
        std::lock_guard<std::mutex> g(mu_);
        for (auto &b : bufs_) hipHostFree(b.ptr);
        bufs_.clear();
    }

  private:
    struct Buf {
        void *ptr;
        size_t size;
        bool busy;
    };
    std::mutex mu_;
    std::vector<Buf> bufs_;
};

enum Stage { ST_FIT = 0, ST_PREP = 1, ST_SUM = 2 };

// One request's host-side description and arena placement.
struct HostReq {
    int K = 0, M = 0;
    int width = 3;             // modes (l, m, n), or (l, m, k, n) for generic Kerr
    int n_ph = 2;              // splined phases: Phi_phi, Phi_r (+ Phi_theta)
    std::vector<double> t;
    TermLayout terms;
    ReqLayout L{};
    size_t upload_bytes = 0;   // [0, upload_bytes) of the layout comes from the host
    bool mfma = false;         // binary32 sums of this request run on the matrix-core path
    ~HostReq() { free_term_layout(&terms); }
};

int validate_fit_args(int K, const double *t, int M, const int32_t *lmn, const void *pp,
                      const void *pr, const void *amp, int max_knots, int max_modes,
                      int width = 3, const void *pt = nullptr) {
    if (!t || !lmn || !pp || !pr || !amp || (width == 4 && !pt))
        return fail(FEW_E_ARG, "null pointer argument");
    if (K < 4 || K > max_knots)
        return fail(FEW_E_KNOTS, "K = %d outside [4, %d]", K, max_knots);
    for (int i = 0; i < K; ++i)
        if (!std::isfinite(t[i])) return fail(FEW_E_KNOTS, "knot %d is not finite", i);
    for (int i = 0; i + 1 < K; ++i)
        if (!(t[i + 1] > t[i]))
            return fail(FEW_E_KNOTS, "knots not strictly increasing at %d", i);
    if (M < 1 || M > max_modes) return fail(FEW_E_MODES, "M = %d outside [1, %d]", M, max_modes);
    for (int k = 0; k < M; ++k) {
        const int32_t *md = lmn + (size_t)width * k;
        int l = md[0], m = md[1], kp = width == 4 ? md[2] : 0, n = md[width - 1];
        if (l < 2 || l > kMaxL || m < 0 || m > l || n < -kMaxAbsN || n > kMaxAbsN ||
            kp < -kMaxAbsK || kp > kMaxAbsK)
            return fail(FEW_E_MODES,
                        "mode %d = (l %d, m %d, k %d, n %d) invalid (2<=l<=%d, 0<=m<=l, |k|<=%d, "
                        "|n|<=%d)",
                        k, l, m, kp, n, kMaxL, kMaxAbsK, kMaxAbsN);
    }
    return FEW_OK;
}

int validate_sum_args(const double *t, int K, double theta, double phi, double scale,
                      double t_start, double dt, int64_t n, const void *out) {
    if (!out) return fail(FEW_E_ARG, "null output pointer");
    if (!std::isfinite(theta) || !std::isfinite(phi) || !std::isfinite(scale) ||
        !std::isfinite(t_start) || !std::isfinite(dt))
        return fail(FEW_E_ARG, "non-finite scalar argument");
    if (!(dt > 0.0)) return fail(FEW_E_ARG, "dt must be > 0");
    if (n < 1) return fail(FEW_E_ARG, "n_samples must be >= 1");
    if ((n + 255) / 64 + K > (int64_t)0x3fffffff) return fail(FEW_E_ARG, "n_samples too large");
    if (!(t_start >= t[0])) return fail(FEW_E_RANGE, "t_start before the first knot");
    if (!(sample_time(t_start, dt, n - 1) <= t[K - 1]))
        return fail(FEW_E_RANGE, "last sample after the last knot");
    return FEW_OK;
}

// Fill the upload region [0, upload_bytes) of a request layout in host memory.
void stage_upload(const HostReq &r, char *dst) {
    std::memcpy(dst + r.L.off_t, r.t.data(), sizeof(double) * r.K);
    std::memcpy(dst + r.L.off_segs, r.terms.segs, sizeof(int) * 4 * r.terms.n_segs);
    std::memcpy(dst + r.L.off_term_ptr, r.terms.term_ptr, sizeof(int) * (r.terms.n_terms + 1));
    std::memcpy(dst + r.L.off_term_src, r.terms.term_src, sizeof(int) * 2 * r.terms.n_src);
    std::memcpy(dst + r.L.off_chunks, r.terms.chunks, sizeof(int) * (r.terms.n_chunks + 1));
    std::memcpy(dst + r.L.off_mrows, r.terms.mrows, sizeof(int) * 2 * (r.terms.n_mrows + 1));
}

// Recently used term layouts, keyed by the full mode list (an MCMC client
// resubmits the same mode sets many times; building a layout costs ~0.1 ms at
// 3843 modes).  Most recently used first; entries are matched by a hash of the
// list, then by the list itself.
class LayoutCache {
  public:
    ~LayoutCache() {
        for (auto &e : entries_) free_term_layout(&e.layout);
    }
    // Fill *out with an owned copy of the layout of M modes of `width` ints.
    int get(int M, const int32_t *lmn, int width, TermLayout *out) {
        const size_t words = (size_t)width * M;
        const uint64_t h = hash(words, lmn) ^ (uint64_t)width;
        std::lock_guard<std::mutex> g(mu_);
        for (size_t i = 0; i < entries_.size(); ++i) {
            Entry &e = entries_[i];
            if (e.hash == h && e.width == width && e.lmn.size() == words &&
                std::memcmp(e.lmn.data(), lmn, sizeof(int32_t) * words) == 0) {
                int rc = copy(e.layout, out);
                if (!rc && i != 0) std::rotate(entries_.begin(), entries_.begin() + i,
                                               entries_.begin() + i + 1);
                return rc;
            }
        }
        TermLayout L;
        int rc = build_term_layout(M, lmn, width, kMaxGap, &L);
        if (rc) return rc;
        rc = copy(L, out);
        if (rc) {
            free_term_layout(&L);
            return rc;
        }
        if (entries_.size() == kCap) {
            free_term_layout(&entries_.back().layout);
            entries_.pop_back();
        }
        entries_.insert(entries_.begin(),
                        Entry{h, width, std::vector<int32_t>(lmn, lmn + words), L});
        return FEW_OK;
    }

  private:
    static constexpr size_t kCap = 256;
    struct Entry {
        uint64_t hash;
        int width;
        std::vector<int32_t> lmn;
        TermLayout layout;
    };
    // FNV-1a over the 32-bit words of the list
    static uint64_t hash(size_t words, const int32_t *lmn) {
        uint64_t h = 1469598103934665603ULL;
        for (size_t i = 0; i < words; ++i) {
            h ^= (uint32_t)lmn[i];
            h *= 1099511628211ULL;
        }
        return h;
    }
    static int copy(const TermLayout &a, TermLayout *b) {
        *b = TermLayout{};
        b->n_segs = a.n_segs;
        b->n_terms = a.n_terms;
        b->n_src = a.n_src;
        b->n_chunks = a.n_chunks;
        for (int q = 0; q < kTermGroups - 1; ++q) b->grp[q] = a.grp[q];
        b->max_seg_terms = a.max_seg_terms;
        b->n_mrows = a.n_mrows;
        b->n_min = a.n_min;
        b->n_max = a.n_max;
        b->l_max = a.l_max;
        b->mfma = a.mfma;
        b->mrows = (int *)std::malloc(sizeof(int) * 2 * (size_t)(a.n_mrows + 1));
        b->segs = (int *)std::malloc(sizeof(int) * 4 * (size_t)a.n_segs);
        b->term_ptr = (int *)std::malloc(sizeof(int) * (size_t)(a.n_terms + 1));
        b->term_src = (int *)std::malloc(sizeof(int) * 2 * (size_t)std::max(a.n_src, 1));
        b->chunks = (int *)std::malloc(sizeof(int) * (size_t)(a.n_chunks + 1));
        if (!b->segs || !b->term_ptr || !b->term_src || !b->chunks || !b->mrows) {
            free_term_layout(b);
            return FEW_E_NOMEM;
        }
        std::memcpy(b->mrows, a.mrows, sizeof(int) * 2 * (size_t)(a.n_mrows + 1));
        std::memcpy(b->chunks, a.chunks, sizeof(int) * (size_t)(a.n_chunks + 1));
        std::memcpy(b->segs, a.segs, sizeof(int) * 4 * (size_t)a.n_segs);
        std::memcpy(b->term_ptr, a.term_ptr, sizeof(int) * (size_t)(a.n_terms + 1));
        std::memcpy(b->term_src, a.term_src, sizeof(int) * 2 * (size_t)a.n_src);
        return FEW_OK;
    }
    std::mutex mu_;
    std::vector<Entry> entries_;
};

int make_host_req(int K, const double *t, int M, const int32_t *lmn, bool fp32, HostReq *r,
                  LayoutCache *cache, int width = 3, bool allow_mfma = true) {
    r->K = K;
    r->M = M;
    r->width = width;
    r->n_ph = width == 4 ? 3 : 2;
    r->t.assign(t, t + K);
    int rc = cache->get(M, lmn, width, &r->terms);
    if (rc) return fail(rc, "mode list rejected while building the term layout");
    r->mfma = fp32 && allow_mfma && r->terms.mfma && width == 3;
    r->L = request_layout(fp32, K, M, r->terms.n_segs, r->terms.n_terms, r->terms.n_src,
                          r->terms.n_chunks, r->n_ph, r->mfma, r->terms.n_mrows);
    r->upload_bytes = r->L.upload_end;
    return FEW_OK;
}

// Where one request's arrays live on the device: the host-uploaded arrays
// ([0, dev_begin) of its layout) at `up`, the device-produced ones at `dev`.
// A request in one block has dev = up + dev_begin; a batch packs every
// request's upload region together so one small copy stages them all.
struct ReqBase {
    char *up, *dev;
};

ReqBase one_block(const HostReq &r, char *base) { return {base, base + r.L.dev_begin}; }

template <class T>
T *at_up(const HostReq &r, ReqBase b, size_t off) {
    (void)r;
    return (T *)(b.up + off);
}

template <class T>
T *at_dev(const HostReq &r, ReqBase b, size_t off) {
    return (T *)(b.dev + (off - r.L.dev_begin));
}

FitJob fit_job(const HostReq &r, ReqBase base, const double *pp, const double *pr,
               const double *amp, const double *pt = nullptr) {
    FitJob j{};
    j.t = at_up<const double>(r, base, r.L.off_t);
    j.phi_phi = pp;
    j.phi_r = pr;
    j.phi_theta = pt;
    j.n_ph = r.n_ph;
    j.amp = amp;
    j.pcoef = at_dev<double>(r, base, r.L.off_pcoef);
    j.acoef = at_dev<double>(r, base, r.L.off_acoef);
    j.acoef_pmajor = r.mfma ? 1 : 0;
    j.K = r.K;
    j.M = r.M;
    j.amp_blocks = (2 * r.M + kFitSeriesPerBlock - 1) / kFitSeriesPerBlock;
    return j;
}

// How a launch cuts a request into tiles: `parts` contiguous sample parts and
// the short-tile region at the end of each.
struct Tiling {
    int parts;
    long long short_len;
    bool split = false;     // short tiles are term-split tiles (binary32)
};

// Single-request launch: one part per XCD; binary32 parts end in short tiles
// worth FEW_SHORT_QUARTERS / 4 of one round of long tiles over the `resident`
// workgroups.  Batched launches use Tiling{1, 0}.
Tiling single_tiling(bool fp32, int resident) {
    Tiling t{kParts, 0};
    if (fp32 && resident > 0)
        t.short_len = (long long)resident * tile_samples(true) * FEW_SHORT_QUARTERS / 4 / kParts;
    return t;
}

PrepJob prep_job(const HostReq &r, ReqBase base, double theta, double phi, double scale,
                 double t_start, double dt, int64_t n, bool fp32, Tiling tl) {
    PrepJob j{};
    j.t = at_up<const double>(r, base, r.L.off_t);
    j.acoef = at_dev<const double>(r, base, r.L.off_acoef);
    j.term_ptr = at_up<const int>(r, base, r.L.off_term_ptr);
    j.term_src = at_up<const int2>(r, base, r.L.off_term_src);
    j.ybuf = at_dev<double2>(r, base, r.L.off_ybuf);
    j.table = at_dev<char>(r, base, r.L.off_table);
    j.starts = at_dev<long long>(r, base, r.L.off_starts);
    j.tile_pref = at_dev<int>(r, base, r.L.off_tile_pref);
    j.theta = theta;
    j.phi = phi;
    j.scale = scale;
    j.t_start = t_start;
    j.dt = dt;
    j.n = n;
    j.K = r.K;
    j.M = r.M;
    j.n_terms = r.terms.n_terms;
    j.n_src = r.terms.n_src;
    j.tile = tile_samples(fp32);
    j.short_tile = tl.split ? split_tile_samples() : short_tile_samples(fp32);
    j.short_len = tl.short_len;
    j.parts = tl.parts;
    // about one (interval, term) pair per lane of a 256-lane fold workgroup
    j.fold_terms = std::max(1, std::min(64, 256 / (r.K - 1)));
    j.fold_blocks = (r.terms.n_terms + j.fold_terms - 1) / j.fold_terms;
    j.segs = at_up<const int4>(r, base, r.L.off_segs);
    j.mrows = at_up<const int2>(r, base, r.L.off_mrows);
    j.mtab = r.mfma ? at_dev<char>(r, base, r.L.off_mtab) : nullptr;
    j.mscale = r.mfma ? at_dev<float>(r, base, r.L.off_mscale) : nullptr;
    j.n_mrows = r.terms.n_mrows;
    j.n_min = r.terms.n_min;
    j.n_segs = r.terms.n_segs;
    j.l_max = r.terms.l_max;
    return j;
}

SumJob sum_job(const HostReq &r, ReqBase base, double t_start, double dt, int64_t n, void *out,
               Tiling tl) {
    SumJob j{};
    j.t = at_up<const double>(r, base, r.L.off_t);
    j.pcoef = at_dev<const double>(r, base, r.L.off_pcoef);
    j.table = at_dev<char>(r, base, r.L.off_table);
    j.segs = at_up<const int4>(r, base, r.L.off_segs);
    j.chunks = at_up<const int>(r, base, r.L.off_chunks);
    j.starts = at_dev<const long long>(r, base, r.L.off_starts);
    j.tile_pref = at_dev<const int>(r, base, r.L.off_tile_pref);
    j.out = out;
    j.t_start = t_start;
    j.dt = dt;
    j.n = n;
    j.K = r.K;
    j.n_terms = r.terms.n_terms;
    j.n_segs = r.terms.n_segs;
    j.n_chunks = r.terms.n_chunks;
    j.n_ph = r.n_ph;
    j.short_len = tl.short_len;
    j.parts = tl.parts;
    j.wave_base = 0;
    for (int q = 0; q < kTermGroups - 1; ++q) j.grp[q] = r.terms.grp[q];
    j.split = tl.split ? 1 : 0;
    j.mtab = r.mfma ? at_dev<const char>(r, base, r.L.off_mtab) : nullptr;
    j.mscale = r.mfma ? at_dev<const float>(r, base, r.L.off_mscale) : nullptr;
    j.mrows = at_up<const int2>(r, base, r.L.off_mrows);
    j.n_mrows = r.terms.n_mrows;
    j.n_min = r.terms.n_min;
    j.sample_base = 0;
    return j;
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan and spline objects.
// ---------------------------------------------------------------------------
struct ServedReq {
    uint64_t ticket;
    few_request r;
    HostReq h;
    int status = FEW_PENDING;
    size_t footprint = 0;
    // recorded on the plan stream at submit: the batch stream waits for it, so
    // work the caller enqueued there before few_submit (producing the inputs,
    // last using the output buffer) is complete before the request runs
    hipEvent_t ready = nullptr;
    // request log: microseconds since plan creation (host steady clock)
    double t_arrive = 0.0, t_admit = -1.0;
    long long batch = -1;
    int batch_size = 0;
};

struct Batch {
    int slot;                  // stream index
    size_t arena_off = SIZE_MAX;
    void *pinned = nullptr;
    hipEvent_t done = nullptr;
    std::vector<ServedReq *> reqs;
};

struct few_plan_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool fp32 = false;
    int max_knots = kMaxKnots, max_modes = 65536, max_inflight = 2;
    int resident_wg = 0;        // binary32 summation workgroups resident at once
    int resident_wg3 = 0;       // the same for the generic-Kerr kernel
    int mf_wg = 0;              // matrix-core summation workgroups (one per compute unit)
    bool allow_mfma = true;     // binary32 requests may take the matrix-core path
    // inner-product partial sums (grown on demand; the plan stream is drained
    // before a smaller buffer is released)
    double2 *inner_partial = nullptr;
    double2 *scratch = nullptr;   // device address of the static partial-sum array (no-alloc path)
    size_t inner_off = SIZE_MAX;
    long long inner_cap = 0;
    uint64_t budget = 0;
    int flags = 0;
    char *arena_base = nullptr;
    Arena arena;
    PinnedPool pinned;
    // synchronous-path staging: two alternating pinned slots
    void *stage[2] = {nullptr, nullptr};
    size_t stage_size[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_pending[2] = {false, false};
    int stage_next = 0;
    std::mutex sync_mu;
    std::set<few_spline> splines;
    LayoutCache layouts;
    // timing
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> timed;
    std::vector<hipEvent_t> ev_pool;
    double acc_ms[3] = {0, 0, 0};
    int64_t acc_n[3] = {0, 0, 0};
    // served path
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServedReq *> pending;
    std::unordered_map<uint64_t, ServedReq *> tickets;
    std::vector<Batch *> inflight;
    std::vector<hipStream_t> bstreams;
    std::vector<bool> slot_busy;
    std::thread worker;
    bool stop = false, worker_started = false;
    uint64_t next_ticket = 1;
    unsigned *counters = nullptr;   // one persistent-kernel counter per stream slot
    // few_batch on the plan stream: its own counter
    unsigned *sync_counter = nullptr;
    // XCD split of the matrix-core summation: one per served stream slot,
    // then the plan stream's
    std::unique_ptr<XcdSplit[]> xsplit;
    std::atomic<unsigned long long> sum_launches{0};    // FEW_FLAG_TIMING_SPARSE
    // Arena blocks (and pinned buffers) released once the event recorded after
    // the last work that uses them has completed: few_spline_free, few_batch
    // blocks and grown inner-product buffers.  The served scheduler carves the
    // same arena for batches on other streams, so a block is never handed out
    // again while queued plan-stream work still reads it.
    struct Deferred {
        size_t arena_off;
        void *pinned;
        hipEvent_t ev;
    };
    std::mutex def_mu;                  // deferred and sync_events
    std::vector<Deferred> deferred;
    std::vector<hipEvent_t> sync_events;   // pool of timing-disabled events
    // request log (few_plan_log), written under mu
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    FILE *log = nullptr;
    long long n_batches = 0;
};

struct few_spline_s {
    few_plan plan = nullptr;
    HostReq h;
    size_t arena_off = SIZE_MAX;
};

namespace {

hipEvent_t pool_event(few_plan p) {
    if (!p->ev_pool.empty()) {
        hipEvent_t e = p->ev_pool.back();
        p->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Run launch() between two timing events when FEW_FLAG_TIMING is set (or
// FEW_FLAG_TIMING_SUM, for summation launches).
template <typename F>
int timed_launch(few_plan p, int stage, hipStream_t s, F launch) {
    hipEvent_t a = nullptr, b = nullptr;
    bool timed = (p->flags & FEW_FLAG_TIMING) || ((p->flags & FEW_FLAG_TIMING_SUM) && stage == ST_SUM);
    if (timed && stage == ST_SUM && (p->flags & FEW_FLAG_TIMING_SPARSE))
        timed = p->sum_launches++ % 8 == 0;
    if (timed) {
        a = pool_event(p);
        b = pool_event(p);
        if (a && b) hipEventRecord(a, s);
    }
    hipError_t e = launch();
    if (e != hipSuccess) return fail(FEW_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    if (a && b) {
        hipEventRecord(b, s);
        p->timed.push_back({stage, {a, b}});
    }
    return FEW_OK;
}

// Copy `bytes` of pinned host memory (from hipHostMalloc, host-coherent) to
// the device on stream s with the upload kernel: the GPU reads the host
// buffer directly, so the copy is ordered on the compute queue like the
// kernels that use it.
hipError_t pinned_upload(void *dst, void *host, size_t bytes, hipStream_t s) {
    void *src = nullptr;
    hipError_t e = hipHostGetDevicePointer(&src, host, 0);
    if (e != hipSuccess) return e;
    return launch_upload(src, dst, bytes, s);
}

// Pack a request's host tables into the next pinned slot (waiting, if need
// be, until the launch that last read that slot has completed); *slot is the
// slot's index and *dev its device address.
int stage_slot(few_plan p, const HostReq &r, int *slot, void **dev) {
    int s = p->stage_next;
    p->stage_next ^= 1;
    if (p->stage_pending[s]) {
        HIP_TRY(hipEventSynchronize(p->stage_ev[s]));
        p->stage_pending[s] = false;
    }
    if (p->stage_size[s] < r.upload_bytes) {
        if (p->stage[s]) hipHostFree(p->stage[s]);
        p->stage[s] = nullptr;
        size_t sz = std::max<size_t>(r.upload_bytes, 1 << 20);
        HIP_TRY(hipHostMalloc(&p->stage[s], sz, hipHostMallocCoherent));
        p->stage_size[s] = sz;
    }
    stage_upload(r, (char *)p->stage[s]);
    HIP_TRY(hipHostGetDevicePointer(dev, p->stage[s], 0));
    *slot = s;
    return FEW_OK;
}

// The slot may be rewritten once the work enqueued so far has read it.
int release_slot(few_plan p, int slot) {
    HIP_TRY(hipEventRecord(p->stage_ev[slot], p->stream));
    p->stage_pending[slot] = true;
    return FEW_OK;
}


void scheduler_main(few_plan p);
int launch_batch(few_plan p, Batch *b, hipStream_t s, unsigned *counter);
size_t batch_bytes(const std::vector<ServedReq *> &reqs);

// A timing-disabled event from the plan's pool (or a new one).
hipEvent_t sync_event(few_plan p) {
    {
        std::lock_guard<std::mutex> g(p->def_mu);
        if (!p->sync_events.empty()) {
            hipEvent_t e = p->sync_events.back();
            p->sync_events.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void put_sync_event(few_plan p, hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> g(p->def_mu);
    p->sync_events.push_back(e);
}

// Release arena block `off` (and pinned buffer `pinned`, if any) once the work
// enqueued so far on stream s has completed.  Without an event (creation or
// record failed) the stream is drained and the block released at once.
void defer_release(few_plan p, size_t off, void *pinned, hipStream_t s) {
    hipEvent_t e = sync_event(p);
    if (e && hipEventRecord(e, s) == hipSuccess) {
        std::lock_guard<std::mutex> g(p->def_mu);
        p->deferred.push_back({off, pinned, e});
        return;
    }
    if (e) put_sync_event(p, e);
    hipStreamSynchronize(s);
    if (off != SIZE_MAX) p->arena.release(off);
    if (pinned) p->pinned.put(pinned);
}

// Release deferred blocks whose work has completed (all of them if wait).
// Returns the number still outstanding.
size_t reap_deferred(few_plan p, bool wait) {
    std::lock_guard<std::mutex> g(p->def_mu);
    for (size_t i = 0; i < p->deferred.size();) {
        auto &d = p->deferred[i];
        if (wait) hipEventSynchronize(d.ev);
        if (hipEventQuery(d.ev) == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (d.arena_off != SIZE_MAX) p->arena.release(d.arena_off);
        if (d.pinned) p->pinned.put(d.pinned);
        p->sync_events.push_back(d.ev);
        p->deferred.erase(p->deferred.begin() + i);
    }
    return p->deferred.size();
}

// Arena allocation for work on the plan stream: retries after releasing the
// deferred blocks whose work has completed, then after waiting for all.
size_t alloc_sync(few_plan p, size_t bytes) {
    size_t off = p->arena.alloc(bytes);
    if (off != SIZE_MAX) return off;
    if (reap_deferred(p, false) == 0) return p->arena.alloc(bytes);
    off = p->arena.alloc(bytes);
    if (off != SIZE_MAX) return off;
    reap_deferred(p, true);
    return p->arena.alloc(bytes);
}

}  // namespace

extern "C" {

const char *few_last_error(void) { return g_err.c_str(); }

int32_t few_plan_create(const few_plan_desc *desc, few_plan *out) {
    try {
        if (!desc || !out) return fail(FEW_E_ARG, "null argument");
        if (desc->precision != FEW_FP64 && desc->precision != FEW_MIXED)
            return fail(FEW_E_ARG, "unknown precision %d", desc->precision);
        if (desc->max_knots < 0 || desc->max_knots > kMaxKnots)
            return fail(FEW_E_ARG, "max_knots must be in [0, %d]", kMaxKnots);
        if (desc->max_modes < 0) return fail(FEW_E_ARG, "max_modes < 0");
        if (desc->max_inflight < 0 || desc->max_inflight > 8)
            return fail(FEW_E_ARG, "max_inflight must be in [0, 8]");
        int ndev = 0;
        HIP_TRY(hipGetDeviceCount(&ndev));
        if (desc->device < 0 || desc->device >= ndev)
            return fail(FEW_E_ARG, "device %d not present (%d devices)", desc->device, ndev);
        HIP_TRY(hipSetDevice(desc->device));
        few_plan p = new (std::nothrow) few_plan_s;
        if (!p) return fail(FEW_E_NOMEM, "host allocation failed");
        p->device = desc->device;
        p->stream = (hipStream_t)desc->stream;
        p->fp32 = desc->precision == FEW_MIXED;
        p->resident_wg = p->fp32 ? sum_resident_workgroups(2) : 0;
        p->resident_wg3 = p->fp32 ? sum_resident_workgroups(3) : 0;
        p->mf_wg = p->fp32 ? mfma_workgroups() : 0;
        p->allow_mfma = p->fp32 && p->mf_wg > 0 && !(desc->flags & FEW_FLAG_VECTOR_ONLY);
        p->max_knots = desc->max_knots ? desc->max_knots : kMaxKnots;
        p->max_modes = desc->max_modes ? desc->max_modes : 65536;
        p->max_inflight = desc->max_inflight ? desc->max_inflight : 2;
        p->budget = desc->hbm_budget_bytes ? desc->hbm_budget_bytes : (2ull << 30);
        p->flags = desc->flags;
        void *base = nullptr;
        hipError_t e = hipMalloc(&base, p->budget);
        if (e != hipSuccess) {
            delete p;
            return fail(FEW_E_NOMEM, "arena hipMalloc(%llu) failed: %s",
                        (unsigned long long)desc->hbm_budget_bytes, hipGetErrorString(e));
        }
        p->arena_base = (char *)base;
        p->arena.init(p->arena_base, p->budget);
        // device address of this GPU's static partial-sum array, looked up now
        // with the plan's device current
        e = noalloc_scratch(p->device, &p->scratch);
        if (e != hipSuccess) {
            hipFree(base);
            delete p;
            return fail(FEW_E_HIP, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        }
        // persistent-kernel counters (one 256-byte block per served stream
        // slot, then the few_batch one) at the bottom of the arena, so these
        // long-lived blocks never split the space requests allocate from
        {
            const size_t off = p->arena.alloc(256 * (size_t)(p->max_inflight + 1));
            if (off == SIZE_MAX) {
                hipFree(base);
                delete p;
                return fail(FEW_E_TOO_LARGE, "plan budget below the counter blocks");
            }
            p->counters = (unsigned *)p->arena.ptr(off);
            p->sync_counter = p->counters + 64 * p->max_inflight;
        }
        {
            const size_t nb = (size_t)p->max_inflight + 1;
            p->xsplit.reset(new XcdSplit[nb]);
            for (size_t i = 0; i < nb; ++i) {
                void *h = nullptr;
                if (hipHostMalloc(&h, sizeof(unsigned long long) * kMfBalanceWG) != hipSuccess) {
                    for (size_t k = 0; k < i; ++k) hipHostFree(p->xsplit[k].rep);
                    hipFree(base);
                    delete p;
                    return fail(FEW_E_NOMEM, "pinned report array allocation failed");
                }
                std::memset(h, 0, sizeof(unsigned long long) * kMfBalanceWG);
                p->xsplit[i].rep = (unsigned long long *)h;
            }
        }
        for (int s = 0; s < 2; ++s) {
            if (hipEventCreateWithFlags(&p->stage_ev[s], hipEventDisableTiming) != hipSuccess) {
                hipFree(base);
                delete p;
                return fail(FEW_E_HIP, "hipEventCreate failed");
            }
        }
        *out = p;
        return FEW_OK;
    } catch (...) {
        return fail(FEW_E_NOMEM, "exception in few_plan_create");
    }
}

namespace {
double plan_us(few_plan p) {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - p->t0)
        .count();
}

// One JSON line per retired served request (caller holds p->mu).
void log_request(few_plan p, const ServedReq *r, double t_done) {
    if (!p->log) return;
    const char *path = !p->fp32 ? "fp64" : (r->h.mfma ? "mfma" : "vector");
    std::fprintf(p->log,
                 "{\"ticket\": %llu, \"status\": %d, \"knots\": %d, \"modes\": %d, "
                 "\"samples\": %lld, \"path\": \"%s\", \"batch\": %lld, "
                 "\"batch_size\": %d, \"arrive_us\": %.1f, \"admit_us\": %.1f, "
                 "\"done_us\": %.1f}\n",
                 (unsigned long long)r->ticket, r->status, r->h.K, r->h.M,
                 (long long)r->r.n_samples, path, r->batch, r->batch_size, r->t_arrive,
                 r->t_admit, t_done);
}
}  // namespace

int32_t few_plan_log(few_plan p, const char *path) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    std::lock_guard<std::mutex> g(p->mu);
    if (p->log) {
        std::fclose(p->log);
        p->log = nullptr;
    }
    if (!path) return FEW_OK;
    p->log = std::fopen(path, "a");
    if (!p->log) return fail(FEW_E_ARG, "cannot open request log %s", path);
    return FEW_OK;
}

int32_t few_plan_destroy(few_plan p) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    try {
        hipSetDevice(p->device);
        {
            std::unique_lock<std::mutex> g(p->mu);
            p->stop = true;
        }
        p->cv_work.notify_all();
        if (p->worker_started) p->worker.join();
        for (hipStream_t s : p->bstreams) {
            hipStreamSynchronize(s);
            hipStreamDestroy(s);
        }
        for (auto &kv : p->tickets) {
            if (kv.second->ready) hipEventDestroy(kv.second->ready);
            delete kv.second;
        }
        for (ServedReq *r : p->pending)
            if (!p->tickets.count(r->ticket)) {
                if (r->ready) hipEventDestroy(r->ready);
                delete r;
            }
        hipStreamSynchronize(p->stream);
        reap_deferred(p, true);
        for (hipEvent_t e : p->sync_events) hipEventDestroy(e);
        for (few_spline s : p->splines) delete s;
        for (auto &t : p->timed) {
            hipEventDestroy(t.second.first);
            hipEventDestroy(t.second.second);
        }
        for (hipEvent_t e : p->ev_pool) hipEventDestroy(e);
        for (int s = 0; s < 2; ++s) {
            if (p->stage[s]) hipHostFree(p->stage[s]);
            hipEventDestroy(p->stage_ev[s]);
        }
        p->pinned.clear();
        hipFree(p->arena_base);
        if (p->xsplit)
            for (int i = 0; i <= p->max_inflight; ++i) hipHostFree(p->xsplit[i].rep);
        if (p->log) std::fclose(p->log);
        delete p;
        return FEW_OK;
    } catch (...) {
        return fail(FEW_E_STATE, "exception in few_plan_destroy");
    }
}

namespace {
int spline_fit_impl(few_plan p, int32_t K, const double *t_knots, const double *phi_phi,
                    const double *phi_theta, const double *phi_r, int32_t M,
                    const int32_t *modes, int width, const double *amp, few_spline *out) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    if (!out) return fail(FEW_E_ARG, "null output handle");
    try {
        int rc = validate_fit_args(K, t_knots, M, modes, phi_phi, phi_r, amp, p->max_knots,
                                   p->max_modes, width, phi_theta);
        if (rc) return rc;
        std::lock_guard<std::mutex> g(p->sync_mu);
        HIP_TRY(hipSetDevice(p->device));
        few_spline s = new (std::nothrow) few_spline_s;
        if (!s) return fail(FEW_E_NOMEM, "host allocation failed");
        rc = make_host_req(K, t_knots, M, modes, p->fp32, &s->h, &p->layouts, width,
                           p->allow_mfma);
        if (rc) {
            delete s;
            return rc;
        }
        if (s->h.L.total > p->budget) {
            delete s;
            return fail(FEW_E_TOO_LARGE, "spline needs %zu bytes, plan budget %llu",
                        s->h.L.total, (unsigned long long)p->budget);
        }
        s->arena_off = alloc_sync(p, s->h.L.total);
        if (s->arena_off == SIZE_MAX) {
            delete s;
            return fail(FEW_E_NOMEM, "plan arena exhausted");
        }
        s->plan = p;
        char *base = p->arena.ptr(s->arena_off);
        // the fit launch carries the upload: no separate copy launch
        int slot = 0;
        void *staged = nullptr;
        rc = stage_slot(p, s->h, &slot, &staged);
        if (!rc) {
            FitJob job = fit_job(s->h, one_block(s->h, base), phi_phi, phi_r, amp, phi_theta);
            job.t = (const double *)((const char *)staged + s->h.L.off_t);
            job.up_src = (const uint4 *)staged;
            job.up_dst = (uint4 *)base;
            job.up_bytes = (long long)s->h.upload_bytes;
            rc = timed_launch(p, ST_FIT, p->stream,
                              [&] { return launch_fit(job, s->h.t.data(), p->stream); });
            const int rr = release_slot(p, slot);
            if (!rc) rc = rr;
        }
        if (rc) {
            defer_release(p, s->arena_off, nullptr, p->stream);
            delete s;
            return rc;
        }
        p->splines.insert(s);
        *out = s;
        return FEW_OK;
    } catch (...) {
        return fail(FEW_E_NOMEM, "exception in few_spline_fit");
    }
}
}  // namespace

int32_t few_spline_fit(few_plan p, int32_t K, const double *t_knots, const double *phi_phi,
                       const double *phi_r, int32_t M, const int32_t *lmn, const double *amp,
                       few_spline *out) {
    return spline_fit_impl(p, K, t_knots, phi_phi, nullptr, phi_r, M, lmn, 3, amp, out);
}

int32_t few_spline_fit_kerr(few_plan p, int32_t K, const double *t_knots,
                            const double *phi_phi, const double *phi_theta, const double *phi_r,
                            int32_t M, const int32_t *lmkn, const double *amp, few_spline *out) {
    return spline_fit_impl(p, K, t_knots, phi_phi, phi_theta, phi_r, M, lmkn, 4, amp, out);
}

int32_t few_spline_free(few_spline s) {
    if (!s || !s->plan) return fail(FEW_E_STATE, "bad spline handle");
    few_plan p = s->plan;
    std::lock_guard<std::mutex> g(p->sync_mu);
    if (!p->splines.count(s)) return fail(FEW_E_STATE, "spline not owned by its plan");
    // the block returns to the arena once the work queued on the plan stream so
    // far (which may still read it) has completed
    HIP_TRY(hipSetDevice(p->device));
    defer_release(p, s->arena_off, nullptr, p->stream);
    p->splines.erase(s);
    delete s;
    return FEW_OK;
}

int32_t few_spline_coefs(few_spline s, int32_t which, void *dst) {
    if (!s || !s->plan) return fail(FEW_E_STATE, "bad spline handle");
    if (!dst) return fail(FEW_E_ARG, "null destination");
    few_plan p = s->plan;
    HIP_TRY(hipSetDevice(p->device));
    char *base = p->arena.ptr(s->arena_off);
    if (which == 0) {
        if (s->h.mfma)
            HIP_TRY(launch_acoef_export((const double *)(base + s->h.L.off_acoef),
                                        (double *)dst, s->h.K, s->h.M, p->stream));
        else
            HIP_TRY(hipMemcpyAsync(dst, base + s->h.L.off_acoef,
                                   sizeof(double) * 8 * (size_t)(s->h.K - 1) * s->h.M,
                                   hipMemcpyDeviceToDevice, p->stream));
    } else if (which == 1) {
        HIP_TRY(hipMemcpyAsync(dst, base + s->h.L.off_pcoef,
                               sizeof(double) * 8 * s->h.n_ph * (size_t)(s->h.K - 1),
                               hipMemcpyDeviceToDevice, p->stream));
    } else {
        return fail(FEW_E_ARG, "which must be 0 (amplitudes) or 1 (phases)");
    }
    return FEW_OK;
}

namespace {
// Shared by few_mode_sum (out != null) and few_inner_product (data, out2).
int sum_impl(few_plan p, few_spline s, double theta, double phi, double scale, double t_start,
             double dt, int64_t n, void *out, const void *data, double *out2,
             double scale_im = 0.0, bool noalloc = false) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    if (!s || s->plan != p) return fail(FEW_E_STATE, "spline does not belong to this plan");
    const bool inner = data != nullptr;
    try {
        if (inner && !out2) return fail(FEW_E_ARG, "null result pointer");
        int rc = validate_sum_args(s->h.t.data(), s->h.K, theta, phi, scale, t_start, dt, n,
                                   inner ? data : out);
        if (rc) return rc;
        std::lock_guard<std::mutex> g(p->sync_mu);
        HIP_TRY(hipSetDevice(p->device));
        char *base = p->arena.ptr(s->arena_off);
        Tiling tl = single_tiling(p->fp32, s->h.n_ph == 3 ? p->resident_wg3 : p->resident_wg);
        tl.split = p->fp32 && tl.short_len > 0 && s->h.terms.n_terms >= kGroupMinTerms &&
                   s->h.terms.max_seg_terms <= kSplitTerms;
        PrepJob pj = prep_job(s->h, one_block(s->h, base), theta, phi, scale, t_start, dt, n,
                              p->fp32, tl);
        pj.scale_im = scale_im;
        SumJob sj = sum_job(s->h, one_block(s->h, base), t_start, dt, n, out, tl);
        // tiles per part; the grid holds parts x slots tiles.  Every size check
        // comes before the first launch.
        long long slots = part_tile_bound(n, tl.parts, tl.short_len, s->h.K,
                                          tile_samples(p->fp32), pj.short_tile);
        if (slots * tl.parts > 0x7fffffffLL) return fail(FEW_E_ARG, "too many samples");
        const bool mf = s->h.mfma;
        const long long need =
            !inner ? 0 : mf ? (long long)p->mf_wg : inner_slots(tl.parts, (int)slots, p->fp32);
        // matrix-core requests fold straight into the fp16 operand table
        auto prep = [&]() -> hipError_t {
            return mf ? launch_fold_pack(pj, p->stream) : launch_prepare(pj, p->fp32, p->stream);
        };
        auto sum = [&]() -> hipError_t {
            if (mf) {
                if (inner) return launch_sum_mfma_inner(sj, p->mf_wg, 2.0 * dt, out2, p->stream);
                SumJob sb = sj;
                p->xsplit[p->max_inflight].apply(&sb, p->mf_wg);
                return launch_sum_mfma(sb, p->mf_wg, p->stream);
            }
            return inner ? launch_sum_inner(sj, (int)slots, p->fp32, 2.0 * dt, out2, p->stream)
                         : launch_sum(sj, (int)slots, p->fp32, p->stream);
        };
        if (noalloc) {
            // partials in the static per-GPU array: no arena growth, no events
            if (need > kNoAllocSlots)
                return fail(FEW_E_TOO_LARGE,
                            "%lld partial-sum slots exceed the no-alloc limit of %lld "
                            "(about 16 million samples in binary64, 130 million in binary32, "
                            "at 100 knots)",
                            need, (long long)kNoAllocSlots);
            sj.data = data;
            sj.partial = p->scratch;
            HIP_TRY(prep());
            HIP_TRY(sum());
            return FEW_OK;
        }
        if (inner && need > p->inner_cap) {
            const long long cap = need + need / 4;
            const size_t off = alloc_sync(p, sizeof(double2) * (size_t)cap);
            if (off == SIZE_MAX) return fail(FEW_E_NOMEM, "plan arena exhausted (partials)");
            if (p->inner_off != SIZE_MAX) defer_release(p, p->inner_off, nullptr, p->stream);
            p->inner_off = off;
            p->inner_partial = (double2 *)p->arena.ptr(off);
            p->inner_cap = cap;
        }
        if (inner) {
            sj.data = data;
            sj.partial = p->inner_partial;
        }
        rc = timed_launch(p, ST_PREP, p->stream, prep);
        if (rc) return rc;
        return timed_launch(p, ST_SUM, p->stream, sum);
    } catch (...) {
        return fail(FEW_E_NOMEM, "exception in the summation call");
    }
}
}  // namespace

int32_t few_mode_sum(few_plan p, few_spline s, double theta, double phi, double scale,
                     double t_start, double dt, int64_t n, void *out) {
    return sum_impl(p, s, theta, phi, scale, t_start, dt, n, out, nullptr, nullptr);
}

int32_t few_mode_sum_ssb(few_plan p, few_spline s, double theta_s, double phi_s,
                         double theta_k, double phi_k, double scale, double t_start, double dt,
                         int64_t n, void *out) {
    double th, ph, rr, ri;
    if (detector_frame(theta_s, phi_s, theta_k, phi_k, &th, &ph, &rr, &ri) != FEW_OK)
        return fail(FEW_E_ARG, "non-finite sky or spin angle");
    if (!std::isfinite(scale)) return fail(FEW_E_ARG, "non-finite scale");
    return sum_impl(p, s, th, ph, scale * rr, t_start, dt, n, out, nullptr, nullptr,
                    scale * ri);
}

int32_t few_inner_product(few_plan p, few_spline s, double theta, double phi, double scale,
                          double t_start, double dt, int64_t n, const void *data,
                          double *out2) {
    if (!data) return fail(FEW_E_ARG, "null data pointer");
    return sum_impl(p, s, theta, phi, scale, t_start, dt, n, nullptr, data, out2);
}

int32_t few_inner_product_noalloc(few_plan p, few_spline s, double theta, double phi,
                                  double scale, double t_start, double dt, int64_t n,
                                  const void *data, double *out2) {
    if (!data) return fail(FEW_E_ARG, "null data pointer");
    return sum_impl(p, s, theta, phi, scale, t_start, dt, n, nullptr, data, out2, 0.0, true);
}

int32_t few_host_xcd_split_step(const double *w_prev, const double *times, double *w_next) {
    if (!w_prev || !times || !w_next) return fail(FEW_E_ARG, "null argument");
    for (int x = 0; x < 8; ++x)
        if (!(times[x] > 0.0) || !std::isfinite(times[x]) || !(w_prev[x] > 0.0) ||
            !std::isfinite(w_prev[x]))
            return fail(FEW_E_ARG, "times and weights must be finite and > 0");
    xcd_split_step(w_prev, times, w_next);
    return FEW_OK;
}

int32_t few_plan_timing(few_plan p, few_timing *out, int32_t reset) {
    if (!p || !out) return fail(FEW_E_ARG, "null argument");
    std::lock_guard<std::mutex> g(p->sync_mu);
    HIP_TRY(hipSetDevice(p->device));
    for (auto &t : p->timed) {
        HIP_TRY(hipEventSynchronize(t.second.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, t.second.first, t.second.second));
        p->acc_ms[t.first] += ms;
        p->acc_n[t.first] += 1;
        p->ev_pool.push_back(t.second.first);
        p->ev_pool.push_back(t.second.second);
    }
    p->timed.clear();
    out->spline_ms = p->acc_ms[ST_FIT];
    out->spline_launches = p->acc_n[ST_FIT];
    out->prepare_ms = p->acc_ms[ST_PREP];
    out->prepare_launches = p->acc_n[ST_PREP];
    out->sum_ms = p->acc_ms[ST_SUM];
    out->sum_launches = p->acc_n[ST_SUM];
    if (reset) {
        for (int i = 0; i < 3; ++i) {
            p->acc_ms[i] = 0;
            p->acc_n[i] = 0;
        }
        p->sum_launches = 0;        // FEW_FLAG_TIMING_SPARSE: the next launch is timed
    }
    return FEW_OK;
}

// ---------------------------------------------------------------------------
// Served path.
// ---------------------------------------------------------------------------
int32_t few_submit(few_plan p, const few_request *req, uint64_t *ticket) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    if (!req || !ticket) return fail(FEW_E_ARG, "null argument");
    try {
        int rc = validate_fit_args(req->n_knots, req->t_knots, req->n_modes, req->lmn,
                                   req->phi_phi, req->phi_r, req->amp, p->max_knots,
                                   p->max_modes);
        if (rc) return rc;
        rc = validate_sum_args(req->t_knots, req->n_knots, req->theta, req->phi, req->scale,
                               req->t_start, req->dt, req->n_samples, req->out);
        if (rc) return rc;
        ServedReq *r = new (std::nothrow) ServedReq;
        if (!r) return fail(FEW_E_NOMEM, "host allocation failed");
        r->r = *req;
        rc = make_host_req(req->n_knots, req->t_knots, req->n_modes, req->lmn, p->fp32, &r->h,
                           &p->layouts, 3, p->allow_mfma);
        if (rc) {
            delete r;
            return rc;
        }
        r->r.t_knots = r->h.t.data();
        r->r.lmn = nullptr;   // consumed into the term layout
        r->footprint = r->h.L.total + 3 * 256 + sizeof(FitJob) + sizeof(PrepJob) + sizeof(SumJob);
        // the arena also holds one 256-byte counter block per stream slot
        if (r->footprint + 256 * (size_t)p->max_inflight + 256 > p->budget) {
            size_t need = r->footprint;
            delete r;
            return fail(FEW_E_TOO_LARGE, "request needs %zu bytes, plan budget %llu", need,
                        (unsigned long long)p->budget);
        }
        auto reject = [&](int code, const char *what, hipError_t e) {
            if (r->ready) put_sync_event(p, r->ready);
            delete r;
            return fail(code, "%s%s%s", what, e != hipSuccess ? ": " : "",
                        e != hipSuccess ? hipGetErrorString(e) : "");
        };
        hipError_t he = hipSetDevice(p->device);
        if (he != hipSuccess) return reject(FEW_E_HIP, "hipSetDevice", he);
        // the request's batch waits for what the caller has enqueued on the plan
        // stream so far (its inputs may still be in production there)
        r->ready = sync_event(p);
        if (!r->ready) return reject(FEW_E_HIP, "event creation failed", hipSuccess);
        he = hipEventRecord(r->ready, p->stream);
        if (he != hipSuccess) return reject(FEW_E_HIP, "hipEventRecord", he);
        std::unique_lock<std::mutex> g(p->mu);
        if (p->stop) return reject(FEW_E_STATE, "plan is being destroyed", hipSuccess);
        if (!p->worker_started) {
            if (p->bstreams.empty()) {
                p->bstreams.assign(p->max_inflight, nullptr);
                for (int s = 0; s < p->max_inflight; ++s) {
                    he = hipStreamCreateWithFlags(&p->bstreams[s], hipStreamNonBlocking);
                    if (he != hipSuccess) {
                        for (int q = 0; q < s; ++q) hipStreamDestroy(p->bstreams[q]);
                        p->bstreams.clear();
                        return reject(FEW_E_HIP, "hipStreamCreateWithFlags", he);
                    }
                }
                p->slot_busy.assign(p->max_inflight, false);
            }
            p->worker = std::thread(scheduler_main, p);
            p->worker_started = true;
        }
        r->ticket = p->next_ticket++;
        r->t_arrive = plan_us(p);
        p->tickets[r->ticket] = r;
        p->pending.push_back(r);
        *ticket = r->ticket;
        g.unlock();
        p->cv_work.notify_one();
        return FEW_OK;
    } catch (...) {
        return fail(FEW_E_NOMEM, "exception in few_submit");
    }
}

int32_t few_poll(few_plan p, uint64_t ticket) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    std::lock_guard<std::mutex> g(p->mu);
    auto it = p->tickets.find(ticket);
    if (it == p->tickets.end()) return fail(FEW_E_STATE, "unknown or retired ticket");
    int st = it->second->status;
    if (st == FEW_PENDING) return FEW_PENDING;
    delete it->second;
    p->tickets.erase(it);
    if (st == FEW_E_NOMEM)
        return fail(st, "request not admitted: with nothing in flight the plan arena cannot "
                        "hold it (memory is held by synchronous-path splines or buffers)");
    if (st != FEW_OK) return fail(st, "request failed on the device path");
    return FEW_OK;
}

int32_t few_wait(few_plan p, uint64_t ticket) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    {
        std::unique_lock<std::mutex> g(p->mu);
        auto it = p->tickets.find(ticket);
        if (it == p->tickets.end()) return fail(FEW_E_STATE, "unknown or retired ticket");
        ServedReq *r = it->second;
        p->cv_done.wait(g, [&] { return r->status != FEW_PENDING; });
    }
    return few_poll(p, ticket);
}

int32_t few_mode_select(few_plan p, int32_t K, int32_t M, const double *amp, double eps,
                        int32_t *keep) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    if (!amp || !keep) return fail(FEW_E_ARG, "null pointer argument");
    if (K < 1) return fail(FEW_E_KNOTS, "K must be >= 1");
    if (M < 1 || M > kMaxSelectModes)
        return fail(FEW_E_MODES, "M = %d outside [1, %d]", M, kMaxSelectModes);
    if (!(eps >= 0.0 && eps < 1.0)) return fail(FEW_E_ARG, "eps must be in [0, 1)");
    std::lock_guard<std::mutex> g(p->sync_mu);
    HIP_TRY(hipSetDevice(p->device));
    HIP_TRY(launch_select(amp, K, M, eps, (p->flags & FEW_FLAG_SELECT_SORTED) != 0, keep,
                          p->stream));
    return FEW_OK;
}

int32_t few_batch(few_plan p, int32_t n, const few_request *reqs) {
    if (!p) return fail(FEW_E_STATE, "null plan");
    if (n < 1 || !reqs) return fail(FEW_E_ARG, "need n >= 1 requests");
    try {
        std::vector<std::unique_ptr<ServedReq>> own;
        std::vector<ServedReq *> list;
        for (int i = 0; i < n; ++i) {
            const few_request *q = &reqs[i];
            int rc = validate_fit_args(q->n_knots, q->t_knots, q->n_modes, q->lmn, q->phi_phi,
                                       q->phi_r, q->amp, p->max_knots, p->max_modes);
            if (!rc)
                rc = validate_sum_args(q->t_knots, q->n_knots, q->theta, q->phi, q->scale,
                                       q->t_start, q->dt, q->n_samples, q->out);
            if (rc) return rc;
            own.emplace_back(new ServedReq);
            ServedReq *r = own.back().get();
            r->r = *q;
            rc = make_host_req(q->n_knots, q->t_knots, q->n_modes, q->lmn, p->fp32, &r->h,
                               &p->layouts, 3, p->allow_mfma);
            if (rc) return rc;
            r->r.t_knots = r->h.t.data();
            list.push_back(r);
        }
        std::lock_guard<std::mutex> g(p->sync_mu);
        HIP_TRY(hipSetDevice(p->device));
        reap_deferred(p, false);
        const size_t bytes = batch_bytes(list);
        if (bytes > p->budget) return fail(FEW_E_TOO_LARGE, "batch needs %zu bytes", bytes);
        Batch b;
        b.slot = -1;
        b.reqs = list;
        b.arena_off = alloc_sync(p, bytes);
        if (b.arena_off == SIZE_MAX) return fail(FEW_E_NOMEM, "plan arena exhausted");
        int rc = launch_batch(p, &b, p->stream, p->sync_counter);
        if (rc != FEW_OK) {
            hipStreamSynchronize(p->stream);
            if (b.done) hipEventDestroy(b.done);
            p->arena.release(b.arena_off);
            if (b.pinned) p->pinned.put(b.pinned);
            return rc;
        }
        {
            std::lock_guard<std::mutex> dg(p->def_mu);
            p->deferred.push_back({b.arena_off, b.pinned, b.done});
        }
        return FEW_OK;
    } catch (...) {
        return fail(FEW_E_NOMEM, "exception in few_batch");
    }
}

}  // extern "C"

namespace {

// Build and launch one batch on stream slot `slot`.  Called without p->mu held.
int launch_batch(few_plan p, Batch *b, hipStream_t s, unsigned *counter) {
    const int n = (int)b->reqs.size();
    // served requests: order after the caller's work on the plan stream
    for (ServedReq *r : b->reqs)
        if (r->ready) HIP_TRY(hipStreamWaitEvent(s, r->ready, 0));
    // arena block: [FitJob[n] | PrepJob[n] | SumJob[n] | upload region of every
    // request | device-produced region of every request]; one copy stages the
    // job arrays and all upload regions
    size_t off_fit = 0;
    size_t off_prep = (off_fit + sizeof(FitJob) * n + 255) & ~(size_t)255;
    size_t off_sum = (off_prep + sizeof(PrepJob) * n + 255) & ~(size_t)255;
    size_t cur = (off_sum + sizeof(SumJob) * n + 255) & ~(size_t)255;
    std::vector<size_t> up_off(n), dev_off(n);
    for (int i = 0; i < n; ++i) {
        up_off[i] = cur;
        cur += (b->reqs[i]->h.L.dev_begin + 255) & ~(size_t)255;
    }
    const size_t upload_end = cur;
    for (int i = 0; i < n; ++i) {
        dev_off[i] = cur;
        const HostReq &h = b->reqs[i]->h;
        cur += (h.L.total - h.L.dev_begin + 255) & ~(size_t)255;
    }
    char *dev = p->arena.ptr(b->arena_off);
    b->pinned = p->pinned.get(upload_end);
    if (!b->pinned) return fail(FEW_E_NOMEM, "pinned staging allocation failed");
    char *host = (char *)b->pinned;
    FitJob *fj = (FitJob *)(host + off_fit);
    PrepJob *pj = (PrepJob *)(host + off_prep);
    SumJob *sj = (SumJob *)(host + off_sum);
    const bool fp32 = p->fp32;
    const int tile = tile_samples(fp32);
    if (n == 1) {
        // A batch of one request runs the single-request launches (sample
        // parts per XCD and short tiles at the end of each part), which drain
        // a long request better than the persistent batch grid; a sample gets
        // the same rounded operations either way.
        ServedReq *r = b->reqs[0];
        const ReqBase rb{dev + up_off[0], dev + dev_off[0]};
        stage_upload(r->h, host + up_off[0]);
        Tiling tl = single_tiling(fp32, r->h.n_ph == 3 ? p->resident_wg3 : p->resident_wg);
        tl.split = fp32 && tl.short_len > 0 && r->h.terms.n_terms >= kGroupMinTerms &&
                   r->h.terms.max_seg_terms <= kSplitTerms;
        const FitJob f = fit_job(r->h, rb, r->r.phi_phi, r->r.phi_r, r->r.amp);
        const PrepJob q = prep_job(r->h, rb, r->r.theta, r->r.phi, r->r.scale, r->r.t_start,
                                   r->r.dt, r->r.n_samples, fp32, tl);
        const SumJob u = sum_job(r->h, rb, r->r.t_start, r->r.dt, r->r.n_samples, r->r.out, tl);
        const long long slots = part_tile_bound(r->r.n_samples, tl.parts, tl.short_len, r->h.K,
                                                tile, q.short_tile);
        if (slots * tl.parts > 0x7fffffffLL) return fail(FEW_E_ARG, "too many samples");
        HIP_TRY(pinned_upload(dev, host, upload_end, s));
        HIP_TRY(launch_fit(f, r->h.t.data(), s));
        if (r->h.mfma) {
            SumJob ub = u;
            p->xsplit[(counter - p->counters) / 64].apply(&ub, p->mf_wg);   // this stream's
            HIP_TRY(launch_fold_pack(q, s));
            HIP_TRY(launch_sum_mfma(ub, p->mf_wg, s));
        } else {
            HIP_TRY(launch_prepare(q, fp32, s));
            HIP_TRY(launch_sum(u, (int)slots, fp32, s));
        }
        b->done = sync_event(p);
        if (!b->done) return fail(FEW_E_HIP, "event creation failed");
        HIP_TRY(hipEventRecord(b->done, s));
        return FEW_OK;
    }
    // vector-path jobs first in the prepare and sum job arrays, then the
    // matrix-core ones (each set has its own launches)
    int nv = 0;
    for (ServedReq *r : b->reqs) nv += r->h.mfma ? 0 : 1;
    int max_amp_blocks = 0, max_K = 4, max_fold_blocks = 0, max_K_mf = 4;
    long long waves = 0, mf_total = 0;
    int kv = 0, km = nv;
    for (int i = 0; i < n; ++i) {
        ServedReq *r = b->reqs[i];
        const ReqBase rb{dev + up_off[i], dev + dev_off[i]};
        stage_upload(r->h, host + up_off[i]);
        fj[i] = fit_job(r->h, rb, r->r.phi_phi, r->r.phi_r, r->r.amp);
        const int k = r->h.mfma ? km++ : kv++;
        pj[k] = prep_job(r->h, rb, r->r.theta, r->r.phi, r->r.scale, r->r.t_start, r->r.dt,
                         r->r.n_samples, fp32, Tiling{1, 0});
        sj[k] = sum_job(r->h, rb, r->r.t_start, r->r.dt, r->r.n_samples, r->r.out,
                        Tiling{1, 0});
        if (r->h.mfma) {
            sj[k].sample_base = mf_total;
            mf_total += r->r.n_samples;
            max_K_mf = std::max(max_K_mf, r->h.K);
        } else {
            sj[k].wave_base = (int)waves;
            waves += tile_upper_bound(r->r.n_samples, r->h.K, tile);
            max_fold_blocks = std::max(max_fold_blocks, pj[k].fold_blocks);
        }
        max_amp_blocks = std::max(max_amp_blocks, fj[i].amp_blocks);
        max_K = std::max(max_K, r->h.K);
    }
    if (waves > 0x3fffffff) return fail(FEW_E_ARG, "batch too large");
    const PrepJob *pd = (const PrepJob *)(dev + off_prep);
    const SumJob *sd = (const SumJob *)(dev + off_sum);
    HIP_TRY(pinned_upload(dev, host, upload_end, s));
    HIP_TRY(launch_fit_batch((const FitJob *)(dev + off_fit), n, max_amp_blocks, max_K, s));
    if (nv > 0) {
        HIP_TRY(launch_prepare_batch(pd, nv, max_fold_blocks, fp32, s));
        HIP_TRY(launch_sum_batch(sd, nv, (int)waves, fp32, true, counter, s));
    }
    if (nv < n) {
        HIP_TRY(launch_fold_pack_batch(pd + nv, n - nv, max_K_mf, s));
        HIP_TRY(launch_sum_mfma_batch(sd + nv, n - nv, mf_total, p->mf_wg, s));
    }
    b->done = sync_event(p);
    if (!b->done) return fail(FEW_E_HIP, "event creation failed");
    HIP_TRY(hipEventRecord(b->done, s));
    return FEW_OK;
}

size_t batch_bytes(const std::vector<ServedReq *> &reqs) {
    size_t n = reqs.size();
    size_t cur = 0;
    cur = (cur + sizeof(FitJob) * n + 255) & ~(size_t)255;
    cur = (cur + sizeof(PrepJob) * n + 255) & ~(size_t)255;
    cur = (cur + sizeof(SumJob) * n + 255) & ~(size_t)255;
    for (ServedReq *r : reqs) {
        cur += (r->h.L.dev_begin + 255) & ~(size_t)255;
        cur += (r->h.L.total - r->h.L.dev_begin + 255) & ~(size_t)255;
    }
    return cur;
}

void scheduler_main(few_plan p) {
    hipSetDevice(p->device);
    std::unique_lock<std::mutex> g(p->mu);
    for (;;) {
        // retire finished batches
        bool retired = false;
        for (size_t i = 0; i < p->inflight.size();) {
            Batch *b = p->inflight[i];
            hipError_t q = hipEventQuery(b->done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            int st = (q == hipSuccess) ? FEW_OK : FEW_E_HIP;
            const double t_done = plan_us(p);
            for (ServedReq *r : b->reqs) {
                r->status = st;
                put_sync_event(p, r->ready);
                r->ready = nullptr;
                log_request(p, r, t_done);
            }
            if (p->log) std::fflush(p->log);
            p->arena.release(b->arena_off);
            p->pinned.put(b->pinned);
            put_sync_event(p, b->done);
            p->slot_busy[b->slot] = false;
            delete b;
            p->inflight.erase(p->inflight.begin() + i);
            retired = true;
        }
        if (retired) p->cv_done.notify_all();
        // admit: arrival order, as many as fit the arena, one free stream slot
        int slot = -1;
        for (int s = 0; s < p->max_inflight; ++s)
            if (!p->slot_busy[s]) {
                slot = s;
                break;
            }
        if (slot >= 0 && !p->pending.empty()) {
            std::vector<ServedReq *> take;
            size_t off = SIZE_MAX;
            for (ServedReq *r : p->pending) {
                take.push_back(r);
                if (take.size() > 256) {
                    take.pop_back();
                    break;
                }
            }
            // blocks freed by completed plan-stream work (freed splines,
            // few_batch blocks) return to the arena first
            reap_deferred(p, false);
            while (!take.empty()) {
                off = p->arena.alloc(batch_bytes(take));
                if (off != SIZE_MAX) break;
                take.pop_back();
            }
            if (off == SIZE_MAX && p->inflight.empty()) {
                // Nothing of this plan runs that could free memory: if no
                // deferred release is outstanding either, the head request
                // cannot be admitted until the caller frees memory held by
                // the synchronous path, so fail it rather than wait forever.
                if (reap_deferred(p, false) == 0 &&
                    p->arena.alloc_probe(batch_bytes({p->pending.front()})) == false) {
                    ServedReq *r = p->pending.front();
                    p->pending.pop_front();
                    r->status = FEW_E_NOMEM;
                    put_sync_event(p, r->ready);
                    r->ready = nullptr;
                    log_request(p, r, plan_us(p));
                    if (p->log) std::fflush(p->log);
                    p->cv_done.notify_all();
                    continue;
                }
            }
            if (off != SIZE_MAX && !take.empty()) {
                for (size_t i = 0; i < take.size(); ++i) p->pending.pop_front();
                Batch *b = new Batch;
                b->slot = slot;
                b->arena_off = off;
                b->reqs = take;
                const double t_admit = plan_us(p);
                for (ServedReq *r : take) {
                    r->t_admit = t_admit;
                    r->batch = p->n_batches;
                    r->batch_size = (int)take.size();
                }
                ++p->n_batches;
                p->slot_busy[slot] = true;
                g.unlock();
                int rc = launch_batch(p, b, p->bstreams[slot], p->counters + 64 * slot);
                g.lock();
                if (rc != FEW_OK) {
                    if (b->done) {
                        hipEventSynchronize(b->done);
                        put_sync_event(p, b->done);
                    } else {
                        hipStreamSynchronize(p->bstreams[slot]);
                    }
                    const double t_done = plan_us(p);
                    for (ServedReq *r : b->reqs) {
                        r->status = rc;
                        put_sync_event(p, r->ready);
                        r->ready = nullptr;
                        log_request(p, r, t_done);
                    }
                    if (p->log) std::fflush(p->log);
                    p->arena.release(b->arena_off);
                    if (b->pinned) p->pinned.put(b->pinned);
                    p->slot_busy[slot] = false;
                    delete b;
                    p->cv_done.notify_all();
                } else {
                    p->inflight.push_back(b);
                }
                continue;
            }
        }
        if (p->stop && p->pending.empty() && p->inflight.empty()) break;
        if (p->inflight.empty() && p->pending.empty()) {
            p->cv_work.wait(g, [&] { return p->stop || !p->pending.empty(); });
        } else if (!p->inflight.empty()) {
            // batches in flight: their completion is polled back to back (a
            // timed wait sleeps ~60 us, which a request's latency would carry)
            g.unlock();
            std::this_thread::yield();
            g.lock();
        } else {
            p->cv_work.wait_for(g, std::chrono::microseconds(50));
        }
    }
}

}  // namespace
