// C-ABI layer: argument checks, workspace, stream ordering of the search stages.
//
// The staging follows Algorithms 2 and 3 (Lemire, arXiv:0811.3301, Sec. 7 and Sec. 8): envelope
// of the query, LB_Keogh of every candidate, LB_Improved of the survivors (Algorithm 3 only),
// DTW of what remains against the best-so-far.  The sequential scan's threshold b, which
// starts at infinity and shrinks in database order, is replaced by a seeded threshold: the
// DTW of the candidates with the smallest LB_Keogh, computed first.
#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace lbimp;
using u64 = unsigned long long;

static thread_local std::string g_err;

// Fixed device scratch of lbimp_nn_search_noalloc.  The library's code object holds one copy
// per GPU it is loaded on, kept until the process ends.  In host code the array's name is not
// a device address: the address of each GPU's copy is looked up once per device when a
// context is created there, and only that address is used afterwards.
static __device__ __align__(256) unsigned char scratch[LBIMP_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPTRY(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(LBIMP_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr int kStages = 8;
constexpr int kMaxSeeds = 64;
constexpr int kPoolStreams = 4;  // concurrent groups of a ragged batch
constexpr int kTuneKnobs = LBIMP_TUNE_KNOBS;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Two-pass carving of one workspace allocation: measure with base == nullptr, then assign.
struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Pinned host buffer for an upload; `ev` marks the end of the last copy that read it.
struct PinnedChunk {
    void *ptr = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
};
constexpr size_t kPinnedRing = 8;

// Batches that share a tuning choice: database shape, band, p, k, mode, Q up to a power of 2.
struct TuneKey {
    int64_t N;
    int n, wb, p, k, mode, qb;
    bool operator<(const TuneKey &o) const {
        return std::tie(N, n, wb, p, k, mode, qb) < std::tie(o.N, o.n, o.wb, o.p, o.k, o.mode, o.qb);
    }
};

int pow2_at_least(int64_t v) {
    int b = 1;
    while (b < v && b < (1 << 30)) b <<= 1;
    return b;
}

}  // namespace

struct lbimp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    void *ws = nullptr;
    size_t ws_cap = 0;
    bool timing = false;
    bool timed_valid = false;
    int seeds = 32;             // option "seeds"
    int lbi_pipeline = 1;       // option "lbi_pipeline"
    bool dtw_low_latency = false;  // option "dtw_group_per_pair" (lbimp_dtw_band only)
    int sweep_shape = 0;           // option "sweep_shape"
    bool use_graph = true;         // option "graph" (lbimp_nn_search_ragged)
    int ragged_streams = kPoolStreams;  // option "ragged_streams"
    int pd_prefilter = 0;               // option "pd_prefilter" (0, 1 or 2)
    bool pd_fine_bound = false;         // option "pd_fine": lbimp_db_pd_bound on the 32-part cover
    bool lbi_abandon = false;           // option "lbi_abandon"
    bool lbi_buckets = false;           // option "lbi_buckets"
    bool dtw_split = false;             // option "dtw_split"
    int64_t dtw_pool_slots = 1 << 18;   // option "dtw_pool_slots"
    size_t ws_limit = 0;                // option "workspace_limit" (bytes, 0: none)
    // ragged batches: stream pool, captured graph, pinned staging of the grouping metadata
    hipStream_t graph_stream = nullptr;
    hipStream_t pool[kPoolStreams] = {};
    hipEvent_t join_ev[kPoolStreams] = {};
    hipEvent_t fork_ev = nullptr, enter_ev = nullptr, exit_ev = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_sig = 0;
    std::vector<PinnedChunk> pinned;  // ring of staging buffers, each reusable once its upload ran
    bool autotune = false;            // option "autotune"
    std::map<TuneKey, std::array<int, kTuneKnobs>> tuned;  // in the order of LBIMP_TUNE_KNOBS
    hipEvent_t tev[2] = {};
    hipEvent_t ev[kStages + 1] = {};
};

struct lbimp_db {
    int device = 0;
    int64_t N = 0;
    int n = 0;
    float *rows = nullptr;  // [N][n] row-major copy (gathers of the second pass and the DTW)
    float4 *il = nullptr;   // interleaved tiles for the LB_Keogh sweep
    double *pd = nullptr;   // [N][kPdParts] piecewise sums (Sec. 9) of the pass-0 scan
    float4 *pdf = nullptr;  // sums over the 32-part cover, interleaved by 64-candidate tile (n >= kPdfMinN)
};

static int persistent_grid(const lbimp_ctx *ctx) { return std::max(1, ctx->num_cu); }  // CUs; kernels size by occupancy

// Workspace allocated for a request of `bytes` (headroom so that slightly larger calls reuse it).
static size_t reserve_size(size_t bytes) { return align_up(bytes + bytes / 8, 1 << 20); }

static int reserve(lbimp_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_cap) return LBIMP_OK;
    HIPTRY(hipStreamSynchronize(ctx->stream));
    if (ctx->graph_stream) HIPTRY(hipStreamSynchronize(ctx->graph_stream));
    if (ctx->ws) HIPTRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
    size_t cap = reserve_size(bytes);
    if (hipMalloc(&ctx->ws, cap) != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws = nullptr;
        return fail(LBIMP_E_NOMEM, "workspace allocation of %zu bytes failed", cap);
    }
    ctx->ws_cap = cap;
    return LBIMP_OK;
}

// Address of this device's copy of `scratch` (the device must be current).
static int init_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(LBIMP_E_UNSUPPORTED, "device %d: at most %d devices", device,
                                                         kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return LBIMP_OK;
    void *ptr = nullptr;
    HIPTRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(LBIMP_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = ptr;
    return LBIMP_OK;
}

static int check_ctx(lbimp_ctx *ctx) {
    if (!ctx) return fail(LBIMP_E_INVALID, "null context");
    HIPTRY(hipSetDevice(ctx->device));
    return LBIMP_OK;
}

static int check_shape(int64_t count, int32_t n, int32_t w, int32_t p) {
    if (count < 0) return fail(LBIMP_E_INVALID, "negative count");
    if (n < 1 || n > LBIMP_MAX_LEN) return fail(LBIMP_E_INVALID, "series length %d outside [1, %d]", n, LBIMP_MAX_LEN);
    if (w < 0) return fail(LBIMP_E_INVALID, "locality constraint w = %d < 0", w);
    if (p < 1) return fail(LBIMP_E_INVALID, "exponent p = %d < 1", p);
    if (p > 2 && p != LBIMP_P_INF)
        return fail(LBIMP_E_UNSUPPORTED, "exponent p = %d: p = 1, p = 2 and p = infinity are implemented", p);
    if (count > INT32_MAX) return fail(LBIMP_E_INVALID, "more than 2^31-1 series");
    return LBIMP_OK;
}

static int band_of(int32_t n, int32_t w) { return std::min<int32_t>(w, n - 1); }

static void stage_mark(lbimp_ctx *ctx, int i) {
    if (ctx->timing) (void)hipEventRecord(ctx->ev[i], ctx->stream);
}

// ------------------------------------------------------------------ one homogeneous search
namespace {

// Choices that change speed, never results.
struct Knobs {
    int seeds;          // seeding DTWs (at least k are used)
    int lbi_pipeline;   // blocks loaded ahead by the register LB_Improved kernel (0 or 1)
    int sweep_shape;    // tiling of the LB_Keogh sweep
    bool dtw_group;     // survivors' DTW with a group of lanes per pair (else a lane per pair)
    bool seed_lane;     // seeding DTWs with a lane per pair (else a group of lanes per pair)
    bool cascade;       // abandon on the row minimum plus the LB_Keogh terms still to come
    int pd = 0;         // pass 0: piecewise-sum bound of every candidate; 1: 8-part cover, LB_Keogh only of
                        // its survivors; 2: 32-part cover, LB_Keogh inside the LB_Improved pass
    bool lbi_abandon = false;  // early abandoning inside the LB_Improved pass
    bool lbi_buckets = false;  // LB_Improved over bucketed survivor lists (XCD-local row reuse)
    bool dtw_split = false;    // survivors' DTW in two row phases, the pairs still running repacked between
};

struct SearchSpec {  // Q queries of one length against one database
    const lbimp_db *db;
    const float *queries;  // device [Q][n]
    int64_t Q;
    int w, p, k, mode;
    int64_t *idx;          // device outputs, row q (or qmap[q]) of [*][k]
    float *dist;
    const int64_t *qmap;   // device [Q] output rows, or nullptr for the identity
    Knobs kn;
    const int64_t *kq = nullptr;  // device [Q] per-query k (each <= k), or nullptr: k for every query
    int ldo = 0;                  // output row stride in entries (0: k)
    size_t ws_limit = 0;          // workspace bound in bytes (0: none); the candidates are split into chunks to meet it
    int64_t pool_slots = 1 << 18; // bound on the row-phase DTW's parked-pair slots
};

struct SearchDims {
    int n, n4, ldq, wb, qg, S, WL, k, p;
    int64_t N, Np, Q, Qp, ldres, nw;
    int64_t C, nchunks;  // candidates per chunk (a multiple of kChunkAlign unless the whole database) and chunk count
    int64_t bs;          // candidates per bucket of the LB_Improved survivor lists
    int nb;              // buckets per chunk (1: the lists are not bucketed)
    size_t ring_bytes;  // strip-boundary scratch of the wide-band DTW
    bool brute, improved, from_minima, pd;
    bool fine;           // pass 0 on the 32-part cover, then LB_Improved with LB_Keogh fused (pd = 2)
    bool split;          // survivors' DTW in two row phases (lane-per-pair kernel)
    int split_row;       // first row of the second phase
    int64_t pool_cap;    // parked-pair slots of the phases' pool
};

struct SearchBufs {
    float *Ue, *Le, *S1, *ring;
    int *seeds, *list0, *list1, *list2, *counters, *cntb;
    u64 *best, *thr, *res, *wmin;
    long long *prefix, *tot;
    double *qpd;
    float *qpf;
    float *pool;   // parked pairs of the row-phase DTW ([wb*2 + 3][pool_cap])
    int *parkcnt;  // [Q] parked pairs per query, then the pool's slot counter
};

constexpr int64_t kChunkAlign = 2048;  // chunk sizes are multiples of the sweep's largest tile group

// Sizes of a search over the candidates split into chunks of C (C = N: one chunk).
static void chunk_dims(const SearchSpec &sp, int64_t C, SearchDims &d) {
    d.C = std::max<int64_t>(std::min(C, d.N), 1);
    d.nchunks = d.N ? (d.N + d.C - 1) / d.C : 1;
    d.Np = (d.C + 63) / 64 * 64;  // row stride of the first-pass bounds of one chunk
    d.S = d.brute ? 0 : (int)std::min<int64_t>(std::max(sp.kn.seeds, sp.k), d.C);
    // result keys: the k kept from earlier chunks, then the seeds' and the survivors' of a chunk
    d.ldres = d.brute ? std::max<int64_t>(d.C, 1) + (d.nchunks > 1 ? d.k : 0) : d.S + d.C + (d.nchunks > 1 ? d.k : 0);
    d.nw = d.fine ? pdf_scan_waves(d.C) : d.pd ? pd_scan_waves(d.C) : sweep_waves(sp.kn.sweep_shape, d.C, sp.Q);
    // seeds come from the per-wave minima of the sweep once there are enough of them
    d.from_minima = !d.brute && d.nw >= 4 * (int64_t)kMaxSeeds;
    // LB_Improved survivors bucketed by candidate range: about 2 MiB of rows per bucket, so that
    // one bucket's rows stay in an XCD's L2 while the pairs of every query read them
    const int64_t span = compact_wave_span();
    d.bs = std::max<int64_t>(span, ((int64_t)(2 << 20) / (4 * (int64_t)d.n)) / span * span);
    d.nb = (d.improved && sp.kn.lbi_buckets && d.C > d.bs) ? (int)((d.C + d.bs - 1) / d.bs) : 1;
    // row phases: the second starts at half the series (a multiple of the kernel's row group);
    // the pool holds up to a quarter of the chunk's pairs, at most the context's bound
    const int lr = lane_rows(d.wb);
    d.split_row = d.n / 2 / lr * lr;
    d.pool_cap = std::min<int64_t>(sp.pool_slots, d.Q * d.C / 4);
    if (sp.ws_limit)  // at most an eighth of a workspace bound
        d.pool_cap = std::min<int64_t>(d.pool_cap, (int64_t)(sp.ws_limit / 8 / (sizeof(float) * (2 * d.wb + 3))));
    d.split = sp.kn.dtw_split && d.improved && !sp.kn.dtw_group && d.wb <= kLaneMaxW && d.split_row >= lr &&
              d.split_row < d.n - d.n % lr && d.pool_cap >= 64;
}

void layout(Carver &c, const SearchDims &d, SearchBufs &b);

// pass 0 on the 32-part cover needs the database's fine sums and the register LB_Improved kernel
// (which computes LB_Keogh itself in that flow)
bool fine_supported(const lbimp_db *db, bool improved, int wb) {
    return improved && db->pdf != nullptr && wb <= kLbiRegMaxW;
}

int dims_of(const SearchSpec &sp, int num_cu, SearchDims &d) {
    d.n = sp.db->n;
    d.n4 = (d.n + 3) / 4;
    d.ldq = d.n4 * 4;
    d.N = sp.db->N;
    d.Q = sp.Q;
    d.k = sp.k;
    d.p = sp.p;
    d.wb = band_of(d.n, sp.w);
    d.qg = sweep_query_group(sp.kn.sweep_shape, sp.Q);
    d.Qp = (sp.Q + d.qg - 1) / d.qg * d.qg;
    d.brute = sp.mode == LBIMP_MODE_BRUTE;
    d.improved = sp.mode == LBIMP_MODE_IMPROVED;
    d.WL = d.improved ? lbi_batch(d.n, d.wb) : 1;
    if (d.improved && d.WL == 0)
        return fail(LBIMP_E_UNSUPPORTED, "LB_Improved state for n = %d, w = %d exceeds LDS", d.n, d.wb);
    d.pd = sp.kn.pd != 0 && !d.brute;
    d.fine = d.pd && sp.kn.pd == 2 && fine_supported(sp.db, d.improved, d.wb);  // else the 8-part cover
    d.ring_bytes = dtw_strip_scratch(d.p, d.n, d.wb, num_cu);
    chunk_dims(sp, d.N, d);
    if (sp.ws_limit && d.N > kChunkAlign) {
        // halve the chunk until the workspace fits the bound (or the chunk is one tile group)
        auto bytes = [&]() {
            Carver cv{nullptr};
            SearchBufs b;
            layout(cv, d, b);
            return cv.off;
        };
        int64_t C = d.N;
        while (bytes() > sp.ws_limit && C > kChunkAlign) {
            C = std::max<int64_t>(kChunkAlign, (C / 2 + kChunkAlign - 1) / kChunkAlign * kChunkAlign);
            chunk_dims(sp, C, d);
        }
    }
    return LBIMP_OK;
}

void layout(Carver &c, const SearchDims &d, SearchBufs &b) {
    const bool any = d.N > 0;
    b.Ue = c.take<float>((size_t)d.Qp * d.ldq);
    b.Le = c.take<float>((size_t)d.Qp * d.ldq);
    b.S1 = (d.brute || !any) ? nullptr : c.take<float>((size_t)d.Q * d.Np);
    b.seeds = (d.brute || !any) ? nullptr : c.take<int>((size_t)d.Q * std::max(d.S, 1));
    b.best = c.take<u64>((size_t)d.Q);
    b.thr = c.take<u64>((size_t)d.Q);
    // k-NN result keys (kept sorted between chunks); for k = 1 the best key is enough
    b.res = (d.k > 1 || !any) ? c.take<u64>((size_t)d.Q * d.ldres) : nullptr;
    b.list0 = (d.pd && !d.fine && any) ? c.take<int>((size_t)d.Q * d.C) : nullptr;
    b.qpd = (d.pd && !d.fine && any) ? c.take<double>((size_t)d.Q * 2 * kPdParts) : nullptr;
    b.qpf = (d.fine && any) ? c.take<float>((size_t)d.Q * kPdfQuery) : nullptr;
    b.pool = (d.split && any) ? c.take<float>((size_t)(2 * d.wb + 3) * d.pool_cap) : nullptr;
    b.parkcnt = (d.split && any) ? c.take<int>((size_t)d.Q + 1) : nullptr;
    b.list1 = (d.brute || !any) ? nullptr : c.take<int>((size_t)d.Q * d.C);
    b.list2 = (d.improved && any) ? c.take<int>((size_t)d.Q * d.C) : nullptr;
    b.counters = c.take<int>((size_t)d.Q * kCounters);  // cnt1, cnt2, rescnt, abandoned, cnt0 ([kCounters][Q])
    b.cntb = (d.nb > 1 && any) ? c.take<int>((size_t)d.Q * d.nb) : nullptr;  // bucketed pass-1 counts [nb][Q]
    b.tot = d.nchunks > 1 ? c.take<long long>((size_t)d.Q * 3) : nullptr;  // cnt1, cnt2, cnt0 over all chunks
    b.prefix = c.take<long long>((size_t)d.Q * d.nb + 1);
    b.wmin = (d.from_minima && any) ? c.take<u64>((size_t)d.Q * d.nw) : nullptr;
    b.ring = (d.ring_bytes && any) ? c.take<float>(d.ring_bytes / sizeof(float)) : nullptr;
}

// Seeds of a whole search: min(S, C_j) per chunk j.
int64_t seeds_total(const SearchDims &d) {
    if (d.brute || d.N == 0) return 0;
    int64_t t = 0;
    for (int64_t c0 = 0; c0 < d.N; c0 += d.C) t += std::min<int64_t>(d.S, d.N - c0);
    return t;
}

// h: the counters [kCounters][Q]; tot: [3][Q] totals of cnt1, cnt2, cnt0 over chunks, or null.
void fill_stats(const SearchDims &d, int64_t Q, const int *h, const long long *tot, const int64_t *ids,
                lbimp_stats *out) {
    const int64_t S = seeds_total(d);
    for (int64_t q = 0; q < Q; ++q) {
        lbimp_stats &st = out[ids ? ids[q] : q];
        st.candidates = d.N;
        st.seeded = S;
        st.dtw_abandoned = d.brute ? 0 : h[3 * Q + q];
        if (d.N == 0) {
            st = lbimp_stats{0, 0, 0, 0, 0, 0, 0};
        } else if (d.brute) {
            st.pruned_pd = st.pruned_keogh = st.pruned_improved = 0;
            st.dtw_started = d.N;
        } else {
            const int64_t c1 = tot ? tot[q] : h[q];
            const int64_t c2 = d.improved ? (tot ? tot[Q + q] : h[Q + q]) : c1;
            const int64_t c0 = d.pd ? (tot ? tot[2 * Q + q] : h[4 * Q + q]) : d.N - S;  // pass-0 survivors
            st.pruned_pd = d.N - S - c0;
            st.pruned_keogh = c0 - c1;
            st.pruned_improved = c1 - c2;
            st.dtw_started = S + c2;
        }
    }
}

}  // namespace

// Enqueue the whole path of one search on stream s (Algorithms 2 and 3 with a seeded threshold).
static int enqueue_search(lbimp_ctx *ctx, const SearchSpec &sp, const SearchDims &d, const SearchBufs &b,
                          hipStream_t s, bool mark) {
    auto stage = [&](int i) {
        if (mark) stage_mark(ctx, i);
    };
    const int64_t Q = d.Q, N = d.N;
    const int n = d.n, wb = d.wb, p = d.p, k = d.k;
    const int ldo = sp.ldo ? sp.ldo : k;
    int *cnt1 = b.counters, *cnt2 = b.counters + Q, *rescnt = b.counters + 2 * Q, *abandoned = b.counters + 3 * Q,
        *cnt0 = b.counters + 4 * Q;
    if (N == 0) {  // nothing to search: every slot is empty
        HIPTRY(launch_fill_i32(b.counters, 0, Q * kCounters, s));
        for (int i = 0; i <= 7; ++i) stage(i);
        HIPTRY(launch_finalize_k(b.res, 1, rescnt, Q, k, sp.kq, ldo, p, sp.idx, sp.dist, sp.qmap, s));
        stage(8);
        return LBIMP_OK;
    }
    const int grid = persistent_grid(ctx);  // compute units: each persistent kernel sizes its grid by occupancy
    const u64 *T = k == 1 ? b.best : b.thr;  // pruning threshold keys of the two passes
    QueryData qd{sp.queries, n, b.Ue, b.Le, d.ldq};
    const lbimp_db *db = sp.db;

    stage(0);
    // the envelope kernel also resets the best-so-far and threshold keys and the counters of the
    // Q queries
    HIPTRY(launch_envelope(sp.queries, Q, d.Qp, n, wb, b.Ue, b.Le, d.ldq, s, b.best, b.thr, b.counters));
    stage(1);
    const bool chunked = d.nchunks > 1;
    if (chunked) HIPTRY(launch_fill_u64(reinterpret_cast<u64 *>(b.tot), 0, Q * 3, s));
    if (d.fine)
        HIPTRY(launch_pdf_query(b.Ue, b.Le, d.ldq, Q, n, b.qpf, s));
    else if (d.pd)
        HIPTRY(launch_pd_query(b.Ue, b.Le, d.ldq, Q, n, b.qpd, s));
    // The candidates are searched in chunks [c0, c0 + cj), each through the whole path; the
    // threshold carries over (the best key for k = 1, the k best keys for k > 1), so every chunk
    // prunes at least as well as the first.  Candidate indices stay global: the chunk's
    // first-pass bounds are addressed through a base shifted back by c0.
    for (int64_t c0 = 0; c0 < N; c0 += d.C) {
        const int64_t cj = std::min(d.C, N - c0), c1 = c0 + cj;
        const bool first = c0 == 0;
        auto stage_first = [&](int i) {
            if (first) stage(i);
        };
        if (d.brute) {
            for (int i = 2; i <= 6; ++i) stage_first(i);
            PairList all{nullptr, 0, nullptr, cj, c0};
            HIPTRY(launch_dtw(p, db->rows, n, wb, qd, all, b.prefix, Q, nullptr, grid, k == 1 ? b.best : nullptr,
                              k == 1 ? nullptr : b.thr, b.res, d.ldres, rescnt, nullptr, nullptr, false, false,
                              b.ring, d.ring_bytes, nullptr, 0, s));
        } else {
            float *S1v = b.S1 - c0;  // S1v[q * Np + c] is candidate c of this chunk
            if (d.fine) {
                // pass 0 on the 32-part cover, fp32, 128 bytes per candidate (the chunk starts at a
                // multiple of 64 candidates, a tile of the interleaved sums)
                HIPTRY(launch_pdf_scan(p, db->pdf + (c0 / 64) * (kPdFine / 4) * 64, cj, n, b.qpf, Q, b.S1, d.Np,
                                       false, b.wmin, s, c0));
            } else if (d.pd) {
                // pass 0: the piecewise-sum bound (Sec. 9) of every candidate, 64 bytes per candidate
                HIPTRY(launch_pd_scan(p, db->pd + c0 * kPdParts, cj, n, b.qpd, Q, b.S1, d.Np, false, false,
                                      b.wmin, s, c0));
            } else {
                // pass 1: LB_Keogh of every candidate (Algorithm 2/3, first bound)
                HIPTRY(launch_lbk_sweep(p, sp.kn.sweep_shape, db->il + (c0 / 64) * d.n4 * 64, cj, d.n4,
                                        reinterpret_cast<float4 *>(b.Ue), reinterpret_cast<float4 *>(b.Le), d.n4, Q,
                                        b.S1, d.Np, false, false, b.wmin, s, c0));
            }
            stage_first(2);
            const int Sj = (int)std::min<int64_t>(d.S, cj);
            const int64_t nwj =
                d.fine ? pdf_scan_waves(cj) : d.pd ? pd_scan_waves(cj) : sweep_waves(sp.kn.sweep_shape, cj, Q);
            const bool minima = d.from_minima && nwj >= 4 * (int64_t)kMaxSeeds;
            HIPTRY(launch_select_seeds(S1v, d.Np, c1, Q, Sj, minima ? b.wmin : nullptr, nwj, b.seeds, s, c0));
            stage_first(3);
            // Seeds: few pairs per query on the critical path, so a group of lanes per pair (low
            // latency); they run to completion, their DTWs finishing together.
            const bool seed_ll = !sp.kn.seed_lane;
            PairList seedl{b.seeds, Sj, nullptr, Sj};
            HIPTRY(launch_dtw(p, db->rows, n, wb, qd, seedl, b.prefix, Q, nullptr, grid, k == 1 ? b.best : nullptr,
                              k == 1 ? nullptr : b.thr, b.res, d.ldres, rescnt, abandoned, nullptr, false, seed_ll,
                              b.ring, d.ring_bytes, nullptr, 0, s));
            if (k > 1) HIPTRY(launch_kth_key(b.res, d.ldres, rescnt, Q, k, sp.kq, b.thr, s));
            stage_first(4);
            PairList dl{b.list1, d.C, cnt1, 0};
            if (d.fine) {
                // the pass-0 survivors go straight to LB_Improved, which computes their LB_Keogh
                // (pass 1) from the same read of each row: cnt0 counts the pass-0 survivors, cnt1
                // those whose LB_Keogh stays below the threshold, cnt2 those of LB_Improved
                PairList l0{b.list1, d.C, cnt0, 0};
                if (d.nb > 1) {  // bucketed by candidate range (XCD-local row reuse in LB_Improved)
                    HIPTRY(launch_fill_i32(b.cntb, 0, Q * d.nb, s));
                    HIPTRY(launch_compact(S1v, d.Np, c1, Q, T, b.list1, d.C, cnt0, s, c0, d.bs, b.cntb));
                    l0 = PairList{b.list1, d.C, b.cntb, 0, 0, d.nb, d.bs, Q};
                } else {
                    HIPTRY(launch_compact(S1v, d.Np, c1, Q, T, b.list1, d.C, cnt0, s, c0));
                }
                stage_first(5);
                HIPTRY(launch_items_prefix(l0.cnt, 0, Q * d.nb, d.WL, b.prefix, s));
                HIPTRY(launch_lbi(p, db->rows, (int64_t)N * n * 4, n, wb, qd, l0, S1v, d.Np, b.prefix, Q, nullptr,
                                  grid, T, b.list2, d.C, cnt2, nullptr, 1, false, s, true, cnt1, S1v));
                dl = PairList{b.list2, d.C, cnt2, 0};
            } else {
                if (d.pd) {
                    // the pass-0 survivors, then LB_Keogh of their rows (pass 1) over their S1 entries;
                    // the others keep their pass-0 bound, at or above the threshold
                    HIPTRY(launch_compact(S1v, d.Np, c1, Q, T, b.list0, d.C, cnt0, s, c0));
                    HIPTRY(launch_items_prefix(cnt0, 0, Q, lbk_gather_batch(), b.prefix, s));
                    HIPTRY(launch_lbk_gather(p, db->rows, n, qd, PairList{b.list0, d.C, cnt0, 0}, b.prefix, Q, grid,
                                             S1v, d.Np, s));
                }
                if (d.nb > 1) {  // survivors bucketed by candidate range for the LB_Improved pass
                    HIPTRY(launch_fill_i32(b.cntb, 0, Q * d.nb, s));
                    HIPTRY(launch_compact(S1v, d.Np, c1, Q, T, b.list1, d.C, cnt1, s, c0, d.bs, b.cntb));
                } else {
                    HIPTRY(launch_compact(S1v, d.Np, c1, Q, T, b.list1, d.C, cnt1, s, c0));
                }
                stage_first(5);
                if (d.improved) {  // pass 2: LB_Improved of the survivors (Algorithm 3)
                    if (d.nb > 1) {
                        dl = PairList{b.list1, d.C, b.cntb, 0, 0, d.nb, d.bs, Q};
                        HIPTRY(launch_items_prefix(b.cntb, 0, Q * d.nb, d.WL, b.prefix, s));
                    } else {
                        HIPTRY(launch_items_prefix(cnt1, 0, Q, d.WL, b.prefix, s));
                    }
                    HIPTRY(launch_lbi(p, db->rows, (int64_t)N * n * 4, n, wb, qd, dl, S1v, d.Np, b.prefix, Q, nullptr,
                                      grid, T, b.list2, d.C, cnt2, nullptr, sp.kn.lbi_pipeline, sp.kn.lbi_abandon, s));
                    dl = PairList{b.list2, d.C, cnt2, 0};
                }
            }
            stage_first(6);
            const bool dtw_ll = sp.kn.dtw_group && (wb <= kLaneMaxW || dtw_wavereg_wide_supported(n, wb));
            HIPTRY(launch_items_prefix(dl.cnt, 0, Q, dtw_batch(n, wb, dtw_ll), b.prefix, s));
            if (d.split) {
                // rows [0, R) of every survivor, parking the pairs still running in the pool (their
                // slots listed per query in list1, free once LB_Improved has read it); then rows
                // [R, n) of the parked pairs, repacked 64 to a wave
                HIPTRY(launch_fill_i32(b.parkcnt, 0, Q + 1, s));
                const DtwPhase ph0{0, d.split_row, false, b.pool, d.pool_cap, b.parkcnt + Q, b.list1, d.C, b.parkcnt};
                HIPTRY(launch_dtw(p, db->rows, n, wb, qd, dl, b.prefix, Q, nullptr, grid, k == 1 ? b.best : nullptr,
                                  k == 1 ? nullptr : b.thr, b.res, d.ldres, rescnt, abandoned, nullptr, true, false,
                                  b.ring, d.ring_bytes, sp.kn.cascade ? S1v : nullptr, d.Np, s, &ph0));
                HIPTRY(launch_items_prefix(b.parkcnt, 0, Q, dtw_batch(n, wb, false), b.prefix, s));
                const DtwPhase ph1{d.split_row, 0, true, b.pool, d.pool_cap, nullptr, nullptr, 0, nullptr};
                HIPTRY(launch_dtw(p, db->rows, n, wb, qd, PairList{b.list1, d.C, b.parkcnt, 0}, b.prefix, Q, nullptr,
                                  grid, k == 1 ? b.best : nullptr, k == 1 ? nullptr : b.thr, b.res, d.ldres, rescnt,
                                  abandoned, nullptr, true, false, b.ring, d.ring_bytes,
                                  sp.kn.cascade ? S1v : nullptr, d.Np, s, &ph1));
            } else {
                HIPTRY(launch_dtw(p, db->rows, n, wb, qd, dl, b.prefix, Q, nullptr, grid, k == 1 ? b.best : nullptr,
                                  k == 1 ? nullptr : b.thr, b.res, d.ldres, rescnt, abandoned, nullptr, true, dtw_ll,
                                  b.ring, d.ring_bytes, sp.kn.cascade ? S1v : nullptr, d.Np, s));
            }
        }
        if (chunked && c1 < N) {  // the next chunk starts from the k best keys so far
            if (k > 1) HIPTRY(launch_res_shrink(b.res, d.ldres, rescnt, Q, k, sp.kq, b.thr, s));
            if (!d.brute) HIPTRY(launch_chunk_counts(b.counters, b.tot, Q, s));
        }
    }
    if (chunked && !d.brute) HIPTRY(launch_chunk_counts(b.counters, b.tot, Q, s));
    stage(7);
    if (k == 1)
        HIPTRY(launch_finalize1(b.best, Q, p, sp.idx, sp.dist, sp.qmap, ldo, s));
    else
        HIPTRY(launch_finalize_k(b.res, d.ldres, rescnt, Q, k, sp.kq, ldo, p, sp.idx, sp.dist, sp.qmap, s));
    stage(8);
    return LBIMP_OK;
}

static Knobs ctx_knobs(const lbimp_ctx *ctx) {
    Knobs k{ctx->seeds, ctx->lbi_pipeline, ctx->sweep_shape, false, false, true, ctx->pd_prefilter, ctx->lbi_abandon};
    k.lbi_buckets = ctx->lbi_buckets;
    k.dtw_split = ctx->dtw_split;
    return k;
}

static TuneKey tune_key(const lbimp_db *db, int64_t Q, int wb, int p, int k, int mode) {
    return TuneKey{db->N, db->n, wb, p, k, mode, pow2_at_least(Q)};
}

static Knobs knobs_of(const std::array<int, kTuneKnobs> &v) {
    Knobs k{v[0], v[2], v[1], v[3] != 0, v[4] != 0, v[5] != 0, v[6], v[7] != 0};
    k.lbi_buckets = v[8] != 0;
    k.dtw_split = v[9] != 0;
    return k;
}

static std::array<int, kTuneKnobs> knob_values(const Knobs &k) {
    return {k.seeds, k.sweep_shape, k.lbi_pipeline, k.dtw_group ? 1 : 0, k.seed_lane ? 1 : 0,
            k.cascade ? 1 : 0, k.pd, k.lbi_abandon ? 1 : 0, k.lbi_buckets ? 1 : 0, k.dtw_split ? 1 : 0};
}

// The tuned choice for this batch shape if there is one, else the context's options.
static Knobs knobs_for(const lbimp_ctx *ctx, const lbimp_db *db, int64_t Q, int wb, int p, int k, int mode) {
    auto it = ctx->tuned.find(tune_key(db, Q, wb, p, k, mode));
    return it == ctx->tuned.end() ? ctx_knobs(ctx) : knobs_of(it->second);
}

static int check_search(int64_t Q, int32_t n, int32_t w, int32_t p, int32_t k, int32_t mode);
static int acquire_pinned(lbimp_ctx *ctx, size_t bytes, PinnedChunk **out);

// Autotuner: times the whole search of this batch (on the context's stream, HIP events) under
// candidate choices -- seeds, sweep tiling, lane- or group-per-pair DTW for seeds and for
// survivors, pipelined LB_Improved loads -- one knob at a time from the current best (a
// coordinate descent), and records the fastest for the batch's TuneKey.  The queries are
// either device [Q][n] (`qdev`) or gathered from a packed array by host offsets.  Every
// candidate computes the same result; only time differs.
static int tune_search(lbimp_ctx *ctx, const lbimp_db *db, const float *qdev, const float *packed,
                       const int64_t *host_off, int64_t Q, int wb, int p, int k, int mode, Knobs *out) {
    const int n = db->n;
    const bool brute = mode == LBIMP_MODE_BRUTE, improved = mode == LBIMP_MODE_IMPROVED;
    const int seed_opts[] = {8, 16, 32, 64};
    const int shape_opts[] = {0, 2, 3, 4, 5};
    // workspace: [queries (gathered) | offsets | idx | dist][search buffers of the largest candidate]
    size_t search_bytes = 0;
    for (int sd : seed_opts)
        for (int sh : shape_opts)
            for (int pdv : {0, 1, 2})
                for (bool bk : {false, true}) {
                    SearchSpec sp{db, nullptr, Q, wb, p, k, mode, nullptr, nullptr, nullptr,
                                  Knobs{sd, 1, sh, false, false, true, pdv}};
                    sp.kn.lbi_buckets = bk;
                    sp.kn.dtw_split = true;  // the largest layout: with the row-phase pool
                    sp.ws_limit = ctx->ws_limit;
                    sp.pool_slots = ctx->dtw_pool_slots;
                    SearchDims d;
                    if (int r = dims_of(sp, ctx->num_cu, d)) return r;
                    SearchBufs b;
                    Carver cv{nullptr};
                    layout(cv, d, b);
                    search_bytes = std::max(search_bytes, cv.off);
                }
    auto carve_tune = [&](Carver &c, float *&qb, int64_t *&ob, int64_t *&ib, float *&db_) {
        qb = qdev ? nullptr : c.take<float>((size_t)Q * n);
        ob = qdev ? nullptr : c.take<int64_t>((size_t)Q);
        ib = c.take<int64_t>((size_t)Q * k);
        db_ = c.take<float>((size_t)Q * k);
        c.off = align_up(c.off, 256);
    };
    float *qb = nullptr, *dist = nullptr;
    int64_t *ob = nullptr, *idx = nullptr;
    size_t head = 0;
    {
        Carver cv{nullptr};
        carve_tune(cv, qb, ob, idx, dist);
        head = cv.off;
        if (int r = reserve(ctx, head + search_bytes)) return r;
        Carver c2{static_cast<char *>(ctx->ws)};
        carve_tune(c2, qb, ob, idx, dist);
    }
    hipStream_t s = ctx->stream;
    const float *queries = qdev;
    if (!qdev) {  // gather the batch's queries into the tuning area
        PinnedChunk *pc = nullptr;
        if (int r = acquire_pinned(ctx, sizeof(int64_t) * (size_t)Q, &pc)) return r;
        std::memcpy(pc->ptr, host_off, sizeof(int64_t) * (size_t)Q);
        HIPTRY(hipMemcpyAsync(ob, pc->ptr, sizeof(int64_t) * (size_t)Q, hipMemcpyHostToDevice, s));
        HIPTRY(hipEventRecord(pc->ev, s));
        HIPTRY(launch_gather_rows(packed, ob, n, Q, qb, s));
        queries = qb;
    }
    for (auto &e : ctx->tev)
        if (!e) HIPTRY(hipEventCreate(&e));
    auto time_of = [&](const Knobs &kn, float *ms) -> int {
        SearchSpec sp{db, queries, Q, wb, p, k, mode, idx, dist, nullptr, kn};
        sp.ws_limit = ctx->ws_limit;
        sp.pool_slots = ctx->dtw_pool_slots;
        SearchDims d;
        if (int r = dims_of(sp, ctx->num_cu, d)) return r;
        SearchBufs b;
        Carver c{static_cast<char *>(ctx->ws) + head};
        layout(c, d, b);
        if (int r = enqueue_search(ctx, sp, d, b, s, false)) return r;  // warm-up
        // the best of three timings of two searches each: choices a few percent apart are told
        // apart reliably, and a timing disturbed by other work on the device is discarded
        float best_t = 0.f;
        for (int trial = 0; trial < 3; ++trial) {
            HIPTRY(hipEventRecord(ctx->tev[0], s));
            for (int rep = 0; rep < 2; ++rep)
                if (int r = enqueue_search(ctx, sp, d, b, s, false)) return r;
            HIPTRY(hipEventRecord(ctx->tev[1], s));
            HIPTRY(hipEventSynchronize(ctx->tev[1]));
            float t = 0.f;
            HIPTRY(hipEventElapsedTime(&t, ctx->tev[0], ctx->tev[1]));
            best_t = trial == 0 ? t : std::min(best_t, t);
        }
        *ms = best_t;
        return LBIMP_OK;
    };
    Knobs best = ctx_knobs(ctx);
    float best_ms = 0.f;
    if (int r = time_of(best, &best_ms)) return r;
    auto consider = [&](Knobs kn) -> int {
        if (knob_values(kn) == knob_values(best)) return LBIMP_OK;
        float ms = 0.f;
        if (int r = time_of(kn, &ms)) return r;
        if (ms < best_ms) {
            best_ms = ms;
            best = kn;
        }
        return LBIMP_OK;
    };
    if (!brute) {
        const Knobs b0 = best;
        for (int sd : seed_opts) {
            Knobs kn = b0;
            kn.seeds = sd;
            if (int r = consider(kn)) return r;
        }
        const Knobs b1 = best;
        for (int sh : shape_opts) {
            Knobs kn = b1;
            kn.sweep_shape = sh;
            if (int r = consider(kn)) return r;
        }
        Knobs kn = best;
        kn.seed_lane = !kn.seed_lane;
        if (int r = consider(kn)) return r;
    }
    if (wb <= kLaneMaxW || dtw_wavereg_wide_supported(db->n, wb)) {
        Knobs kn = best;
        kn.dtw_group = !kn.dtw_group;
        if (int r = consider(kn)) return r;
    }
    if (improved && wb <= kLbiRegMaxW) {
        Knobs kn = best;
        for (int depth = 0; depth <= 1; ++depth) {
            kn.lbi_pipeline = depth;
            if (int r = consider(kn)) return r;
        }
    }
    if (improved) {
        Knobs kn = best;
        kn.lbi_abandon = !kn.lbi_abandon;
        if (int r = consider(kn)) return r;
        kn = best;
        kn.lbi_buckets = !kn.lbi_buckets;  // pays where the rows of the survivors come from HBM or MALL
        if (int r = consider(kn)) return r;
    }
    if (!brute) {
        Knobs kn = best;
        kn.cascade = !kn.cascade;
        if (int r = consider(kn)) return r;
        // pass 0 on the 8-part cover pays where the first pass is bound by database reads (few
        // queries); on the 32-part cover where the series are smooth enough for it to prune
        // almost as well as LB_Keogh.  A new first pass can move the best seed count.
        const Knobs b2 = best;
        for (int pv = 0; pv <= 2; ++pv) {
            if (pv == 2 && !fine_supported(db, improved, wb)) continue;
            kn = b2;
            kn.pd = pv;
            if (int r = consider(kn)) return r;
        }
        if (best.pd != b2.pd) {
            const Knobs b3 = best;
            for (int sd : seed_opts) {
                kn = b3;
                kn.seeds = sd;
                if (int r = consider(kn)) return r;
            }
        }
    }
    if (improved && wb <= kLaneMaxW && !best.dtw_group) {
        // two row phases for the survivors' DTW, repacking the pairs still running at half the series
        Knobs kn = best;
        kn.dtw_split = !kn.dtw_split;
        if (int r = consider(kn)) return r;
    }
    ctx->tuned[tune_key(db, Q, wb, p, k, mode)] = knob_values(best);
    *out = best;
    return LBIMP_OK;
}

static int check_search(int64_t Q, int32_t n, int32_t w, int32_t p, int32_t k, int32_t mode) {
    if (int r = check_shape(Q, n, w, p)) return r;
    if (k < 1 || k > 64) return fail(LBIMP_E_INVALID, "k = %d outside [1, 64]", k);
    if (mode < LBIMP_MODE_BRUTE || mode > LBIMP_MODE_IMPROVED) return fail(LBIMP_E_INVALID, "unknown mode %d", mode);
    return LBIMP_OK;
}

// A staging buffer of at least `bytes` whose previous upload has completed: the host waits
// only when every buffer of the ring is still being read.
static int acquire_pinned(lbimp_ctx *ctx, size_t bytes, PinnedChunk **out) {
    for (auto &c : ctx->pinned) {
        if (c.cap < bytes) continue;
        const hipError_t e = hipEventQuery(c.ev);
        if (e == hipSuccess) {
            *out = &c;
            return LBIMP_OK;
        }
        if (e != hipErrorNotReady) return fail(LBIMP_E_DEVICE, "hipEventQuery: %s", hipGetErrorString(e));
    }
    PinnedChunk *slot = nullptr;
    if (ctx->pinned.size() < kPinnedRing) {
        ctx->pinned.emplace_back();
        slot = &ctx->pinned.back();
        HIPTRY(hipEventCreateWithFlags(&slot->ev, hipEventDisableTiming));
    } else {
        slot = &ctx->pinned[0];  // the ring is full: reuse the first buffer once its copy has run
        for (auto &c : ctx->pinned)
            if (c.cap >= bytes) {
                slot = &c;
                break;
            }
        HIPTRY(hipEventSynchronize(slot->ev));
    }
    if (slot->cap < bytes) {
        if (slot->ptr) HIPTRY(hipHostFree(slot->ptr));
        slot->ptr = nullptr;
        slot->cap = 0;
        const size_t cap = align_up(std::max<size_t>(bytes + bytes / 4, 1 << 16), 1 << 16);
        if (hipHostMalloc(&slot->ptr, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            slot->ptr = nullptr;
            return fail(LBIMP_E_NOMEM, "pinned staging allocation of %zu bytes failed", cap);
        }
        slot->cap = cap;
    }
    *out = slot;
    return LBIMP_OK;
}

static int ensure_pool(lbimp_ctx *ctx) {
    if (ctx->graph_stream) return LBIMP_OK;
    HIPTRY(hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
    for (int i = 0; i < kPoolStreams; ++i) {
        HIPTRY(hipStreamCreateWithFlags(&ctx->pool[i], hipStreamNonBlocking));
        HIPTRY(hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming));
    }
    HIPTRY(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
    HIPTRY(hipEventCreateWithFlags(&ctx->enter_ev, hipEventDisableTiming));
    HIPTRY(hipEventCreateWithFlags(&ctx->exit_ev, hipEventDisableTiming));
    return LBIMP_OK;
}

// Grouping and workspace layout of a ragged batch: queries sharing a database and an
// effective band form one homogeneous search.  offsets may be null (lengths unchecked).
struct RaggedPlan {
    std::map<std::pair<int, int>, std::vector<int64_t>> groups;
    std::vector<SearchSpec> specs;
    std::vector<SearchDims> dims;
    std::vector<SearchBufs> bufs;
    std::vector<float *> qbuf;
    std::vector<int64_t *> qmap, qsrc, kq;
    std::vector<bool> mixed_k;  // the group's queries ask for different k
    int kmax = 1;               // output row stride: the largest k of the batch
    size_t meta_elems = 0;
    int64_t *meta = nullptr;

    // workspace: [metadata: per group query ids, source offsets, k of each query]
    //            [per group: queries + search]
    void carve(Carver &c) {
        meta = c.take<int64_t>(meta_elems);
        size_t o = 0;
        for (size_t g = 0; g < specs.size(); ++g) {
            qmap[g] = meta ? meta + o : nullptr;
            qsrc[g] = meta ? meta + o + specs[g].Q : nullptr;
            kq[g] = meta ? meta + o + 2 * specs[g].Q : nullptr;
            o += 3 * (size_t)specs[g].Q;
        }
        for (size_t g = 0; g < specs.size(); ++g) {
            qbuf[g] = c.take<float>((size_t)specs[g].Q * dims[g].n);
            layout(c, dims[g], bufs[g]);
        }
    }
};

static int plan_ragged(lbimp_ctx *ctx, const lbimp_db *const *dbs, int32_t ndb, const int64_t *offsets,
                       const int32_t *db_of, const int32_t *w, int64_t Q, int32_t p, const int32_t *k, int32_t mode,
                       int64_t *idx, float *dist, RaggedPlan &plan) {
    if (!dbs || ndb < 1 || !db_of || !w || !k) return fail(LBIMP_E_INVALID, "null pointer or no database");
    for (int i = 0; i < ndb; ++i) {
        if (!dbs[i]) return fail(LBIMP_E_INVALID, "null database %d", i);
        if (dbs[i]->device != ctx->device) return fail(LBIMP_E_INVALID, "database %d lives on another device", i);
    }
    for (int64_t q = 0; q < Q; ++q) {
        const int b = db_of[q];
        if (b < 0 || b >= ndb) return fail(LBIMP_E_INVALID, "query %lld: database %d of %d", (long long)q, b, ndb);
        if (offsets) {
            const int64_t len = offsets[q + 1] - offsets[q];
            if (offsets[q] < 0 || len != dbs[b]->n)
                return fail(LBIMP_E_INVALID, "query %lld: length %lld, database length %d", (long long)q,
                            (long long)len, dbs[b]->n);
        }
        if (int r = check_search(1, dbs[b]->n, w[q], p, k[q], mode)) return r;
        plan.groups[{b, band_of(dbs[b]->n, w[q])}].push_back(q);
        plan.kmax = std::max(plan.kmax, (int)k[q]);
    }
    const size_t G = plan.groups.size();
    plan.dims.resize(G);
    plan.bufs.resize(G);
    plan.qbuf.resize(G);
    plan.qmap.resize(G);
    plan.qsrc.resize(G);
    plan.kq.resize(G);
    plan.mixed_k.resize(G);
    plan.specs.reserve(G);
    for (auto &kv : plan.groups) {
        const int64_t Qg = (int64_t)kv.second.size();
        const lbimp_db *db = dbs[kv.first.first];
        int kg = 1;  // the group runs as one search for its largest k; each query keeps its own k
        bool mixed = false;
        for (int64_t q : kv.second) {
            mixed |= k[q] != k[kv.second[0]];
            kg = std::max(kg, (int)k[q]);
        }
        plan.mixed_k[plan.specs.size()] = mixed;
        SearchSpec sp{db, nullptr, Qg, kv.first.second, p, kg, mode, idx, dist, nullptr,
                      knobs_for(ctx, db, Qg, kv.first.second, p, kg, mode)};
        sp.ldo = plan.kmax;
        sp.ws_limit = ctx->ws_limit;
        sp.pool_slots = ctx->dtw_pool_slots;
        plan.specs.push_back(sp);
        if (int r = dims_of(plan.specs.back(), ctx->num_cu, plan.dims[plan.specs.size() - 1])) return r;
        plan.meta_elems += 3 * (size_t)Qg;
    }
    return LBIMP_OK;
}

extern "C" {

const char *lbimp_last_error(void) { return g_err.c_str(); }

int lbimp_ctx_create(int device, void *hip_stream, lbimp_ctx **out) {
    if (!out) return fail(LBIMP_E_INVALID, "null output pointer");
    *out = nullptr;
    int count = 0;
    HIPTRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(LBIMP_E_INVALID, "device %d of %d", device, count);
    HIPTRY(hipSetDevice(device));
    lbimp_ctx *ctx = new (std::nothrow) lbimp_ctx;
    if (!ctx) return fail(LBIMP_E_NOMEM, "host allocation failed");
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    if (int r = init_scratch(device)) {
        delete ctx;
        return r;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
    *out = ctx;
    return LBIMP_OK;
}

int lbimp_ctx_set_stream(lbimp_ctx *ctx, void *hip_stream) {
    if (!ctx) return fail(LBIMP_E_INVALID, "null context");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return LBIMP_OK;
}

void lbimp_ctx_destroy(lbimp_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->graph_stream) (void)hipStreamSynchronize(ctx->graph_stream);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    for (int i = 0; i < kPoolStreams; ++i) {
        if (ctx->pool[i]) (void)hipStreamDestroy(ctx->pool[i]);
        if (ctx->join_ev[i]) (void)hipEventDestroy(ctx->join_ev[i]);
    }
    for (hipEvent_t e : {ctx->fork_ev, ctx->enter_ev, ctx->exit_ev, ctx->tev[0], ctx->tev[1]})
        if (e) (void)hipEventDestroy(e);
    if (ctx->graph_stream) (void)hipStreamDestroy(ctx->graph_stream);
    for (auto &c : ctx->pinned) {
        if (c.ev) (void)hipEventSynchronize(c.ev), (void)hipEventDestroy(c.ev);
        if (c.ptr) (void)hipHostFree(c.ptr);
    }
    if (ctx->ws) (void)hipFree(ctx->ws);
    delete ctx;
}

int lbimp_ctx_set_timing(lbimp_ctx *ctx, int enable) {
    if (int r = check_ctx(ctx)) return r;
    if (enable && !ctx->ev[0])
        for (auto &e : ctx->ev) HIPTRY(hipEventCreate(&e));
    ctx->timing = enable != 0;
    ctx->timed_valid = false;
    return LBIMP_OK;
}

int lbimp_ctx_set_option(lbimp_ctx *ctx, const char *name, int64_t value) {
    if (!ctx || !name) return fail(LBIMP_E_INVALID, "null argument");
    if (!strcmp(name, "seeds")) {
        if (value < 1 || value > kMaxSeeds) return fail(LBIMP_E_INVALID, "seeds must be in [1, %d]", kMaxSeeds);
        ctx->seeds = (int)value;
    } else if (!strcmp(name, "lbi_pipeline")) {
        if (value < 0 || value > 1) return fail(LBIMP_E_INVALID, "lbi_pipeline must be 0 or 1");
        ctx->lbi_pipeline = (int)value;
    } else if (!strcmp(name, "dtw_group_per_pair")) {
        ctx->dtw_low_latency = value != 0;
    } else if (!strcmp(name, "graph")) {
        ctx->use_graph = value != 0;
    } else if (!strcmp(name, "autotune")) {
        ctx->autotune = value != 0;
    } else if (!strcmp(name, "ragged_streams")) {
        if (value < 0 || value > kPoolStreams)
            return fail(LBIMP_E_INVALID, "ragged_streams must be in [0, %d]", kPoolStreams);
        ctx->ragged_streams = (int)value;
    } else if (!strcmp(name, "pd_prefilter")) {
        if (value < 0 || value > 2) return fail(LBIMP_E_INVALID, "pd_prefilter must be 0, 1 or 2");
        ctx->pd_prefilter = (int)value;
    } else if (!strcmp(name, "pd_fine")) {
        ctx->pd_fine_bound = value != 0;
    } else if (!strcmp(name, "dtw_split")) {
        ctx->dtw_split = value != 0;
    } else if (!strcmp(name, "dtw_pool_slots")) {
        if (value < 0 || value > (int64_t)1 << 26) return fail(LBIMP_E_INVALID, "dtw_pool_slots must be in [0, 2^26]");
        ctx->dtw_pool_slots = value;
    } else if (!strcmp(name, "lbi_abandon")) {
        ctx->lbi_abandon = value != 0;
    } else if (!strcmp(name, "lbi_buckets")) {
        ctx->lbi_buckets = value != 0;
    } else if (!strcmp(name, "workspace_limit")) {
        if (value < 0) return fail(LBIMP_E_INVALID, "workspace_limit must be >= 0");
        ctx->ws_limit = (size_t)value;
    } else if (!strcmp(name, "sweep_shape")) {
        if (value < 0 || value > 5) return fail(LBIMP_E_INVALID, "sweep_shape must be in [0, 5]");
        ctx->sweep_shape = (int)value;
    } else {
        return fail(LBIMP_E_INVALID, "unknown option '%s'", name);
    }
    return LBIMP_OK;
}

int lbimp_ctx_stage_times(lbimp_ctx *ctx, float *ms, int max) {
    if (int r = check_ctx(ctx)) return -r;
    if (!ms || max < 0) return -fail(LBIMP_E_INVALID, "null output");
    if (!ctx->timing || !ctx->timed_valid) return -fail(LBIMP_E_INVALID, "no timed search recorded");
    HIPTRY(hipEventSynchronize(ctx->ev[kStages]));
    int m = std::min(max, kStages);
    for (int i = 0; i < m; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ctx->ev[i], ctx->ev[i + 1]) != hipSuccess) return -LBIMP_E_DEVICE;
        ms[i] = t;
    }
    return m;
}

int lbimp_db_create(lbimp_ctx *ctx, const float *rows, int64_t N, int32_t n, lbimp_db **out) {
    if (int r = check_ctx(ctx)) return r;
    if (!out) return fail(LBIMP_E_INVALID, "null output pointer");
    *out = nullptr;
    if (int r = check_shape(N, n, 0, 1)) return r;
    if (N > 0 && !rows) return fail(LBIMP_E_INVALID, "null rows");
    lbimp_db *db = new (std::nothrow) lbimp_db;
    if (!db) return fail(LBIMP_E_NOMEM, "host allocation failed");
    db->device = ctx->device;
    db->N = N;
    db->n = n;
    const int n4 = (n + 3) / 4;
    const int64_t T = (N + 63) / 64;
    size_t rbytes = sizeof(float) * (size_t)std::max<int64_t>(N, 1) * n;
    size_t ibytes = sizeof(float4) * (size_t)std::max<int64_t>(T, 1) * n4 * 64;
    size_t pbytes = sizeof(double) * (size_t)std::max<int64_t>(N, 1) * kPdParts;
    const bool fine = n >= kPdfMinN && N > 0;
    size_t fbytes = sizeof(float4) * (size_t)T * (kPdFine / 4) * 64;
    if (hipMalloc(&db->rows, rbytes) != hipSuccess || hipMalloc(&db->il, ibytes) != hipSuccess ||
        hipMalloc(&db->pd, pbytes) != hipSuccess || (fine && hipMalloc(&db->pdf, fbytes) != hipSuccess)) {
        (void)hipGetLastError();
        lbimp_db_destroy(db);
        return fail(LBIMP_E_NOMEM, "database allocation failed");
    }
    if (N > 0) {
        hipError_t e = hipMemcpyAsync(db->rows, rows, sizeof(float) * (size_t)N * n, hipMemcpyDeviceToDevice,
                                      ctx->stream);
        if (e == hipSuccess) e = launch_pack(rows, N, n, db->il, ctx->stream);
        if (e == hipSuccess) e = launch_pd_rows(rows, N, n, db->pd, ctx->stream);
        if (e == hipSuccess && fine) e = launch_pdf_rows(rows, N, n, db->pdf, ctx->stream);
        if (e != hipSuccess) {
            lbimp_db_destroy(db);
            return fail(LBIMP_E_DEVICE, "database upload: %s", hipGetErrorString(e));
        }
    }
    *out = db;
    return LBIMP_OK;
}

void lbimp_db_destroy(lbimp_db *db) {
    if (!db) return;
    (void)hipSetDevice(db->device);
    (void)hipDeviceSynchronize();
    if (db->rows) (void)hipFree(db->rows);
    if (db->il) (void)hipFree(db->il);
    if (db->pd) (void)hipFree(db->pd);
    if (db->pdf) (void)hipFree(db->pdf);
    delete db;
}

int64_t lbimp_db_size(const lbimp_db *db) { return db ? db->N : -1; }
int32_t lbimp_db_length(const lbimp_db *db) { return db ? db->n : -1; }

int lbimp_envelope(lbimp_ctx *ctx, const float *y, int64_t B, int32_t n, int32_t w, float *U, float *L) {
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_shape(B, n, w, 1)) return r;
    if (B == 0) return LBIMP_OK;
    if (!y || !U || !L) return fail(LBIMP_E_INVALID, "null pointer");
    HIPTRY(launch_envelope(y, B, B, n, band_of(n, w), U, L, n, ctx->stream));
    return LBIMP_OK;
}

int lbimp_lb_keogh(lbimp_ctx *ctx, const float *x, int64_t N, int32_t n, const float *U, const float *L,
                   int32_t p, float *lb) {
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_shape(N, n, 0, p)) return r;
    if (N == 0) return LBIMP_OK;
    if (!x || !U || !L || !lb) return fail(LBIMP_E_INVALID, "null pointer");
    const int n4 = (n + 3) / 4;
    const int64_t T = (N + 63) / 64;
    Carver cv{nullptr};
    cv.take<float4>((size_t)T * n4 * 64);
    cv.take<float>((size_t)n4 * 4);
    cv.take<float>((size_t)n4 * 4);
    if (int r = reserve(ctx, cv.off)) return r;
    Carver c2{static_cast<char *>(ctx->ws)};
    float4 *il = c2.take<float4>((size_t)T * n4 * 64);
    float *Ud = c2.take<float>((size_t)n4 * 4);
    float *Ld = c2.take<float>((size_t)n4 * 4);
    HIPTRY(launch_pack(x, N, n, il, ctx->stream));
    HIPTRY(launch_pad_env(U, L, 1, 1, n, Ud, Ld, n4 * 4, ctx->stream));
    HIPTRY(launch_lbk_sweep(p, 0, il, N, n4, reinterpret_cast<float4 *>(Ud), reinterpret_cast<float4 *>(Ld), n4, 1, lb,
                            N, false, true, nullptr, ctx->stream));
    return LBIMP_OK;
}

int lbimp_db_lb_keogh(lbimp_ctx *ctx, const lbimp_db *db, const float *U, const float *L, int64_t Q, int32_t p,
                      float *lb) {
    if (int r = check_ctx(ctx)) return r;
    if (!db) return fail(LBIMP_E_INVALID, "null database");
    if (int r = check_shape(Q, db->n, 0, p)) return r;
    if (Q == 0 || db->N == 0) return LBIMP_OK;
    if (!U || !L || !lb) return fail(LBIMP_E_INVALID, "null pointer");
    const int n = db->n, n4 = (n + 3) / 4;
    const int qg = sweep_query_group(ctx->sweep_shape, Q);
    const int64_t Qp = (Q + qg - 1) / qg * qg;
    Carver cv{nullptr};
    cv.take<float>((size_t)Qp * n4 * 4);
    cv.take<float>((size_t)Qp * n4 * 4);
    if (int r = reserve(ctx, cv.off)) return r;
    Carver c2{static_cast<char *>(ctx->ws)};
    float *Ud = c2.take<float>((size_t)Qp * n4 * 4);
    float *Ld = c2.take<float>((size_t)Qp * n4 * 4);
    HIPTRY(launch_pad_env(U, L, Q, Qp, n, Ud, Ld, n4 * 4, ctx->stream));
    HIPTRY(launch_lbk_sweep(p, ctx->sweep_shape, db->il, db->N, n4, reinterpret_cast<float4 *>(Ud), reinterpret_cast<float4 *>(Ld), n4,
                            Q, lb, db->N, false, true, nullptr, ctx->stream));
    return LBIMP_OK;
}

int lbimp_db_pd_bound(lbimp_ctx *ctx, const lbimp_db *db, const float *U, const float *L, int64_t Q, int32_t p,
                      float *lb) {
    if (int r = check_ctx(ctx)) return r;
    if (!db) return fail(LBIMP_E_INVALID, "null database");
    if (int r = check_shape(Q, db->n, 0, p)) return r;
    if (Q == 0 || db->N == 0) return LBIMP_OK;
    if (!U || !L || !lb) return fail(LBIMP_E_INVALID, "null pointer");
    if (ctx->pd_fine_bound) {  // the 32-part cover (fp32 with rounding margins)
        if (!db->pdf) return fail(LBIMP_E_UNSUPPORTED, "no 32-part sums for series shorter than %d", kPdfMinN);
        Carver cv{nullptr};
        cv.take<float>((size_t)Q * kPdfQuery);
        if (int r = reserve(ctx, cv.off)) return r;
        Carver c2{static_cast<char *>(ctx->ws)};
        float *qpf = c2.take<float>((size_t)Q * kPdfQuery);
        HIPTRY(launch_pdf_query(U, L, db->n, Q, db->n, qpf, ctx->stream));
        HIPTRY(launch_pdf_scan(p, db->pdf, db->N, db->n, qpf, Q, lb, db->N, true, nullptr, ctx->stream, 0));
        return LBIMP_OK;
    }
    Carver cv{nullptr};
    cv.take<double>((size_t)Q * 2 * kPdParts);
    if (int r = reserve(ctx, cv.off)) return r;
    Carver c2{static_cast<char *>(ctx->ws)};
    double *qpd = c2.take<double>((size_t)Q * 2 * kPdParts);
    HIPTRY(launch_pd_query(U, L, db->n, Q, db->n, qpd, ctx->stream));
    HIPTRY(launch_pd_scan(p, db->pd, db->N, db->n, qpd, Q, lb, db->N, false, true, nullptr, ctx->stream));
    return LBIMP_OK;
}

int lbimp_lb_improved(lbimp_ctx *ctx, const float *x, int64_t N, int32_t n, const float *y, const float *U,
                      const float *L, int32_t w, int32_t p, float *lb) {
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_shape(N, n, w, p)) return r;
    if (N == 0) return LBIMP_OK;
    if (!x || !y || !U || !L || !lb) return fail(LBIMP_E_INVALID, "null pointer");
    const int wb = band_of(n, w);
    const int WL = lbi_batch(n, wb);
    if (WL == 0) return fail(LBIMP_E_UNSUPPORTED, "LB_Improved state for n = %d, w = %d exceeds LDS", n, wb);
    const int n4 = (n + 3) / 4;
    const int64_t T = (N + 63) / 64;
    Carver cv{nullptr};
    cv.take<float4>((size_t)T * n4 * 64);
    cv.take<float>((size_t)n4 * 4);
    cv.take<float>((size_t)n4 * 4);
    cv.take<float>((size_t)N);
    cv.take<long long>(2);
    cv.take<int>(1);
    if (int r = reserve(ctx, cv.off)) return r;
    Carver c2{static_cast<char *>(ctx->ws)};
    float4 *il = c2.take<float4>((size_t)T * n4 * 64);
    float *Ud = c2.take<float>((size_t)n4 * 4);
    float *Ld = c2.take<float>((size_t)n4 * 4);
    float *S1 = c2.take<float>((size_t)N);
    long long *prefix = c2.take<long long>(2);
    int *ctr = c2.take<int>(1);
    hipStream_t s = ctx->stream;
    HIPTRY(launch_pack(x, N, n, il, s));
    HIPTRY(launch_pad_env(U, L, 1, 1, n, Ud, Ld, n4 * 4, s));
    HIPTRY(launch_lbk_sweep(p, 0, il, N, n4, reinterpret_cast<float4 *>(Ud), reinterpret_cast<float4 *>(Ld), n4, 1, S1,
                            N, false, false, nullptr, s));
    HIPTRY(launch_fill_i32(ctr, 0, 1, s));
    QueryData qd{y, n, U, L, n};
    PairList pl{nullptr, 0, nullptr, N};
    HIPTRY(launch_lbi(p, x, (int64_t)N * n * 4, n, wb, qd, pl, S1, N, prefix, 1, ctr, persistent_grid(ctx), nullptr, nullptr, 0,
                      nullptr, lb, ctx->lbi_pipeline, false, s));
    return LBIMP_OK;
}

int lbimp_dtw_band(lbimp_ctx *ctx, const float *x, int64_t N, const float *y, int32_t n, int32_t w, int32_t p,
                   float *dist) {
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_shape(N, n, w, p)) return r;
    if (N == 0) return LBIMP_OK;
    if (!x || !y || !dist) return fail(LBIMP_E_INVALID, "null pointer");
    const int wb = band_of(n, w);
    const bool ll = ctx->dtw_low_latency;
    const size_t ring_bytes = ll ? 0 : dtw_strip_scratch(p, n, wb, ctx->num_cu);
    Carver cv{nullptr};
    cv.take<long long>(2);
    cv.take<int>(1);
    cv.take<u64>(1);
    cv.take<float>(ring_bytes / sizeof(float));
    if (int r = reserve(ctx, cv.off)) return r;
    Carver c2{static_cast<char *>(ctx->ws)};
    long long *prefix = c2.take<long long>(2);
    int *ctr = c2.take<int>(1);
    u64 *nothr = c2.take<u64>(1);
    float *ring = c2.take<float>(ring_bytes / sizeof(float));
    hipStream_t s = ctx->stream;
    HIPTRY(launch_fill_i32(ctr, 0, 1, s));
    HIPTRY(launch_fill_u64(nothr, kNoKey, 1, s));
    QueryData qd{y, n, nullptr, nullptr, 0};
    PairList pl{nullptr, 0, nullptr, N};
    // no threshold: nothing is abandoned and nothing appended (out_root receives every distance)
    HIPTRY(launch_dtw(p, x, n, wb, qd, pl, prefix, 1, ctr, persistent_grid(ctx), nullptr, nothr, nullptr, 0,
                      nullptr, nullptr, dist, false, ll, ring, ring_bytes, nullptr, 0, s));
    return LBIMP_OK;
}

int lbimp_dtw_pairs(lbimp_ctx *ctx, const float *x, const float *y, int64_t N, int32_t n, int32_t w, int32_t p,
                    float *dist) {
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_shape(N, n, w, p)) return r;
    if (N == 0) return LBIMP_OK;
    if (!x || !y || !dist) return fail(LBIMP_E_INVALID, "null pointer");
    const int wb = band_of(n, w);
    Carver cv{nullptr};
    cv.take<long long>(2);
    cv.take<int>(1);
    cv.take<int>((size_t)N);
    cv.take<u64>((size_t)N);
    if (int r = reserve(ctx, cv.off)) return r;
    Carver c2{static_cast<char *>(ctx->ws)};
    long long *prefix = c2.take<long long>(2);
    int *ctr = c2.take<int>(1);
    int *self = c2.take<int>((size_t)N);
    u64 *nothr = c2.take<u64>((size_t)N);
    hipStream_t s = ctx->stream;
    // pair c is query c (row c of y) against candidate c (row c of x): a list holding c for
    // query c, one pair per query, computed by the group-of-lanes-per-pair kernels, which stage
    // each pair's own query
    HIPTRY(launch_fill_i32(ctr, 0, 1, s));
    HIPTRY(launch_iota_i32(self, N, s));
    HIPTRY(launch_fill_u64(nothr, kNoKey, N, s));
    QueryData qd{y, n, nullptr, nullptr, 0};
    PairList pl{self, 1, nullptr, 1};
    HIPTRY(launch_dtw(p, x, n, wb, qd, pl, prefix, N, ctr, persistent_grid(ctx), nullptr, nothr, nullptr, 0, nullptr,
                      nullptr, dist, false, true, nullptr, 0, nullptr, 0, s));
    return LBIMP_OK;
}

int lbimp_nn_search(lbimp_ctx *ctx, const lbimp_db *db, const float *queries, int64_t Q, int32_t w, int32_t p,
                    int32_t k, int32_t mode, int64_t *idx, float *dist, lbimp_stats *stats) {
    if (int r = check_ctx(ctx)) return r;
    if (!db) return fail(LBIMP_E_INVALID, "null database");
    if (db->device != ctx->device) return fail(LBIMP_E_INVALID, "database lives on another device");
    if (int r = check_search(Q, db->n, w, p, k, mode)) return r;
    if (Q == 0) return LBIMP_OK;
    if (!queries || !idx || !dist) return fail(LBIMP_E_INVALID, "null pointer");
    const int wb = band_of(db->n, w);
    if (ctx->autotune && db->N > 0 && !ctx->tuned.count(tune_key(db, Q, wb, p, k, mode))) {
        Knobs tuned;
        if (int r = tune_search(ctx, db, queries, nullptr, nullptr, Q, wb, p, k, mode, &tuned)) return r;
    }
    SearchSpec sp{db, queries, Q, w, p, k, mode, idx, dist, nullptr, knobs_for(ctx, db, Q, wb, p, k, mode)};
    sp.ws_limit = ctx->ws_limit;
    sp.pool_slots = ctx->dtw_pool_slots;
    SearchDims d;
    if (int r = dims_of(sp, ctx->num_cu, d)) return r;
    SearchBufs bufs;
    {
        Carver cv{nullptr};
        layout(cv, d, bufs);
        if (int r = reserve(ctx, cv.off)) return r;
        Carver c2{static_cast<char *>(ctx->ws)};
        layout(c2, d, bufs);
    }
    ctx->timed_valid = false;
    if (int r = enqueue_search(ctx, sp, d, bufs, ctx->stream, true)) return r;
    ctx->timed_valid = ctx->timing;
    if (stats) {
        std::vector<int> h((size_t)Q * kCounters);
        HIPTRY(hipMemcpyAsync(h.data(), bufs.counters, sizeof(int) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
        HIPTRY(hipStreamSynchronize(ctx->stream));
        std::vector<long long> ht(bufs.tot ? (size_t)Q * 3 : 0);
        if (bufs.tot)
            HIPTRY(hipMemcpyAsync(ht.data(), bufs.tot, sizeof(long long) * ht.size(), hipMemcpyDeviceToHost,
                                  ctx->stream));
        HIPTRY(hipStreamSynchronize(ctx->stream));
        fill_stats(d, Q, h.data(), bufs.tot ? ht.data() : nullptr, nullptr, stats);
    }
    return LBIMP_OK;
}

int lbimp_nn_search_noalloc(lbimp_ctx *ctx, const lbimp_db *db, const float *queries, int64_t Q, int32_t w, int32_t p,
                            int32_t k, int32_t mode, int64_t *idx, float *dist) {
    if (int r = check_ctx(ctx)) return r;
    if (!db) return fail(LBIMP_E_INVALID, "null database");
    if (db->device != ctx->device) return fail(LBIMP_E_INVALID, "database lives on another device");
    if (int r = check_search(Q, db->n, w, p, k, mode)) return r;
    if (Q == 0) return LBIMP_OK;
    if (!queries || !idx || !dist) return fail(LBIMP_E_INVALID, "null pointer");
    void *base = g_scratch_ptr[ctx->device];
    if (!base) return fail(LBIMP_E_DEVICE, "scratch of device %d not initialised", ctx->device);
    // tuned choices are used when present; nothing is tuned here (tuning needs a workspace)
    const int wb = band_of(db->n, w);
    SearchSpec sp{db, queries, Q, w, p, k, mode, idx, dist, nullptr, knobs_for(ctx, db, Q, wb, p, k, mode)};
    // the candidates are split into chunks small enough for the scratch (or the context's bound)
    sp.ws_limit = ctx->ws_limit ? std::min<size_t>(ctx->ws_limit, LBIMP_NOALLOC_SCRATCH_BYTES)
                                : (size_t)LBIMP_NOALLOC_SCRATCH_BYTES;
    sp.pool_slots = ctx->dtw_pool_slots;
    SearchDims d;
    if (int r = dims_of(sp, ctx->num_cu, d)) return r;
    SearchBufs bufs;
    Carver cv{nullptr};
    layout(cv, d, bufs);
    if (cv.off > (size_t)LBIMP_NOALLOC_SCRATCH_BYTES)
        return fail(LBIMP_E_NOMEM, "search needs %zu bytes of scratch, more than the fixed %zu (LBIMP_NOALLOC_SCRATCH_BYTES)",
                    cv.off, (size_t)LBIMP_NOALLOC_SCRATCH_BYTES);
    Carver c2{static_cast<char *>(base)};
    layout(c2, d, bufs);
    ctx->timed_valid = false;
    if (int r = enqueue_search(ctx, sp, d, bufs, ctx->stream, true)) return r;
    ctx->timed_valid = ctx->timing;
    return LBIMP_OK;
}

int lbimp_nn_search_ragged(lbimp_ctx *ctx, const lbimp_db *const *dbs, int32_t ndb, const float *queries,
                           const int64_t *offsets, const int32_t *db_of, const int32_t *w, int64_t Q, int32_t p,
                           const int32_t *k, int32_t mode, int64_t *idx, float *dist, lbimp_stats *stats) {
    if (int r = check_ctx(ctx)) return r;
    if (Q < 0) return fail(LBIMP_E_INVALID, "negative query count");
    if (Q == 0) return LBIMP_OK;
    if (!queries || !offsets || !idx || !dist) return fail(LBIMP_E_INVALID, "null pointer");
    RaggedPlan plan;
    if (int r = plan_ragged(ctx, dbs, ndb, offsets, db_of, w, Q, p, k, mode, idx, dist, plan)) return r;
    if (ctx->autotune) {  // tune each group shape met for the first time, then plan again with the choices
        bool tuned_any = false;
        for (size_t g = 0; g < plan.specs.size(); ++g) {
            const SearchSpec &sp = plan.specs[g];
            if (sp.db->N == 0 || ctx->tuned.count(tune_key(sp.db, sp.Q, sp.w, p, sp.k, mode))) continue;
            const std::vector<int64_t> &ids = std::next(plan.groups.begin(), g)->second;
            std::vector<int64_t> off(ids.size());
            for (size_t i = 0; i < ids.size(); ++i) off[i] = offsets[ids[i]];
            Knobs kn;
            if (int r = tune_search(ctx, sp.db, nullptr, queries, off.data(), sp.Q, sp.w, p, sp.k, mode, &kn))
                return r;
            tuned_any = true;
        }
        if (tuned_any) {
            plan = RaggedPlan();
            if (int r = plan_ragged(ctx, dbs, ndb, offsets, db_of, w, Q, p, k, mode, idx, dist, plan)) return r;
        }
    }
    auto &groups = plan.groups;
    auto &specs = plan.specs;
    auto &dims = plan.dims;
    auto &bufs = plan.bufs;
    auto &qbuf = plan.qbuf;
    auto &qmap = plan.qmap;
    auto &qsrc = plan.qsrc;
    const int G = (int)specs.size();
    const size_t meta_elems = plan.meta_elems;
    {
        Carver cv{nullptr};
        plan.carve(cv);
        if (int r = reserve(ctx, cv.off)) return r;
        Carver c2{static_cast<char *>(ctx->ws)};
        plan.carve(c2);
    }
    int64_t *meta = plan.meta;
    // upload the metadata through a pinned staging buffer (outside any captured graph)
    {
        PinnedChunk *pc = nullptr;
        if (int r = acquire_pinned(ctx, meta_elems * sizeof(int64_t), &pc)) return r;
        int64_t *h = static_cast<int64_t *>(pc->ptr);
        size_t o = 0;
        for (auto &kv : groups) {
            for (int64_t q : kv.second) h[o++] = q;
            for (int64_t q : kv.second) h[o++] = offsets[q];
            for (int64_t q : kv.second) h[o++] = k[q];
        }
        HIPTRY(hipMemcpyAsync(meta, h, meta_elems * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        HIPTRY(hipEventRecord(pc->ev, ctx->stream));
    }
    // groups run concurrently on `width` pool streams (forked from and joined back to the
    // launching stream), or one after another on the launching stream when width <= 1
    const int width = std::min(ctx->ragged_streams, G);
    if (ctx->use_graph || width > 1)
        if (int r = ensure_pool(ctx)) return r;
    for (int g = 0; g < G; ++g) {
        specs[g].queries = qbuf[g];
        specs[g].qmap = qmap[g];
        specs[g].kq = plan.mixed_k[g] ? plan.kq[g] : nullptr;
    }
    // the groups run concurrently on the context's stream pool, captured once as a graph and
    // replayed while the call's signature (pointers, shapes, grouping, workspace) is unchanged
    auto enqueue_all = [&](hipStream_t main) -> int {
        if (width > 1) {
            HIPTRY(hipEventRecord(ctx->fork_ev, main));
            for (int i = 0; i < width; ++i) HIPTRY(hipStreamWaitEvent(ctx->pool[i], ctx->fork_ev, 0));
        }
        for (int g = 0; g < G; ++g) {
            hipStream_t sg = width > 1 ? ctx->pool[g % width] : main;
            HIPTRY(launch_gather_rows(queries, qsrc[g], dims[g].n, specs[g].Q, qbuf[g], sg));
            if (int r = enqueue_search(ctx, specs[g], dims[g], bufs[g], sg, false)) return r;
        }
        if (width > 1) {
            for (int i = 0; i < width; ++i) {
                HIPTRY(hipEventRecord(ctx->join_ev[i], ctx->pool[i]));
                HIPTRY(hipStreamWaitEvent(main, ctx->join_ev[i], 0));
            }
        }
        return LBIMP_OK;
    };
    uint64_t sig = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { sig = (sig ^ v) * 1099511628211ull; };
    mix((uint64_t)(uintptr_t)ctx->ws);
    mix((uint64_t)(uintptr_t)queries);
    mix((uint64_t)(uintptr_t)idx);
    mix((uint64_t)(uintptr_t)dist);
    mix((uint64_t)Q);
    mix((uint64_t)(uint32_t)p * 131 + (uint64_t)plan.kmax * 7 + (uint64_t)mode);
    mix((uint64_t)width);
    for (int g = 0; g < G; ++g) {
        const lbimp_db *db = specs[g].db;  // a database freed and recreated may reuse an address
        mix((uint64_t)(uintptr_t)db);
        mix((uint64_t)(uintptr_t)db->rows);
        mix((uint64_t)(uintptr_t)db->il);
        mix((uint64_t)db->N);
        mix((uint64_t)db->n);
        mix((uint64_t)specs[g].Q);
        mix((uint64_t)specs[g].w);
        mix((uint64_t)(specs[g].k * 2 + (plan.mixed_k[g] ? 1 : 0)));
        for (int v : knob_values(specs[g].kn)) mix((uint64_t)(uint32_t)v);
    }
    if (!ctx->use_graph && width <= 1) {
        if (int r = enqueue_all(ctx->stream)) return r;
    } else {
        HIPTRY(hipEventRecord(ctx->enter_ev, ctx->stream));
        HIPTRY(hipStreamWaitEvent(ctx->graph_stream, ctx->enter_ev, 0));
        if (ctx->use_graph) {
            if (!ctx->graph_exec || ctx->graph_sig != sig) {
                if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
                ctx->graph_exec = nullptr;
                hipGraph_t graph = nullptr;
                HIPTRY(hipStreamBeginCapture(ctx->graph_stream, hipStreamCaptureModeRelaxed));
                int r = enqueue_all(ctx->graph_stream);
                hipError_t e = hipStreamEndCapture(ctx->graph_stream, &graph);
                if (r) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return r;
                }
                if (e != hipSuccess) return fail(LBIMP_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
                e = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    ctx->graph_exec = nullptr;
                    return fail(LBIMP_E_DEVICE, "graph instantiation: %s", hipGetErrorString(e));
                }
                ctx->graph_sig = sig;
            }
            HIPTRY(hipGraphLaunch(ctx->graph_exec, ctx->graph_stream));
        } else {
            if (int r = enqueue_all(ctx->graph_stream)) return r;
        }
        HIPTRY(hipEventRecord(ctx->exit_ev, ctx->graph_stream));
        HIPTRY(hipStreamWaitEvent(ctx->stream, ctx->exit_ev, 0));
    }
    if (stats) {
        HIPTRY(hipStreamSynchronize(ctx->stream));
        for (int g = 0; g < G; ++g) {
            std::vector<int> h((size_t)specs[g].Q * kCounters);
            HIPTRY(hipMemcpy(h.data(), bufs[g].counters, sizeof(int) * h.size(), hipMemcpyDeviceToHost));
            const std::vector<int64_t> &ids = std::next(groups.begin(), g)->second;
            std::vector<long long> ht(bufs[g].tot ? (size_t)specs[g].Q * 3 : 0);
            if (bufs[g].tot)
                HIPTRY(hipMemcpy(ht.data(), bufs[g].tot, sizeof(long long) * ht.size(), hipMemcpyDeviceToHost));
            fill_stats(dims[g], specs[g].Q, h.data(), bufs[g].tot ? ht.data() : nullptr, ids.data(), stats);
        }
    }
    return LBIMP_OK;
}

int lbimp_autotune(lbimp_ctx *ctx, const lbimp_db *db, const float *queries, int64_t Q, int32_t w, int32_t p,
                   int32_t k, int32_t mode, int32_t *choice) {
    if (int r = check_ctx(ctx)) return r;
    if (!db) return fail(LBIMP_E_INVALID, "null database");
    if (db->device != ctx->device) return fail(LBIMP_E_INVALID, "database lives on another device");
    if (int r = check_search(Q, db->n, w, p, k, mode)) return r;
    if (Q == 0 || db->N == 0) return fail(LBIMP_E_INVALID, "nothing to tune (no queries or empty database)");
    if (!queries) return fail(LBIMP_E_INVALID, "null pointer");
    Knobs kn;
    if (int r = tune_search(ctx, db, queries, nullptr, nullptr, Q, band_of(db->n, w), p, k, mode, &kn)) return r;
    if (choice) {
        const std::array<int, kTuneKnobs> v = knob_values(kn);
        for (int i = 0; i < kTuneKnobs; ++i) choice[i] = v[i];
    }
    return LBIMP_OK;
}

int lbimp_ctx_copy_tuning(lbimp_ctx *dst, const lbimp_ctx *src) {
    if (!dst || !src) return fail(LBIMP_E_INVALID, "null context");
    if (dst->device != src->device) return fail(LBIMP_E_INVALID, "contexts on different devices");
    for (const auto &kv : src->tuned) dst->tuned[kv.first] = kv.second;
    return LBIMP_OK;
}

int lbimp_nn_search_ragged_workspace(lbimp_ctx *ctx, const lbimp_db *const *dbs, int32_t ndb,
                                     const int32_t *db_of, const int32_t *w, int64_t Q, int32_t p,
                                     const int32_t *k, int32_t mode, uint64_t *bytes) {
    if (int r = check_ctx(ctx)) return r;
    if (!bytes) return fail(LBIMP_E_INVALID, "null output pointer");
    *bytes = 0;
    if (Q < 0) return fail(LBIMP_E_INVALID, "negative query count");
    if (Q == 0) return LBIMP_OK;
    RaggedPlan plan;
    if (int r = plan_ragged(ctx, dbs, ndb, nullptr, db_of, w, Q, p, k, mode, nullptr, nullptr, plan)) return r;
    Carver cv{nullptr};
    plan.carve(cv);
    *bytes = reserve_size(cv.off);
    return LBIMP_OK;
}

int lbimp_ctx_workspace_bytes(lbimp_ctx *ctx, uint64_t *bytes) {
    if (!ctx || !bytes) return fail(LBIMP_E_INVALID, "null argument");
    *bytes = ctx->ws_cap;
    return LBIMP_OK;
}

}  // extern "C"
