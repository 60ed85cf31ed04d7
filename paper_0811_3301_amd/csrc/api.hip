// C-ABI layer: argument checks, workspace, stream ordering of the search stages.
//
// The staging follows Algorithms 2 and 3 (Lemire, arXiv:0811.3301, Sec. 7 and Sec. 8): envelope
// of the query, LB_Keogh of every candidate, LB_Improved of the survivors (Algorithm 3 only),
// DTW of what remains against the best-so-far.  The sequential scan's threshold b, which
// starts at infinity and shrinks in database order, is replaced by a seeded threshold: the
// DTW of the candidates with the smallest LB_Keogh, computed first.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace lbimp;
using u64 = unsigned long long;

static thread_local std::string g_err;

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
    bool lbi_pipeline = true;   // option "lbi_pipeline"
    bool dtw_low_latency = false;  // option "dtw_group_per_pair" (lbimp_dtw_band only)
    int sweep_shape = 0;           // option "sweep_shape"
    hipEvent_t ev[kStages + 1] = {};
};

struct lbimp_db {
    int device = 0;
    int64_t N = 0;
    int n = 0;
    float *rows = nullptr;  // [N][n] row-major copy (gathers of the second pass and the DTW)
    float4 *il = nullptr;   // interleaved tiles for the LB_Keogh sweep
};

static int persistent_grid(const lbimp_ctx *ctx) { return std::max(1, ctx->num_cu); }  // CUs; kernels size by occupancy

static int reserve(lbimp_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_cap) return LBIMP_OK;
    HIPTRY(hipStreamSynchronize(ctx->stream));
    if (ctx->ws) HIPTRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
    size_t cap = align_up(bytes + bytes / 8, 1 << 20);
    if (hipMalloc(&ctx->ws, cap) != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws = nullptr;
        return fail(LBIMP_E_NOMEM, "workspace allocation of %zu bytes failed", cap);
    }
    ctx->ws_cap = cap;
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
    if (p > 2) return fail(LBIMP_E_UNSUPPORTED, "exponent p = %d: only p = 1 and p = 2 are implemented", p);
    if (count > INT32_MAX) return fail(LBIMP_E_INVALID, "more than 2^31-1 series");
    return LBIMP_OK;
}

static int band_of(int32_t n, int32_t w) { return std::min<int32_t>(w, n - 1); }

static void stage_mark(lbimp_ctx *ctx, int i) {
    if (ctx->timing) (void)hipEventRecord(ctx->ev[i], ctx->stream);
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
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
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
        ctx->lbi_pipeline = value != 0;
    } else if (!strcmp(name, "dtw_group_per_pair")) {
        ctx->dtw_low_latency = value != 0;
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
    if (hipMalloc(&db->rows, rbytes) != hipSuccess || hipMalloc(&db->il, ibytes) != hipSuccess) {
        (void)hipGetLastError();
        lbimp_db_destroy(db);
        return fail(LBIMP_E_NOMEM, "database allocation failed");
    }
    if (N > 0) {
        hipError_t e = hipMemcpyAsync(db->rows, rows, sizeof(float) * (size_t)N * n, hipMemcpyDeviceToDevice,
                                      ctx->stream);
        if (e == hipSuccess) e = launch_pack(rows, N, n, db->il, ctx->stream);
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
    HIPTRY(launch_items_prefix(nullptr, N, 1, WL, prefix, s));
    QueryData qd{y, n, U, L, n};
    PairList pl{nullptr, 0, nullptr, N};
    HIPTRY(launch_lbi(p, x, (int64_t)N * n * 4, n, wb, qd, pl, S1, N, prefix, 1, ctr, persistent_grid(ctx), nullptr, nullptr, 0,
                      nullptr, lb, ctx->lbi_pipeline, s));
    return LBIMP_OK;
}

int lbimp_dtw_band(lbimp_ctx *ctx, const float *x, int64_t N, const float *y, int32_t n, int32_t w, int32_t p,
                   float *dist) {
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_shape(N, n, w, p)) return r;
    if (N == 0) return LBIMP_OK;
    if (!x || !y || !dist) return fail(LBIMP_E_INVALID, "null pointer");
    const int wb = band_of(n, w);
    Carver cv{nullptr};
    cv.take<long long>(2);
    cv.take<int>(1);
    cv.take<u64>(1);
    if (int r = reserve(ctx, cv.off)) return r;
    Carver c2{static_cast<char *>(ctx->ws)};
    long long *prefix = c2.take<long long>(2);
    int *ctr = c2.take<int>(1);
    u64 *nothr = c2.take<u64>(1);
    hipStream_t s = ctx->stream;
    HIPTRY(launch_fill_i32(ctr, 0, 1, s));
    HIPTRY(launch_fill_u64(nothr, kNoKey, 1, s));
    const bool ll = ctx->dtw_low_latency;
    HIPTRY(launch_items_prefix(nullptr, N, 1, dtw_batch(n, wb, ll), prefix, s));
    QueryData qd{y, n, nullptr, nullptr, 0};
    PairList pl{nullptr, 0, nullptr, N};
    // no threshold: nothing is abandoned and nothing appended (out_root receives every distance)
    HIPTRY(launch_dtw(p, x, n, wb, qd, pl, prefix, 1, ctr, persistent_grid(ctx), nullptr, nothr, nullptr, 0,
                      nullptr, nullptr, dist, false, ll, s));
    return LBIMP_OK;
}

int lbimp_nn_search(lbimp_ctx *ctx, const lbimp_db *db, const float *queries, int64_t Q, int32_t w, int32_t p,
                    int32_t k, int32_t mode, int64_t *idx, float *dist, lbimp_stats *stats) {
    if (int r = check_ctx(ctx)) return r;
    if (!db) return fail(LBIMP_E_INVALID, "null database");
    if (db->device != ctx->device) return fail(LBIMP_E_INVALID, "database lives on another device");
    if (int r = check_shape(Q, db->n, w, p)) return r;
    if (k < 1 || k > 64) return fail(LBIMP_E_INVALID, "k = %d outside [1, 64]", k);
    if (mode < LBIMP_MODE_BRUTE || mode > LBIMP_MODE_IMPROVED) return fail(LBIMP_E_INVALID, "unknown mode %d", mode);
    if (Q == 0) return LBIMP_OK;
    if (!queries || !idx || !dist) return fail(LBIMP_E_INVALID, "null pointer");

    const int n = db->n, n4 = (n + 3) / 4, ldq = n4 * 4;
    const int64_t N = db->N;
    const int wb = band_of(n, w);
    const int64_t Np = (N + 63) / 64 * 64;
    const int qg = sweep_query_group(ctx->sweep_shape, Q);
    const int64_t Qp = (Q + qg - 1) / qg * qg;
    const bool brute = mode == LBIMP_MODE_BRUTE;
    const bool improved = mode == LBIMP_MODE_IMPROVED;
    const int S = brute ? 0 : (int)std::min<int64_t>(std::max(ctx->seeds, k), N);
    const int WL = improved ? lbi_batch(n, wb) : 1;
    if (improved && WL == 0)
        return fail(LBIMP_E_UNSUPPORTED, "LB_Improved state for n = %d, w = %d exceeds LDS", n, wb);
    const int64_t ldres = brute ? N : S + N;
    hipStream_t s = ctx->stream;

    if (N == 0) {  // nothing to search: every slot is empty
        Carver cv{nullptr};
        cv.take<u64>((size_t)Q);
        cv.take<int>((size_t)Q);
        if (int r = reserve(ctx, cv.off)) return r;
        Carver c2{static_cast<char *>(ctx->ws)};
        u64 *res = c2.take<u64>((size_t)Q);
        int *rescnt = c2.take<int>((size_t)Q);
        HIPTRY(launch_fill_i32(rescnt, 0, Q, s));
        HIPTRY(launch_finalize_k(res, 1, rescnt, Q, k, p, idx, dist, s));
        if (stats) {
            HIPTRY(hipStreamSynchronize(s));
            for (int64_t q = 0; q < Q; ++q) stats[q] = lbimp_stats{0, 0, 0, 0, 0, 0};
        }
        return LBIMP_OK;
    }

    // ---- workspace layout
    // Seeds come from the per-wave minima of the sweep once there are enough of them.
    const int64_t nw = sweep_waves(ctx->sweep_shape, N, Q);
    const bool seeds_from_minima = !brute && nw >= 4 * (int64_t)kMaxSeeds;
    auto layout = [&](Carver &c, float *&Ue, float *&Le, float *&S1, int *&seeds, u64 *&best, u64 *&thr, u64 *&res,
                      int *&list1, int *&list2, int *&counters, long long *&prefix, u64 *&wmin) {
        Ue = c.take<float>((size_t)Qp * ldq);
        Le = c.take<float>((size_t)Qp * ldq);
        S1 = brute ? nullptr : c.take<float>((size_t)Q * Np);
        seeds = brute ? nullptr : c.take<int>((size_t)Q * std::max(S, 1));
        best = c.take<u64>((size_t)Q);
        thr = c.take<u64>((size_t)Q);
        res = k > 1 ? c.take<u64>((size_t)Q * ldres) : nullptr;
        list1 = brute ? nullptr : c.take<int>((size_t)Q * N);
        list2 = improved ? c.take<int>((size_t)Q * N) : nullptr;
        counters = c.take<int>((size_t)Q * 4 + 8);  // cnt1, cnt2, rescnt, abandoned, item counters
        prefix = c.take<long long>((size_t)Q + 1);
        wmin = seeds_from_minima ? c.take<u64>((size_t)Q * nw) : nullptr;
    };
    float *Ue, *Le, *S1;
    int *seeds, *list1, *list2, *counters;
    u64 *best, *thr, *res, *wmin;
    long long *prefix;
    {
        Carver cv{nullptr};
        layout(cv, Ue, Le, S1, seeds, best, thr, res, list1, list2, counters, prefix, wmin);
        if (int r = reserve(ctx, cv.off)) return r;
        Carver c2{static_cast<char *>(ctx->ws)};
        layout(c2, Ue, Le, S1, seeds, best, thr, res, list1, list2, counters, prefix, wmin);
    }
    int *cnt1 = counters, *cnt2 = counters + Q, *rescnt = counters + 2 * Q, *abandoned = counters + 3 * Q;
    int *ctr = counters + 4 * Q;
    const int grid = persistent_grid(ctx);  // compute units: each persistent kernel sizes its grid by occupancy
    const u64 *T = k == 1 ? best : thr;  // pruning threshold keys of the two passes
    QueryData qd{queries, n, Ue, Le, ldq};

    ctx->timed_valid = false;
    stage_mark(ctx, 0);
    HIPTRY(launch_fill_i32(counters, 0, Q * 4 + 8, s));
    HIPTRY(launch_fill_u64(best, kNoKey, Q, s));
    HIPTRY(launch_fill_u64(thr, kNoKey, Q, s));
    HIPTRY(launch_envelope(queries, Q, Qp, n, wb, Ue, Le, ldq, s));
    stage_mark(ctx, 1);

    if (brute) {
        for (int i = 2; i <= 5; ++i) stage_mark(ctx, i);
        stage_mark(ctx, 6);
        HIPTRY(launch_items_prefix(nullptr, N, Q, dtw_batch(n, wb, false), prefix, s));
        PairList all{nullptr, 0, nullptr, N};
        HIPTRY(launch_dtw(p, db->rows, n, wb, qd, all, prefix, Q, ctr + 0, grid, k == 1 ? best : nullptr,
                          k == 1 ? nullptr : thr, res, ldres, rescnt, nullptr, nullptr, false, false, s));
    } else {
        // pass 1: LB_Keogh of every candidate (Algorithm 2/3, first bound)
        HIPTRY(launch_lbk_sweep(p, ctx->sweep_shape, db->il, N, n4, reinterpret_cast<float4 *>(Ue), reinterpret_cast<float4 *>(Le),
                                n4, Q, S1, Np, true, false, wmin, s));
        stage_mark(ctx, 2);
        HIPTRY(launch_select_seeds(S1, Np, N, Q, S, wmin, nw, seeds, s));
        stage_mark(ctx, 3);
        // Seeds: few pairs per query on the critical path, so a group of lanes per pair (low
        // latency); they run to completion, their DTWs finishing together.
        HIPTRY(launch_items_prefix(nullptr, S, Q, dtw_batch(n, wb, true), prefix, s));
        PairList sp{seeds, S, nullptr, S};
        HIPTRY(launch_dtw(p, db->rows, n, wb, qd, sp, prefix, Q, ctr + 0, grid, k == 1 ? best : nullptr,
                          k == 1 ? nullptr : thr, res, ldres, rescnt, abandoned, nullptr, false, true, s));
        if (k > 1) HIPTRY(launch_kth_key(res, ldres, rescnt, Q, k, thr, s));
        stage_mark(ctx, 4);
        HIPTRY(launch_compact(S1, Np, N, Q, T, list1, N, cnt1, s));
        stage_mark(ctx, 5);
        PairList dl{list1, N, cnt1, 0};
        if (improved) {  // pass 2: LB_Improved of the survivors (Algorithm 3)
            HIPTRY(launch_items_prefix(cnt1, 0, Q, WL, prefix, s));
            HIPTRY(launch_lbi(p, db->rows, (int64_t)N * n * 4, n, wb, qd, dl, S1, Np, prefix, Q, ctr + 1, grid, T,
                              list2, N, cnt2, nullptr, ctx->lbi_pipeline, s));
            dl = PairList{list2, N, cnt2, 0};
        }
        stage_mark(ctx, 6);
        HIPTRY(launch_items_prefix(dl.cnt, 0, Q, dtw_batch(n, wb, false), prefix, s));
        HIPTRY(launch_dtw(p, db->rows, n, wb, qd, dl, prefix, Q, ctr + 2, grid, k == 1 ? best : nullptr,
                          k == 1 ? nullptr : thr, res, ldres, rescnt, abandoned, nullptr, true, false, s));
    }
    stage_mark(ctx, 7);
    if (k == 1)
        HIPTRY(launch_finalize1(best, Q, p, idx, dist, s));
    else
        HIPTRY(launch_finalize_k(res, ldres, rescnt, Q, k, p, idx, dist, s));
    stage_mark(ctx, 8);
    ctx->timed_valid = ctx->timing;

    if (stats) {
        std::vector<int> h((size_t)Q * 4);
        HIPTRY(hipMemcpyAsync(h.data(), counters, sizeof(int) * h.size(), hipMemcpyDeviceToHost, s));
        HIPTRY(hipStreamSynchronize(s));
        for (int64_t q = 0; q < Q; ++q) {
            lbimp_stats &st = stats[q];
            st.candidates = N;
            st.seeded = S;
            st.dtw_abandoned = brute ? 0 : h[3 * Q + q];
            if (brute) {
                st.pruned_keogh = st.pruned_improved = 0;
                st.dtw_started = N;
            } else {
                const int64_t c1 = h[q], c2 = improved ? h[Q + q] : c1;
                st.pruned_keogh = N - S - c1;
                st.pruned_improved = c1 - c2;
                st.dtw_started = S + c2;
            }
        }
    }
    return LBIMP_OK;
}

}  // extern "C"
