// Host-logic checks of the library over the HIP stub: every entry point with valid and
// invalid arguments, ragged batches with and without autotuning (every p and mode), searches
// split into candidate chunks by a workspace bound, the allocation-free entry point (no
// allocation, refusal before any launch), and the invariants of the per-query statistics.
// Built with AddressSanitizer and UBSan, so any host memory error fails the run.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lbimp.h"

extern "C" long long hip_stub_launches();
extern "C" long long hip_stub_allocations();

static int failures = 0;

#define CHECK(cond, ...)                                                 \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "FAILED %s:%d: %s: ", __FILE__, __LINE__, #cond); \
            fprintf(stderr, __VA_ARGS__);                                \
            fprintf(stderr, "\n");                                       \
            ++failures;                                                  \
        }                                                                \
    } while (0)

#define OK(x)                                                                               \
    do {                                                                                    \
        const int r_ = (x);                                                                 \
        if (r_ != LBIMP_OK) {                                                               \
            fprintf(stderr, "FAILED %s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #x, r_, lbimp_last_error()); \
            exit(1);                                                                        \
        }                                                                                   \
    } while (0)

template <class T>
static T *dev(size_t count) {
    void *p = nullptr;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) exit(2);
    return static_cast<T *>(p);
}

static uint64_t ws_bytes(lbimp_ctx *ctx) {
    uint64_t b = 0;
    OK(lbimp_ctx_workspace_bytes(ctx, &b));
    return b;
}

// Every candidate is accounted for once: pruned by one of the passes, or its DTW started.
static void check_stats(const std::vector<lbimp_stats> &st, int64_t Q, int64_t N, const char *what) {
    for (int64_t q = 0; q < Q; ++q) {
        const lbimp_stats &s = st[q];
        CHECK(s.candidates == N, "%s q=%lld: candidates %lld", what, (long long)q, (long long)s.candidates);
        CHECK(s.pruned_pd + s.pruned_keogh + s.pruned_improved + s.dtw_started == N, "%s q=%lld: counts do not sum to N",
              what, (long long)q);
        CHECK(s.seeded >= 0 && s.seeded <= N && s.dtw_abandoned >= 0, "%s q=%lld", what, (long long)q);
    }
}

static void ragged_batches() {
    lbimp_ctx *ctx = nullptr;
    OK(lbimp_ctx_create(0, nullptr, &ctx));
    const int lengths[2] = {64, 200};
    const int64_t sizes[2] = {2500, 1500};
    lbimp_db *dbs[2];
    for (int i = 0; i < 2; ++i) OK(lbimp_db_create(ctx, dev<float>(sizes[i] * lengths[i]), sizes[i], lengths[i], &dbs[i]));
    const int Q = 40;
    std::vector<int32_t> db_of(Q), w(Q), k(Q);
    std::vector<int64_t> off(Q + 1, 0);
    unsigned s = 1;
    auto next = [&]() { return (s = s * 1103515245u + 12345u) >> 16; };
    for (int q = 0; q < Q; ++q) {
        db_of[q] = next() & 1;
        w[q] = db_of[q] == 0 ? (next() & 1 ? 6 : 13) : (next() & 1 ? 20 : 70);
        k[q] = 1 + next() % 3;
        off[q + 1] = off[q] + lengths[db_of[q]];
    }
    float *packed = dev<float>(off[Q]);
    int64_t *idx = dev<int64_t>(Q * 3);
    float *dist = dev<float>(Q * 3);
    std::vector<lbimp_stats> st(Q);
    uint64_t need = 0;
    OK(lbimp_nn_search_ragged_workspace(ctx, dbs, 2, db_of.data(), w.data(), Q, 1, k.data(), LBIMP_MODE_IMPROVED, &need));
    OK(lbimp_nn_search_ragged(ctx, dbs, 2, packed, off.data(), db_of.data(), w.data(), Q, 1, k.data(),
                              LBIMP_MODE_IMPROVED, idx, dist, st.data()));
    CHECK(ws_bytes(ctx) >= need, "ragged workspace %llu below the reported %llu", (unsigned long long)ws_bytes(ctx),
          (unsigned long long)need);
    for (int p : {1, 2, LBIMP_P_INF})
        for (int mode = LBIMP_MODE_BRUTE; mode <= LBIMP_MODE_IMPROVED; ++mode)
            for (int graph : {1, 0}) {
                OK(lbimp_ctx_set_option(ctx, "graph", graph));
                OK(lbimp_ctx_set_option(ctx, "lbi_buckets", graph));
                OK(lbimp_ctx_set_option(ctx, "autotune", 0));
                OK(lbimp_nn_search_ragged(ctx, dbs, 2, packed, off.data(), db_of.data(), w.data(), Q, p, k.data(), mode,
                                          idx, dist, st.data()));
                for (int q = 0; q < Q; ++q) check_stats({st[q]}, 1, sizes[db_of[q]], "ragged");
                OK(lbimp_ctx_set_option(ctx, "autotune", 1));
                for (int it = 0; it < 3; ++it)
                    OK(lbimp_nn_search_ragged(ctx, dbs, 2, packed, off.data(), db_of.data(), w.data(), Q, p, k.data(),
                                              mode, idx, dist, st.data()));
            }
    // a bounded workspace splits every group into chunks
    OK(lbimp_ctx_set_option(ctx, "workspace_limit", 1 << 16));
    OK(lbimp_nn_search_ragged(ctx, dbs, 2, packed, off.data(), db_of.data(), w.data(), Q, 2, k.data(),
                              LBIMP_MODE_IMPROVED, idx, dist, st.data()));
    for (int q = 0; q < Q; ++q) check_stats({st[q]}, 1, sizes[db_of[q]], "ragged chunked");
    // invalid batches are refused
    std::vector<int32_t> bad(db_of);
    bad[3] = 2;
    CHECK(lbimp_nn_search_ragged(ctx, dbs, 2, packed, off.data(), bad.data(), w.data(), Q, 1, k.data(), 2, idx, dist,
                                 nullptr) == LBIMP_E_INVALID, "database index out of range accepted");
    std::vector<int64_t> badoff(off);
    badoff[5] += 1;
    CHECK(lbimp_nn_search_ragged(ctx, dbs, 2, packed, badoff.data(), db_of.data(), w.data(), Q, 1, k.data(), 2, idx,
                                 dist, nullptr) == LBIMP_E_INVALID, "wrong query length accepted");
    std::vector<int32_t> badk(k);
    badk[0] = 65;
    CHECK(lbimp_nn_search_ragged(ctx, dbs, 2, packed, off.data(), db_of.data(), w.data(), Q, 1, badk.data(), 2, idx,
                                 dist, nullptr) == LBIMP_E_INVALID, "k = 65 accepted");
    for (auto *d : dbs) lbimp_db_destroy(d);
    lbimp_ctx_destroy(ctx);
}

static void chunked_and_noalloc() {
    const int64_t N = 20000, Q = 64;
    const int n = 128;
    for (int64_t limit : {(int64_t)0, (int64_t)8 << 20, (int64_t)1 << 20}) {
        lbimp_ctx *ctx = nullptr;
        OK(lbimp_ctx_create(0, nullptr, &ctx));
        lbimp_db *db = nullptr;
        OK(lbimp_db_create(ctx, dev<float>(N * n), N, n, &db));
        const float *qs = dev<float>(Q * n);
        int64_t *idx = dev<int64_t>(Q * 8);
        float *dist = dev<float>(Q * 8);
        std::vector<lbimp_stats> st(Q);
        OK(lbimp_ctx_set_option(ctx, "workspace_limit", limit));
        for (int k : {1, 3})
            for (int mode = LBIMP_MODE_BRUTE; mode <= LBIMP_MODE_IMPROVED; ++mode)
                for (int pd : {0, 1, 2})
                    for (int p : {1, 2, LBIMP_P_INF}) {
                        OK(lbimp_ctx_set_option(ctx, "pd_prefilter", pd));
                        OK(lbimp_ctx_set_option(ctx, "lbi_buckets", ((p & 3) + pd + k) & 1));
                        OK(lbimp_ctx_set_option(ctx, "lbi_pipeline", ((p & 3) + mode) & 1));
                        OK(lbimp_ctx_set_option(ctx, "dtw_split", (mode + k + pd) & 1));
                        OK(lbimp_ctx_set_option(ctx, "dtw_pool_slots", pd == 1 ? 64 : 1 << 18));
                        OK(lbimp_nn_search(ctx, db, qs, Q, 13, p, k, mode, idx, dist, st.data()));
                        check_stats(st, Q, N, "chunked");
                        const long long a0 = hip_stub_allocations();
                        OK(lbimp_nn_search_noalloc(ctx, db, qs, Q, 13, p, k, mode, idx, dist));
                        CHECK(hip_stub_allocations() == a0, "the allocation-free entry point allocated");
                    }
        // 8 MiB is above the smallest chunk's workspace for 64 queries, so it is met
        if (limit == (8 << 20))
            CHECK(ws_bytes(ctx) <= (uint64_t)limit + limit / 8 + (1 << 20), "workspace %llu above the bound",
                  (unsigned long long)ws_bytes(ctx));
        OK(lbimp_ctx_set_option(ctx, "pd_fine", 1));
        OK(lbimp_db_pd_bound(ctx, db, qs, qs, Q, 2, dev<float>(Q * N)));
        OK(lbimp_ctx_set_option(ctx, "pd_fine", 0));
        int32_t choice[LBIMP_TUNE_KNOBS];
        OK(lbimp_autotune(ctx, db, qs, Q, 13, 1, 3, LBIMP_MODE_IMPROVED, choice));
        OK(lbimp_ctx_set_option(ctx, "autotune", 1));
        OK(lbimp_nn_search(ctx, db, qs, Q, 40, 2, 2, LBIMP_MODE_IMPROVED, idx, dist, st.data()));
        check_stats(st, Q, N, "autotuned");
        lbimp_db_destroy(db);
        lbimp_ctx_destroy(ctx);
    }
    // a search too large for the fixed scratch is refused before anything is enqueued
    lbimp_ctx *ctx = nullptr;
    OK(lbimp_ctx_create(0, nullptr, &ctx));
    lbimp_db *db = nullptr;
    const int64_t NB = 40000;
    OK(lbimp_db_create(ctx, dev<float>(NB * 16), NB, 16, &db));
    const int64_t QB = 4096;
    const float *qs = dev<float>(QB * 16);
    int64_t *idx = dev<int64_t>(QB * 64);
    float *dist = dev<float>(QB * 64);
    const long long l0 = hip_stub_launches(), a0 = hip_stub_allocations();
    CHECK(lbimp_nn_search_noalloc(ctx, db, qs, QB, 2, 1, 64, LBIMP_MODE_IMPROVED, idx, dist) == LBIMP_E_NOMEM,
          "oversized allocation-free search accepted");
    CHECK(hip_stub_launches() == l0 && hip_stub_allocations() == a0, "work enqueued before the refusal");
    lbimp_db_destroy(db);
    lbimp_ctx_destroy(ctx);
}

static void invalid_arguments() {
    lbimp_ctx *ctx = nullptr;
    CHECK(lbimp_ctx_create(3, nullptr, &ctx) == LBIMP_E_INVALID, "device 3 of 1 accepted");
    OK(lbimp_ctx_create(0, nullptr, &ctx));
    lbimp_db *db = nullptr;
    const float *x = dev<float>(100 * 10);
    OK(lbimp_db_create(ctx, x, 100, 10, &db));
    int64_t *idx = dev<int64_t>(64);
    float *dist = dev<float>(64);
    CHECK(lbimp_nn_search(ctx, db, x, 1, -1, 1, 1, 2, idx, dist, nullptr) == LBIMP_E_INVALID, "w < 0 accepted");
    CHECK(lbimp_nn_search(ctx, db, x, 1, 3, 3, 1, 2, idx, dist, nullptr) == LBIMP_E_UNSUPPORTED, "p = 3 accepted");
    CHECK(lbimp_nn_search(ctx, db, x, 1, 3, 1, 0, 2, idx, dist, nullptr) == LBIMP_E_INVALID, "k = 0 accepted");
    CHECK(lbimp_nn_search(ctx, db, x, 1, 3, 1, 1, 7, idx, dist, nullptr) == LBIMP_E_INVALID, "mode 7 accepted");
    CHECK(lbimp_nn_search(ctx, db, nullptr, 1, 3, 1, 1, 2, idx, dist, nullptr) == LBIMP_E_INVALID, "null queries");
    CHECK(lbimp_nn_search(ctx, nullptr, x, 1, 3, 1, 1, 2, idx, dist, nullptr) == LBIMP_E_INVALID, "null database");
    CHECK(lbimp_ctx_set_option(ctx, "no such option", 1) == LBIMP_E_INVALID, "unknown option accepted");
    CHECK(lbimp_ctx_set_option(ctx, "workspace_limit", -1) == LBIMP_E_INVALID, "negative bound accepted");
    CHECK(lbimp_ctx_set_option(ctx, "seeds", 65) == LBIMP_E_INVALID, "65 seeds accepted");
    CHECK(lbimp_ctx_set_option(ctx, "pd_prefilter", 3) == LBIMP_E_INVALID, "pass-0 form 3 accepted");
    CHECK(lbimp_ctx_set_option(ctx, "dtw_pool_slots", -1) == LBIMP_E_INVALID, "negative pool accepted");
    OK(lbimp_ctx_set_option(ctx, "pd_fine", 1));
    CHECK(lbimp_db_pd_bound(ctx, db, x, x, 1, 1, dev<float>(100)) == LBIMP_E_UNSUPPORTED,
          "fine cover accepted for n = 10");
    OK(lbimp_ctx_set_option(ctx, "pd_fine", 0));
    CHECK(lbimp_ctx_set_option(ctx, "lbi_pipeline", 2) == LBIMP_E_INVALID, "pipeline depth 2 accepted");
    // k above N: every slot past the N neighbours is empty, not an error
    OK(lbimp_nn_search(ctx, db, x, 1, 3, 1, 64, 2, idx, dist, nullptr));
    // an empty database
    lbimp_db *empty = nullptr;
    OK(lbimp_db_create(ctx, x, 0, 10, &empty));
    std::vector<lbimp_stats> st(2);
    OK(lbimp_nn_search(ctx, empty, x, 2, 3, 1, 2, 2, idx, dist, st.data()));
    CHECK(st[0].candidates == 0 && st[1].dtw_started == 0, "stats of an empty database");
    lbimp_db_destroy(empty);
    lbimp_db_destroy(db);
    lbimp_ctx_destroy(ctx);
}

int main() {
    invalid_arguments();
    ragged_batches();
    chunked_and_noalloc();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("host logic: all checks passed (%lld launches)\n", hip_stub_launches());
    return 0;
}
