/* The C oracle under AddressSanitizer and UBSan: every function on small seeded inputs over
 * edge shapes (n = 1, bands 0, 1, n - 1 and wider than the series, k above N, an empty
 * database), p = 1, 2 and infinity (0 here).  Memory errors fail the run; the checks are the
 * orderings the bounds must respect and the counts of the sequential search. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_set_num_threads(int threads);
void orc_envelope(const double *y, int n, int w, double *U, double *L);
double orc_lb_keogh_pow(const double *x, const double *U, const double *L, int n, int p);
double orc_lb_improved_pow(const double *x, const double *y, const double *U, const double *L, int n, int w, int p,
                           double *scratch);
double orc_dtw_pow(const double *x, const double *y, int n, int w, int p);
void orc_dtw_pow_many(const double *X, int64_t N, const double *y, int n, int w, int p, double *out);
void orc_lb_many(const double *X, int64_t N, const double *y, int n, int w, int p, double *s1, double *s2);
void orc_nn_bruteforce(const double *DB, int64_t N, const double *Qs, int64_t nq, int n, int w, int p, int k,
                       int64_t *idx, double *dist);
void orc_nn_sequential_many(const double *DB, int64_t N, const double *Qs, int64_t nq, int n, int w, int p,
                            int improved, int64_t *best_idx, double *best_pow, int64_t *counters);

static int failures = 0;
#define CHECK(c, ...)                                              \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "FAILED line %d: %s: ", __LINE__, #c); \
            fprintf(stderr, __VA_ARGS__);                          \
            fprintf(stderr, "\n");                                 \
            ++failures;                                            \
        }                                                          \
    } while (0)

static uint64_t s = 0x9e3779b97f4a7c15ull;
static double unif(void) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return (double)(s >> 11) / 9007199254740992.0 - 0.5;
}

int main(void) {
    orc_set_num_threads(2);
    const int ns[] = {1, 2, 7, 33};
    const int ps[] = {1, 2, 0};
    for (int in = 0; in < 4; ++in) {
        const int n = ns[in];
        const int ws[] = {0, 1, n - 1, n + 3};
        const int64_t N = 37, nq = 3;
        double *X = malloc(sizeof(double) * N * n), *Y = malloc(sizeof(double) * nq * n);
        for (int64_t i = 0; i < N * n; ++i) X[i] = unif();
        for (int64_t i = 0; i < nq * n; ++i) Y[i] = unif();
        double *U = malloc(sizeof(double) * n), *L = malloc(sizeof(double) * n), *scr = malloc(sizeof(double) * 3 * n);
        double *s1 = malloc(sizeof(double) * N), *s2 = malloc(sizeof(double) * N), *d = malloc(sizeof(double) * N);
        for (int iw = 0; iw < 4; ++iw)
            for (int ip = 0; ip < 3; ++ip) {
                const int w = ws[iw] < 0 ? 0 : ws[iw], p = ps[ip];
                orc_envelope(Y, n, w, U, L);
                orc_lb_many(X, N, Y, n, w, p, s1, s2);
                orc_dtw_pow_many(X, N, Y, n, w, p, d);
                for (int64_t c = 0; c < N; ++c) {
                    const double lk = orc_lb_keogh_pow(X + c * n, U, L, n, p);
                    const double li = orc_lb_improved_pow(X + c * n, Y, U, L, n, w, p, scr);
                    const double dt = orc_dtw_pow(X + c * n, Y, n, w, p);
                    CHECK(lk == s1[c] && li == s2[c] && dt == d[c], "n=%d w=%d p=%d c=%lld", n, w, p, (long long)c);
                    CHECK(lk <= li + 1e-12 && li <= dt * (1 + 1e-12) + 1e-12, "bounds out of order n=%d w=%d p=%d", n, w,
                          p);
                }
                for (int k = 1; k <= N + 2; k += 19) {
                    int64_t *idx = malloc(sizeof(int64_t) * nq * k);
                    double *dist = malloc(sizeof(double) * nq * k);
                    orc_nn_bruteforce(X, N, Y, nq, n, w, p, k, idx, dist);
                    for (int64_t q = 0; q < nq; ++q)
                        for (int r = 1; r < k && r < N; ++r)
                            CHECK(dist[q * k + r - 1] <= dist[q * k + r], "k-NN not sorted");
                    free(idx);
                    free(dist);
                }
                int64_t bi[3], cnt[9], bb[1];
                double bp[3], bd[1];
                for (int improved = 0; improved < 2; ++improved) {
                    orc_nn_sequential_many(X, N, Y, nq, n, w, p, improved, bi, bp, cnt);
                    orc_nn_bruteforce(X, N, Y, 1, n, w, p, 1, bb, bd);
                    CHECK(bp[0] == bd[0], "sequential search and brute force disagree n=%d w=%d p=%d", n, w, p);
                    for (int64_t q = 0; q < nq; ++q)
                        CHECK(cnt[3 * q] + cnt[3 * q + 1] + cnt[3 * q + 2] == N, "counts do not sum to N");
                }
            }
        orc_nn_bruteforce(X, 0, Y, 1, n, 1, 1, 2, (int64_t[2]){0}, (double[2]){0});  /* empty database */
        free(X), free(Y), free(U), free(L), free(scr), free(s1), free(s2), free(d);
    }
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle: all checks passed\n");
    return 0;
}
