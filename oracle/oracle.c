/*
 * oracle.c -- plain fp64 CPU oracle for banded DTW_p nearest-neighbour search.
 *
 * TEST INFRASTRUCTURE ONLY.  Used by the tests and by the benchmark's CPU
 * baseline; the device library never links or calls it, and it shares no code
 * with the device path.  It restates the same definitions as reference.py in C
 * so that brute force over large databases finishes in seconds.
 *
 * Exponent convention: p >= 1 is an integer; p == 0 stands for p = infinity.
 * "pow" values are sums of |.|^p (maxima for p = infinity).
 *
 * Definitions followed (Lemire, arXiv:0811.3301):
 *   envelope            Sec. 5, U_i = max_{|k-i|<=w} y_k, L_i = min (windows cut to the series)
 *   LB_Keogh            Sec. 7, ||x - H(x,y)||_p with H the projection onto the envelope of y
 *   LB_Improved         Sec. 8, LB_Keogh(x,y)^p + LB_Keogh(y, H(x,y))^p
 *   DTW_p               Sec. 4 recursion, written in prefix form (paths reversed)
 *   sequential search   Algorithms 2 and 3, b kept as a p-th power, strict "<" tests
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double pw(double d, int p) {
    d = fabs(d);
    if (p == 0 || p == 1) return d;
    if (p == 2) return d * d;
    double r = 1.0;
    for (int k = 0; k < p; ++k) r *= d;
    return r;
}

static double agg(double acc, double term, int p) { return p == 0 ? (term > acc ? term : acc) : acc + term; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops below (the benchmark times the oracle on one core and on all). */
void orc_set_num_threads(int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

/* Sec. 5: naive windowed max/min. */
void orc_envelope(const double *y, int n, int w, double *U, double *L) {
    for (int i = 0; i < n; ++i) {
        int lo = i - w < 0 ? 0 : i - w;
        int hi = i + w > n - 1 ? n - 1 : i + w;
        double mx = y[lo], mn = y[lo];
        for (int k = lo + 1; k <= hi; ++k) {
            if (y[k] > mx) mx = y[k];
            if (y[k] < mn) mn = y[k];
        }
        U[i] = mx;
        L[i] = mn;
    }
}

/* d(v, [lo, hi]) of the set-distance convention (Sec. 2). */
static double interval_dist(double v, double lo, double hi) {
    if (v > hi) return v - hi;
    if (v < lo) return lo - v;
    return 0.0;
}

/* Sec. 7: LB_Keogh_p(x,y)^p with (U, L) the envelope of y. */
double orc_lb_keogh_pow(const double *x, const double *U, const double *L, int n, int p) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc = agg(acc, pw(interval_dist(x[i], L[i], U[i]), p), p);
    return acc;
}

/* Sec. 8: LB_Improved_p(x,y)^p; scratch must hold 3n doubles.  For p = infinity the two
 * LB_Keogh terms combine by a maximum (Theorem 1 of Sec. 5 in its p = infinity form). */
double orc_lb_improved_pow(const double *x, const double *y, const double *U, const double *L, int n, int w, int p,
                           double *scratch) {
    double *xp = scratch, *Up = scratch + n, *Lp = scratch + 2 * n;
    for (int i = 0; i < n; ++i) {
        /* H(x,y)_i: U_i if x_i >= U_i, L_i if x_i <= L_i, else x_i */
        xp[i] = x[i] >= U[i] ? U[i] : (x[i] <= L[i] ? L[i] : x[i]);
    }
    orc_envelope(xp, n, w, Up, Lp);
    return agg(orc_lb_keogh_pow(x, U, L, n, p), orc_lb_keogh_pow(y, Up, Lp, n, p), p);
}

/* Sec. 4: D(i,j) = c(i,j) + min(D(i-1,j), D(i,j-1), D(i-1,j-1)), |i-j| <= w, D(-1,-1) = 0.
 * Two full-length rows; index j+1 holds column j, index 0 is the column j = -1. */
double orc_dtw_pow(const double *x, const double *y, int n, int w, int p) {
    if (n <= 0) return 0.0;
    if (w > n - 1) w = n - 1;
    double *prev = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *cur = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    for (int j = 0; j <= n; ++j) prev[j] = INFINITY;
    prev[0] = 0.0; /* the virtual cell (-1,-1) */
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= n; ++j) cur[j] = INFINITY;
        int lo = i - w < 0 ? 0 : i - w;
        int hi = i + w > n - 1 ? n - 1 : i + w;
        for (int j = lo; j <= hi; ++j) {
            double up = prev[j + 1], left = cur[j], diag = prev[j];
            double m = up < left ? up : left;
            if (diag < m) m = diag;
            double c = pw(x[i] - y[j], p);
            cur[j + 1] = p == 0 ? (c > m ? c : m) : c + m;
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    double r = prev[n];
    free(prev);
    free(cur);
    return r;
}

/* DTW of every database row against y (OpenMP over candidates). */
void orc_dtw_pow_many(const double *X, int64_t N, const double *y, int n, int w, int p, double *out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < N; ++c) out[c] = orc_dtw_pow(X + c * (int64_t)n, y, n, w, p);
}

/* LB_Keogh^p and LB_Improved^p of every row against one query. */
void orc_lb_many(const double *X, int64_t N, const double *y, int n, int w, int p, double *s1, double *s2) {
    double *U = (double *)malloc(sizeof(double) * (size_t)n);
    double *L = (double *)malloc(sizeof(double) * (size_t)n);
    orc_envelope(y, n, w, U, L);
#pragma omp parallel
    {
        double *scratch = (double *)malloc(sizeof(double) * 3 * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
            const double *x = X + c * (int64_t)n;
            if (s1) s1[c] = orc_lb_keogh_pow(x, U, L, n, p);
            if (s2) s2[c] = orc_lb_improved_pow(x, y, U, L, n, w, p, scratch);
        }
        free(scratch);
    }
    free(U);
    free(L);
}

/* Brute-force k-NN (the definition): every DTW, then the k smallest by (distance, index).
 * idx/dist are [nq][k]; dist holds pow-domain values.  Missing entries get -1 / inf. */
void orc_nn_bruteforce(const double *DB, int64_t N, const double *Qs, int64_t nq, int n, int w, int p, int k,
                       int64_t *idx, double *dist) {
    double *D = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int64_t q = 0; q < nq; ++q) {
        orc_dtw_pow_many(DB, N, Qs + q * (int64_t)n, n, w, p, D);
        for (int r = 0; r < k; ++r) {
            int64_t best = -1;
            for (int64_t c = 0; c < N; ++c) {
                int taken = 0;
                for (int s = 0; s < r; ++s) taken |= (idx[q * k + s] == c);
                if (taken) continue;
                if (best < 0 || D[c] < D[best]) best = c; /* strict: the smaller index wins a tie */
            }
            idx[q * k + r] = best;
            dist[q * k + r] = best < 0 ? INFINITY : D[best];
        }
    }
    free(D);
}

/* Algorithms 2 (improved == 0) and 3 (improved != 0), sequential over the database.
 * counters[0..2] = pruned by LB_Keogh, pruned by LB_Improved, DTW computed. */
void orc_nn_sequential(const double *DB, int64_t N, const double *y, int n, int w, int p, int improved,
                       int64_t *best_idx, double *best_pow, int64_t *counters) {
    if (w > n - 1) w = n - 1;
    double *U = (double *)malloc(sizeof(double) * (size_t)n);
    double *L = (double *)malloc(sizeof(double) * (size_t)n);
    double *xp = (double *)malloc(sizeof(double) * (size_t)n);
    double *Up = (double *)malloc(sizeof(double) * (size_t)n);
    double *Lp = (double *)malloc(sizeof(double) * (size_t)n);
    orc_envelope(y, n, w, U, L);
    double b = INFINITY;
    int64_t B = -1;
    counters[0] = counters[1] = counters[2] = 0;
    for (int64_t c = 0; c < N; ++c) {
        const double *x = DB + c * (int64_t)n;
        double beta = 0.0;
        for (int i = 0; i < n; ++i) {
            xp[i] = x[i];
            if (x[i] > U[i]) {
                beta = agg(beta, pw(x[i] - U[i], p), p);
                xp[i] = U[i];
            } else if (x[i] < L[i]) {
                beta = agg(beta, pw(L[i] - x[i], p), p);
                xp[i] = L[i];
            }
        }
        if (!(beta < b)) {
            counters[0]++;
            continue;
        }
        if (improved) {
            orc_envelope(xp, n, w, Up, Lp);
            for (int i = 0; i < n; ++i) beta = agg(beta, pw(interval_dist(y[i], Lp[i], Up[i]), p), p);
            if (!(beta < b)) {
                counters[1]++;
                continue;
            }
        }
        double t = orc_dtw_pow(x, y, n, w, p);
        counters[2]++;
        if (t < b) {
            b = t;
            B = c;
        }
    }
    *best_idx = B;
    *best_pow = b;
    free(U);
    free(L);
    free(xp);
    free(Up);
    free(Lp);
}

/* Sequential Algorithm 2/3 for many queries, one query per thread. */
void orc_nn_sequential_many(const double *DB, int64_t N, const double *Qs, int64_t nq, int n, int w, int p,
                            int improved, int64_t *best_idx, double *best_pow, int64_t *counters) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q)
        orc_nn_sequential(DB, N, Qs + q * (int64_t)n, n, w, p, improved, best_idx + q, best_pow + q, counters + 3 * q);
}
