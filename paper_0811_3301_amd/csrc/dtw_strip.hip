// Lane-per-pair banded DTW_p (Sec. 4 of Lemire, arXiv:0811.3301) for bands too wide to keep
// a whole band row in registers.  The rows of the matrix are cut into strips of C rows; a
// lane holds C cells of one column of its strip in registers, with the C values x_i of its
// candidate, and walks the strip's band columns left to right.  The last row of a strip is
// written, one value per column, to a ring in global memory (one per wave) and read back as
// the row above by the next strip, which keeps the recursion exact:
//   D(i, j) = c(i, j) + min(D(i-1, j-1), D(i-1, j), D(i, j-1)),  D(-1,-1) = 0,
// with c = |x_i - y_j|^p and cells |i - j| > w at +inf.
//
// Strip geometry.  A strip of rows [I0, I0+C) meets the band in columns [I0-w, I0+C-1+w]:
// a left phase of C columns where column u holds rows 0..u (the rest lie below the band),
// a middle where every row is in the band, and a right phase of C columns where column u
// holds rows u..C-1 (the rest lie above it).  Every strip sweeps that whole range, columns
// outside [0, n) included: they read y = -inf, so their cells cost +inf, the phases always
// sit at the same offsets and their out-of-band cells are skipped at compile time.  Strips
// are aligned so the last one ends at row n-1; the first may start above row 0 (rows i < 0
// hold x = +inf and its row -1 carries D(-1,-1) = 0) and starts at column 0 with its middle
// (it has no left phase when w >= C).  Requires w >= C.
// Early abandoning: every path crosses each row, so after a strip the minimum of its last
// row over the band bounds the result.
#include <algorithm>
#include <climits>

#include "device_common.h"

namespace lbimp {

enum StripPhase { kLeft = 0, kMid = 1, kRight = 2 };

// Columns j..j+3 in skewed order: step s updates row r = s - t of column t, interleaving
// four serial chains.  When (r, t) runs, R[r] holds column t-1 at row r (left), R[r-1]
// holds column t at row r-1 (up) and dg[t] the left value of the row above (diagonal); the
// row above the strip comes from tc (this column) and tprev (the column before).  U0 is the
// phase offset of column 0 of the group.
template <int P, int C, int PH, int U0>
__device__ __forceinline__ void strip_cols4(float (&R)[C], const float (&X)[C], const float (&yv)[4],
                                            const float (&tc)[4], float tprev, float (&out)[4]) {
    float dg[4] = {tprev, tc[0], tc[1], tc[2]};
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t] = kInf;
#pragma unroll
    for (int s = 0; s < C + 3; ++s) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int r = s - t;
            const int u = U0 + t;
            if (r < 0 || r >= C) continue;
            if (PH == kLeft && r > u) continue;  // below the band: stays +inf from the strip start
            const float left = R[r];
            if (PH == kRight && r < u) {  // above the band: not computed, R[r] keeps the column before
                dg[t] = left;
                continue;
            }
            const float up = (r == 0) ? tc[t] : ((PH == kRight && r == u) ? kInf : R[r - 1]);
            const float m = __builtin_fminf(__builtin_fminf(left, up), dg[t]);
            const float d = X[r] - yv[t];
            const float v = pacc<P>(m, d);
            R[r] = v;
            dg[t] = left;
            if (r == C - 1) out[t] = v;
        }
    }
}

// The rows of R computed so far must exist here: the left phase stores only +inf to the ring
// (its last row lies below the band), so without this use the compiler sinks the arithmetic of
// every left group past the loads of the later ones and keeps all of them live at once.
template <int C, int ROWS>
__device__ __forceinline__ void pin_rows(const float (&R)[C]) {
#pragma unroll
    for (int r = 0; r < (ROWS < C ? ROWS : C); ++r) asm volatile("" ::"v"(R[r]));
}

// One middle column (every row in the band).
template <int P, int C>
__device__ __forceinline__ float strip_col1(float (&R)[C], const float (&X)[C], float y, float tc, float tprev) {
    float dg = tprev, up = tc;
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const float left = R[r];
        const float m = __builtin_fminf(__builtin_fminf(left, up), dg);
        const float d = X[r] - y;
        const float v = pacc<P>(m, d);
        R[r] = v;
        dg = left;
        up = v;
    }
    return R[C - 1];
}

// Four waves per SIMD need at most 128 VGPRs: the plain variant is held to that (the few values
// that do not fit are per-item setup, spilled outside the column loops).  The variant with the
// LB_Keogh-tail bound keeps U, L reads and its sums and stays at three.
template <int P, int C, bool CASCADE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(CASCADE ? 3 : 4, 8)))
void k_dtw_strip(DtwArgs a, int w, float *__restrict__ ring_base, int rb_log2) {
    extern __shared__ float ypad[];  // ypad[j + w + 4] = y[j] for 0 <= j < n, -inf elsewhere; then U, L
    const int lane = threadIdx.x;
    const int n = a.n;
    const int yoff = w + 4;
    const int plen = n + 2 * w + 8;
    float *sU = ypad + plen, *sL = sU + n;
    constexpr bool cascade = CASCADE;  // a.S1 is set exactly for this instantiation
    const float shrink = cascade_shrink(n);
    const int rmask = (1 << rb_log2) - 1;
    // this wave's ring (a uniform base); slot j of lane l at ring[(j & rmask) * 64 + l], indexed
    // with 32-bit offsets so each access needs one offset register
    float *ring = ring_base + ((size_t)blockIdx.x << rb_log2) * 64;
    auto rslot = [&](int j) { return (unsigned)(((j & rmask) << 6) | lane); };
    const int S = (n + C - 1) / C;
    const int I00 = n - S * C;  // first row of the first strip (<= 0)
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(a.pl, a.prefix, a.Q, 64);
    while (items.get(q, b)) {
        if (q != cur_q) {
            __syncthreads();
            const float *y = a.qd.Y + q * a.qd.ldy;
            stage_lds(ypad, plen, [&](int t) {
                const int j = t - yoff;
                return (j >= 0 && j < n) ? y[j] : -kInf;
            });
            if constexpr (cascade) {
                stage_lds(sU, n, [&](int t) { return a.qd.U[q * a.qd.ldq + t]; });
                stage_lds(sL, n, [&](int t) { return a.qd.L[q * a.qd.ldq + t]; });
            }
            __syncthreads();
            cur_q = q;
        }
        const long long jj = b * 64 + lane;
        const int cl = jj < pair_count(a.pl, q, items.bk) ? pair_cand(a.pl, q, jj, items.bk) : -1;
        bool active = cl >= 0;
        const int c = active ? cl : 0;
        const float *x = a.rows + (int64_t)c * n;
        const u64 *tq = a.tkeys + q;
        int stopped = 0;
        float fin = kInf;
        float s1v = 0.f;
        if constexpr (cascade) s1v = active ? a.S1[q * a.ldS + c] : 0.f;  // S1 may be a chunk's shifted base
        float done = 0.f;  // LB_Keogh^p terms of the rows already computed
        for (int s = 0; s < S; ++s) {
            const int I0 = I00 + s * C;
            float X[C], R[C];
            const int rv = -1 - I0;  // row -1 inside the first strip, else < 0
#pragma unroll
            for (int r = 0; r < C; ++r) {
                X[r] = (I0 + r >= 0) ? x[I0 + r] : kInf;
                R[r] = (r == rv) ? 0.f : kInf;
            }
            const u64 th = __hip_atomic_load(tq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // the row above the strip, D(I0-1, j), lies in the ring for 0 <= j <= jread
            const int jread = s > 0 ? min(n - 1, I0 - 1 + w) : -1;
            auto above = [&](int j) { return (j >= 0 && j <= jread) ? ring[rslot(j)] : kInf; };
            float cmin = kInf;
            int jn = INT_MIN;  // columns [jn, jn+4) are prefetched in tn
            float tn[4];
            auto fetch = [&](int j) {
#pragma unroll
                for (int t = 0; t < 4; ++t) tn[t] = above(j + t);
                jn = j;
            };
            auto finish4 = [&](int j, const float (&out)[4], bool track) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    ring[rslot(j + t)] = out[t];
                    if (track) cmin = fminf(cmin, out[t]);
                }
            };
            float tprev;
            int j;
            if (s == 0) {
                tprev = (I0 == 0) ? 0.f : kInf;  // D(I0-1, -1): the virtual cell when the strip starts at row 0
                j = 0;
            } else {
                j = I0 - w;
                tprev = above(j - 1);
                // left phase: C columns, column u holds rows 0..u
                fetch(j);
#define LBIMP_STRIP_LEFT(G)                                                 \
    if constexpr (4 * (G) < C) {                                            \
        float tc[4], yv[4], out[4];                                         \
        _Pragma("unroll") for (int t = 0; t < 4; ++t) {                     \
            tc[t] = tn[t];                                                  \
            yv[t] = ypad[yoff + j + t];                                     \
        }                                                                   \
        fetch(j + 4);                                                       \
        strip_cols4<P, C, kLeft, 4 * (G)>(R, X, yv, tc, tprev, out);        \
        pin_rows<C, 4 * (G) + 4>(R);                                        \
        finish4(j, out, 4 * (G) + 4 == C);                                  \
        tprev = tc[3];                                                      \
        j += 4;                                                             \
    }
                LBIMP_STRIP_LEFT(0) LBIMP_STRIP_LEFT(1) LBIMP_STRIP_LEFT(2) LBIMP_STRIP_LEFT(3)
                LBIMP_STRIP_LEFT(4) LBIMP_STRIP_LEFT(5) LBIMP_STRIP_LEFT(6) LBIMP_STRIP_LEFT(7)
                LBIMP_STRIP_LEFT(8) LBIMP_STRIP_LEFT(9) LBIMP_STRIP_LEFT(10) LBIMP_STRIP_LEFT(11)
                LBIMP_STRIP_LEFT(12) LBIMP_STRIP_LEFT(13) LBIMP_STRIP_LEFT(14) LBIMP_STRIP_LEFT(15)
#undef LBIMP_STRIP_LEFT
            }
            // middle: columns j .. I0+w-1; the odd columns first, then groups of four
            const int jr = I0 + w;  // first column of the right phase
            for (; (jr - j) & 3; ++j) {
                const float tc1 = above(j);
                const float o = strip_col1<P, C>(R, X, ypad[yoff + j], tc1, tprev);
                ring[rslot(j)] = o;
                cmin = fminf(cmin, o);
                if (j == n - 1) fin = o;
                tprev = tc1;
            }
            for (; j < jr; j += 4) {
                float tc[4], yv[4], out[4];
                if (jn != j) fetch(j);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    tc[t] = tn[t];
                    yv[t] = ypad[yoff + j + t];
                }
                fetch(j + 4);
                strip_cols4<P, C, kMid, 0>(R, X, yv, tc, tprev, out);
                finish4(j, out, true);
                if (j <= n - 1 && n - 1 < j + 4) {  // select, not an indexed (scratch) array
                    const int o = n - 1 - j;
                    fin = o == 0 ? out[0] : o == 1 ? out[1] : o == 2 ? out[2] : out[3];
                }
                tprev = tc[3];
            }
            // right phase: C columns, column u holds rows u..C-1
            if (jn != j) fetch(j);
#define LBIMP_STRIP_RIGHT(G)                                                \
    if constexpr (4 * (G) < C) {                                            \
        float tc[4], yv[4], out[4];                                         \
        _Pragma("unroll") for (int t = 0; t < 4; ++t) {                     \
            tc[t] = tn[t];                                                  \
            yv[t] = ypad[yoff + j + t];                                     \
        }                                                                   \
        fetch(j + 4);                                                       \
        strip_cols4<P, C, kRight, 4 * (G)>(R, X, yv, tc, tprev, out);       \
        finish4(j, out, true);                                              \
        tprev = tc[3];                                                      \
        j += 4;                                                             \
    }
            LBIMP_STRIP_RIGHT(0) LBIMP_STRIP_RIGHT(1) LBIMP_STRIP_RIGHT(2) LBIMP_STRIP_RIGHT(3)
            LBIMP_STRIP_RIGHT(4) LBIMP_STRIP_RIGHT(5) LBIMP_STRIP_RIGHT(6) LBIMP_STRIP_RIGHT(7)
            LBIMP_STRIP_RIGHT(8) LBIMP_STRIP_RIGHT(9) LBIMP_STRIP_RIGHT(10) LBIMP_STRIP_RIGHT(11)
            LBIMP_STRIP_RIGHT(12) LBIMP_STRIP_RIGHT(13) LBIMP_STRIP_RIGHT(14) LBIMP_STRIP_RIGHT(15)
#undef LBIMP_STRIP_RIGHT
            if (a.abandon && s + 1 < S) {
                if constexpr (cascade) {
#pragma unroll
                    for (int r = 0; r < C; ++r)
                        if (I0 + r >= 0) done += lbk_term<P>(X[r], sL[I0 + r], sU[I0 + r]);
                    cmin = cascade_bound(cmin, s1v, done, shrink);
                }
                if (active && make_key(cmin, c) >= th) {
                    active = false;
                    stopped = 1;
                }
                if (!__any(active)) break;
            }
        }
        publish<P>(active, fin, c, q, a.best, a.thr, a.res, a.ldres, a.rescnt, a.out_root);
        if (a.abandoned) {
            const u64 m = __ballot(stopped != 0);
            if (lane == 0 && m) atomicAdd(&a.abandoned[q], __popcll(m));
        }
    }
}

constexpr int kStripRows = 32;

static int ring_log2(int w) {
    int l = 6;
    while ((1 << l) < 2 * w + kStripRows + 8) ++l;
    return l;
}

// LDS: the padded query, then (with the tighter abandon bound) its envelope U, L.
static size_t strip_lds(int n, int w, bool cascade = false) {
    return sizeof(float) * ((size_t)n + 2 * (size_t)w + 8 + (cascade ? 2 * (size_t)n : 0));
}

template <int P>
static int strip_grid(int n, int w, int num_cu) {
    return persistent_grid(k_dtw_strip<P, kStripRows, false>, strip_lds(n, w), num_cu);
}

static int strip_grid_p(int p, int n, int w, int num_cu) {
    return p == 1 ? strip_grid<1>(n, w, num_cu) : p == 2 ? strip_grid<2>(n, w, num_cu) : strip_grid<kPInf>(n, w, num_cu);
}

size_t dtw_strip_scratch(int p, int n, int w, int num_cu) {
    if (w <= kLaneMaxW) return 0;
    const int grid = strip_grid_p(p, n, w, num_cu);
    return sizeof(float) * (size_t)grid * ((size_t)1 << ring_log2(w)) * 64;
}

hipError_t launch_dtw_strip(int p, int w, int num_cu, const DtwArgs &a_in, float *ring, size_t ring_bytes,
                            hipStream_t s) {
    static_assert(kStripRows <= kLaneMaxW + 1, "strips need w >= C");
    if (w <= kLaneMaxW || !ring || ring_bytes < dtw_strip_scratch(p, a_in.n, w, num_cu)) return hipErrorInvalidValue;
    DtwArgs a = a_in;
    if (a.S1 && strip_lds(a.n, w, true) > kLdsBudget) a.S1 = nullptr;  // no room for U, L: row minimum only
    const size_t lds = strip_lds(a.n, w, a.S1 != nullptr);
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    const int rl = ring_log2(w);
    // the ring was sized for the grid of the plain kernel without U, L in LDS; the grid launched
    // here is capped to it
    const int cap = strip_grid_p(p, a.n, w, num_cu);
#define LBIMP_STRIP(PP, CC)                                                                                         \
    hipLaunchKernelGGL((k_dtw_strip<PP, kStripRows, CC>),                                                          \
                       dim3(std::min(cap, persistent_grid(k_dtw_strip<PP, kStripRows, CC>, lds, num_cu))), dim3(64), \
                       lds, s, a, w, ring, rl)
    const bool cas = a.S1 != nullptr;
    if (p == 1) {
        if (cas) LBIMP_STRIP(1, true);
        else LBIMP_STRIP(1, false);
    } else if (p == 2) {
        if (cas) LBIMP_STRIP(2, true);
        else LBIMP_STRIP(2, false);
    } else {
        if (cas) return hipErrorInvalidValue;  // the LB_Keogh tail bound sums p-th powers
        LBIMP_STRIP(kPInf, false);
    }
#undef LBIMP_STRIP
    return hipGetLastError();
}

}  // namespace lbimp
