// Lane-per-pair banded DTW_p (Sec. 4 of Lemire, arXiv:0811.3301), one instantiation per band
// half-width W so that the band lives in registers with compile-time indices.
#pragma once

#include <array>
#include <utility>

#include "device_common.h"

namespace lbimp {

// 64 pairs of one query per wave, lane = candidate.  Row i of the band (columns j = i-W+k,
// k in [0, 2W]) is held in registers D[k]; updating k upwards in place reads D[k] and D[k+1]
// of row i-1 and D[k-1] of row i: the predecessors (i-1,j-1), (i-1,j) and (i,j-1) of the
// recursion written in prefix form (every path reversed).  The query sits in LDS padded with
// +inf on both sides, so columns outside [0, n) cost +inf with no branch; the virtual cell
// (-1,-1) = 0 is D[W] of row -1.  Per cell: one subtract, one 3-way min, one add (|d|, p = 1)
// or fma (d*d, p = 2).
// Early abandoning: after every group of rows the row minimum bounds the result (a path crosses every row
// and costs are non-negative); a lane whose (bound, index) key reaches the threshold key can
// no longer win and stops.  The wave leaves the row loop once every lane has stopped.
template <int P, int W>
__device__ __forceinline__ void dtw_row(float (&D)[2 * W + 1], float xi, const float *yrow) {
    constexpr int BW = 2 * W + 1;
#pragma unroll
    for (int k = 0; k < BW; ++k) {
        const float d = xi - yrow[k];
        const float up = (k + 1 < BW) ? D[k + 1] : kInf;
        const float left = (k > 0) ? D[k - 1] : kInf;
        const float m = __builtin_fminf(__builtin_fminf(D[k], up), left);
        D[k] = pacc<P>(m, d);
    }
}

// R rows at once in skewed order: step s updates cell k = s - r of row r, rows ascending.
// The in-place reads are unchanged -- when (r, k) runs, D[k] and D[k+1] still hold row r-1
// and D[k-1] already holds row r -- but the R dependency chains interleave, which hides the
// latency of the serial left-to-right chain of each row.  More rows hide more latency, but
// past about 520 unrolled cells per step the compiler stops keeping D in registers (it moves
// the array to scratch memory): eight rows up to w = 32, six up to w = 53, four above.
template <int P, int W, int R>
__device__ __forceinline__ void dtw_rowsR(float (&D)[2 * W + 1], const float (&xs)[R], const float *yrow0) {
    constexpr int BW = 2 * W + 1;
#pragma unroll
    for (int s = 0; s < BW + R - 1; ++s) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = s - r;
            if (k >= 0 && k < BW) {
                const float d = xs[r] - yrow0[r + k];
                const float up = (k + 1 < BW) ? D[k + 1] : kInf;
                const float left = (k > 0) ? D[k - 1] : kInf;
                const float m = __builtin_fminf(__builtin_fminf(D[k], up), left);
                D[k] = pacc<P>(m, d);
            }
        }
    }
}

constexpr int lane_rows(int w) { return w <= 32 ? 8 : w <= 53 ? 6 : 4; }

template <int P, int W, bool CASCADE>
__global__ __launch_bounds__(64) void k_dtw_lane(DtwArgs a) {
    constexpr int BW = 2 * W + 1;
    constexpr int kLaneRows = lane_rows(W);
    extern __shared__ float ypad[];  // ypad[t] = y[t - W], +inf outside [0, n); then U, L when a.S1
    const int lane = threadIdx.x;
    const int n = a.n;
    const int plen = n + BW + kLaneRows;
    float *sU = ypad + plen, *sL = sU + n;
    constexpr bool cascade = CASCADE;  // a.S1 is set exactly for this instantiation
    const float shrink = cascade_shrink(n);
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(a.pl, a.prefix, a.Q, 64);
    while (items.get(q, b)) {
        if (q != cur_q) {
            __syncthreads();
            const float *y = a.qd.Y + q * a.qd.ldy;
            stage_lds(ypad, plen, [&](int t) {
                const int j = t - W;
                return (j >= 0 && j < n) ? y[j] : kInf;
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
        float D[BW];
#pragma unroll
        for (int k = 0; k < BW; ++k) D[k] = (k == W) ? 0.f : kInf;
        int stopped = 0;
        const int nfull = n - n % kLaneRows;
        float xs[kLaneRows];
        if (nfull > 0) {
#pragma unroll
            for (int r = 0; r < kLaneRows; ++r) xs[r] = x[r];
        }
        int i0 = 0;
        // The threshold used after each group of rows is loaded one group ahead, from one pointer
        // with no branch around the load, so the wait for it lands where it is used.
        const u64 *tq = a.tkeys + q;
        u64 tcur = __hip_atomic_load(tq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        float s1v = 0.f;
        if constexpr (cascade) s1v = active ? a.S1[q * a.ldS + c] : 0.f;  // S1 may be a chunk's shifted base
        float done = 0.f;  // LB_Keogh^p terms of the rows already computed
        for (; i0 < nfull; i0 += kLaneRows) {
            float xn[kLaneRows];
            const int inext = i0 + kLaneRows < nfull ? i0 + kLaneRows : i0;  // prefetch the next rows
#pragma unroll
            for (int r = 0; r < kLaneRows; ++r) xn[r] = x[inext + r];
            const u64 tnext = __hip_atomic_load(tq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            dtw_rowsR<P, W, kLaneRows>(D, xs, ypad + i0);
            if constexpr (cascade) {
#pragma unroll
                for (int r = 0; r < kLaneRows; ++r) done += lbk_term<P>(xs[r], sL[i0 + r], sU[i0 + r]);
            }
#pragma unroll
            for (int r = 0; r < kLaneRows; ++r) xs[r] = xn[r];
            if (a.abandon) {
                float mn = D[0];
#pragma unroll
                for (int k = 1; k < BW; ++k) mn = fminf(mn, D[k]);
                if constexpr (cascade) mn = cascade_bound(mn, s1v, done, shrink);
                if (active && make_key(mn, c) >= tcur) {
                    active = false;
                    ++stopped;
                }
                tcur = tnext;
                if (!__any(active)) break;
            }
        }
        if (i0 >= nfull)
            for (int i = nfull; i < n; ++i) dtw_row<P, W>(D, x[i], ypad + i);
        publish<P>(active, D[W], c, q, a.best, a.thr, a.res, a.ldres, a.rescnt, a.out_root);
        if (a.abandoned) {
            const u64 m = __ballot(stopped != 0);
            if (lane == 0 && m) atomicAdd(&a.abandoned[q], __popcll(m));
        }
    }
}

template <int P, int W>
static void dtw_lane_launch(int num_cu, const DtwArgs &a_in, hipStream_t s) {
    DtwArgs a = a_in;
    auto lds_of = [&](bool cascade) {
        return sizeof(float) * ((size_t)a.n + 2 * W + 1 + lane_rows(W) + (cascade ? 2 * (size_t)a.n : 0));
    };
    if (a.S1 && lds_of(true) > kLdsBudget) a.S1 = nullptr;  // no room for U, L: row minimum only
    if constexpr (P == kPInf) a.S1 = nullptr;               // the LB_Keogh tail bound sums p-th powers
    const size_t lds = lds_of(a.S1 != nullptr);
    if constexpr (P != kPInf) {
        if (a.S1) {
            hipLaunchKernelGGL((k_dtw_lane<P, W, true>), dim3(persistent_grid(k_dtw_lane<P, W, true>, lds, num_cu)),
                               dim3(64), lds, s, a);
            return;
        }
    }
    hipLaunchKernelGGL((k_dtw_lane<P, W, false>), dim3(persistent_grid(k_dtw_lane<P, W, false>, lds, num_cu)),
                       dim3(64), lds, s, a);
}

using DtwLaneFn = void (*)(int, const DtwArgs &, hipStream_t);

template <int P, int... Ws>
constexpr std::array<DtwLaneFn, sizeof...(Ws)> dtw_lane_table(std::integer_sequence<int, Ws...>) {
    return {&dtw_lane_launch<P, Ws>...};
}

}  // namespace lbimp
