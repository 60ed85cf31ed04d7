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
// Early abandoning: every 4 rows the row minimum bounds the result (a path crosses every row
// and costs are non-negative); a lane whose (bound, index) key reaches the threshold key can
// no longer win and stops.  The wave leaves the row loop once every lane has stopped.
template <int P, int W>
__device__ __forceinline__ void dtw_row(float (&D)[2 * W + 1], float xi, const float *yrow) {
    constexpr int BW = 2 * W + 1;
    float left = kInf;
#pragma unroll
    for (int k = 0; k < BW; ++k) {
        const float d = xi - yrow[k];
        const float up = (k + 1 < BW) ? D[k + 1] : kInf;
        const float m = __builtin_fminf(__builtin_fminf(D[k], up), left);
        const float v = (P == 1) ? m + fabsf(d) : fmaf(d, d, m);
        D[k] = v;
        left = v;
    }
}

template <int P, int W>
__global__ __launch_bounds__(64) void k_dtw_lane(DtwArgs a) {
    constexpr int BW = 2 * W + 1;
    extern __shared__ float ypad[];  // ypad[t] = y[t - W], +inf outside [0, n)
    const int lane = threadIdx.x;
    const int n = a.n;
    const int plen = n + BW + 4;
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    while (next_item(a.ctr, a.prefix, a.Q, q, b)) {
        if (q != cur_q) {
            __syncthreads();
            const float *y = a.qd.Y + q * a.qd.ldy;
            for (int t = lane; t < plen; t += 64) {
                const int j = t - W;
                ypad[t] = (j >= 0 && j < n) ? y[j] : kInf;
            }
            __syncthreads();
            cur_q = q;
        }
        const long long jj = b * 64 + lane;
        bool active = jj < pair_count(a.pl, q);
        const int c = active ? pair_cand(a.pl, q, jj) : 0;
        const float *x = a.rows + (int64_t)c * n;
        float D[BW];
#pragma unroll
        for (int k = 0; k < BW; ++k) D[k] = (k == W) ? 0.f : kInf;
        int stopped = 0;
        const int nfull = n & ~3;
        float xs[4];
        if (nfull > 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) xs[r] = x[r];
        }
        int i0 = 0;
        for (; i0 < nfull; i0 += 4) {
            float xn[4];
            const int inext = i0 + 4 < nfull ? i0 + 4 : i0;  // prefetch the next 4 rows
#pragma unroll
            for (int r = 0; r < 4; ++r) xn[r] = x[inext + r];
#pragma unroll
            for (int r = 0; r < 4; ++r) dtw_row<P, W>(D, xs[r], ypad + i0 + r);
#pragma unroll
            for (int r = 0; r < 4; ++r) xs[r] = xn[r];
            if (a.abandon) {
                float mn = D[0];
#pragma unroll
                for (int k = 1; k < BW; ++k) mn = fminf(mn, D[k]);
                if (active && make_key(mn, c) >= current_threshold(q, a.best, a.thr)) {
                    active = false;
                    ++stopped;
                }
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
static void dtw_lane_launch(int grid, const DtwArgs &a, hipStream_t s) {
    const size_t lds = sizeof(float) * (size_t)(a.n + 2 * W + 1 + 4);
    hipLaunchKernelGGL((k_dtw_lane<P, W>), dim3(grid), dim3(64), lds, s, a);
}

using DtwLaneFn = void (*)(int, const DtwArgs &, hipStream_t);

template <int P, int... Ws>
constexpr std::array<DtwLaneFn, sizeof...(Ws)> dtw_lane_table(std::integer_sequence<int, Ws...>) {
    return {&dtw_lane_launch<P, Ws>...};
}

}  // namespace lbimp
