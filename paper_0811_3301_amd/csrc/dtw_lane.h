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


// PH: row phases (DtwArgs::row0/row1/resume) compiled in; without them the kernel keeps the
// registers (and waves per SIMD) of a plain sweep over all rows.
template <int P, int W, bool CASCADE, bool PH>
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
        const int e = jj < pair_count(a.pl, q, items.bk) ? pair_cand(a.pl, q, jj, items.bk) : -1;
        bool active = e >= 0;
        float D[BW];
        float done = 0.f;  // LB_Keogh^p terms of the rows already computed
        int c;
        if (PH && a.resume) {  // e is the pool slot of a pair parked by the previous launch
            const int64_t sl = active ? e : 0;
            c = active ? reinterpret_cast<const int *>(a.pool)[(int64_t)(BW + 1) * a.pool_cap + sl] : 0;
#pragma unroll
            for (int k = 0; k < BW; ++k) D[k] = active ? a.pool[(int64_t)k * a.pool_cap + sl] : kInf;
            done = active ? a.pool[(int64_t)BW * a.pool_cap + sl] : 0.f;
        } else {
            c = active ? e : 0;
#pragma unroll
            for (int k = 0; k < BW; ++k) D[k] = (k == W) ? 0.f : kInf;
        }
        const float *x = a.rows + (int64_t)c * n;
        int stopped = 0;
        const int nfull = n - n % kLaneRows;
        // rows [a.row0, rpark) first; at rpark (< nfull) the running pairs are parked
        const int rpark = (PH && a.row1 > 0 && a.row1 < nfull) ? a.row1 : nfull;
        float xs[kLaneRows];
        int i0 = PH ? a.row0 : 0;
        // The threshold used after each group of rows is loaded one group ahead, from one pointer
        // with no branch around the load, so the wait for it lands where it is used.
        const u64 *tq = a.tkeys + q;
        u64 tcur = __hip_atomic_load(tq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        float s1v = 0.f;
        if constexpr (cascade) s1v = active ? a.S1[q * a.ldS + c] : 0.f;  // S1 may be a chunk's shifted base
        int stop_at = rpark;
        for (int round = 0; round < 2; ++round) {
            if (i0 < stop_at) {
#pragma unroll
                for (int r = 0; r < kLaneRows; ++r) xs[r] = x[i0 + r];
            }
            for (; i0 < stop_at; i0 += kLaneRows) {
                float xn[kLaneRows];
                const int inext = i0 + kLaneRows < stop_at ? i0 + kLaneRows : i0;  // prefetch the next rows
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
            if (!PH || round > 0 || stop_at >= nfull || i0 < stop_at) break;
            // park the running pairs in wave-contiguous pool slots; those past the pool's end run on
            const u64 m = __ballot(active);
            int base = 0;
            if (lane == 0 && m) base = atomicAdd(a.pool_ctr, __popcll(m));
            base = __shfl(base, 0);
            const int64_t slot = (int64_t)base + __popcll(m & ((1ull << lane) - 1ull));
            const bool fits = active && slot < a.pool_cap;
            if (fits) {
#pragma unroll
                for (int k = 0; k < BW; ++k) a.pool[(int64_t)k * a.pool_cap + slot] = D[k];
                a.pool[(int64_t)BW * a.pool_cap + slot] = done;
                reinterpret_cast<int *>(a.pool)[(int64_t)(BW + 1) * a.pool_cap + slot] = c;
            }
            const u64 mf = __ballot(fits);
            if (mf) {
                int pos = 0;
                if (lane == 0) pos = atomicAdd(&a.park_cnt[q], __popcll(mf));
                pos = __shfl(pos, 0);
                if (fits) a.park_list[q * a.ld_park + pos + __popcll(mf & ((1ull << lane) - 1ull))] = (int)slot;
            }
            active = active && !fits;
            if (!__any(active)) break;
            stop_at = nfull;  // the pairs that found no slot finish here
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
    const bool ph = a.row1 > 0 || a.resume;
#define LBIMP_DTW_LANE(CC, PP)                                                                                         \
    hipLaunchKernelGGL((k_dtw_lane<P, W, CC, PP>), dim3(persistent_grid(k_dtw_lane<P, W, CC, PP>, lds, num_cu)), \
                       dim3(64), lds, s, a)
    if constexpr (P != kPInf) {
        if (a.S1) {
            if (ph)
                LBIMP_DTW_LANE(true, true);
            else
                LBIMP_DTW_LANE(true, false);
            return;
        }
    }
    if (ph)
        LBIMP_DTW_LANE(false, true);
    else
        LBIMP_DTW_LANE(false, false);
#undef LBIMP_DTW_LANE
}

using DtwLaneFn = void (*)(int, const DtwArgs &, hipStream_t);

template <int P, int... Ws>
constexpr std::array<DtwLaneFn, sizeof...(Ws)> dtw_lane_table(std::integer_sequence<int, Ws...>) {
    return {&dtw_lane_launch<P, Ws>...};
}

}  // namespace lbimp
