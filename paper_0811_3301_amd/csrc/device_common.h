// Device helpers shared by the persistent second-pass and DTW kernels.
#pragma once

#include "internal.h"

namespace lbimp {

using u64 = unsigned long long;

__device__ __forceinline__ u64 make_key(float v, int c) {
    return ((u64)__float_as_uint(v) << 32) | (u64)(unsigned)c;
}

template <int P>
__device__ __forceinline__ float root_p(float v) {
    if constexpr (P == 1)
        return v;
    else
        return sqrtf(v);
}

// Persistent work loop: a wave takes the next item from a device counter and maps it to
// (query, batch) by binary search over the per-query item prefix.  Every wave leaves the
// loop once the counter passes the total, so the grid always drains.
__device__ __forceinline__ bool next_item(int *ctr, const long long *__restrict__ prefix, int64_t Q, int64_t &q,
                                          long long &b) {
    int item = 0;
    if ((threadIdx.x & 63) == 0) item = atomicAdd(ctr, 1);
    item = __shfl(item, 0);
    const long long total = prefix[Q];
    if (item >= total) return false;
    int64_t lo = 0, hi = Q;  // largest q with prefix[q] <= item
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= item)
            lo = mid;
        else
            hi = mid;
    }
    q = lo;
    b = item - prefix[lo];
    return true;
}

__device__ __forceinline__ int pair_count(const PairList &pl, int64_t q) {
    return pl.cnt ? pl.cnt[q] : (int)pl.fixed;
}

__device__ __forceinline__ int pair_cand(const PairList &pl, int64_t q, long long j) {
    return pl.list ? pl.list[q * pl.ldl + j] : (int)j;
}


// ------------------------------------------------------------------ banded DTW_p (Sec. 4)
// Shared epilogue: publish the finished DTW of candidate c.
template <int P>
__device__ __forceinline__ void publish(bool active, float d, int c, int64_t q, u64 *best, const u64 *thr, u64 *res,
                                        int64_t ldres, int *rescnt, float *out_root) {
    if (!active) return;
    if (out_root) out_root[c] = root_p<P>(d);
    const u64 key = make_key(d, c);
    if (best) {
        if (key < __hip_atomic_load(&best[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(&best[q], key);
    }
    if (thr && key < thr[q]) {
        int pos = atomicAdd(&rescnt[q], 1);
        res[q * ldres + pos] = key;
    }
}

__device__ __forceinline__ u64 current_threshold(int64_t q, const u64 *best, const u64 *thr) {
    if (best) return __hip_atomic_load(&best[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (thr) return thr[q];
    return kNoKey;
}


// Arguments of the lane-per-pair DTW kernels (one instantiation per band half-width).
struct DtwArgs {
    const float *rows;
    int n;
    QueryData qd;
    PairList pl;
    const long long *prefix;
    int64_t Q;
    int *ctr;
    u64 *best;
    const u64 *thr;
    u64 *res;
    int64_t ldres;
    int *rescnt;
    int *abandoned;
    float *out_root;
    bool abandon;
};

hipError_t launch_dtw_lane_p1(int w, int grid, const DtwArgs &a, hipStream_t s);
hipError_t launch_dtw_lane_p2(int w, int grid, const DtwArgs &a, hipStream_t s);

}  // namespace lbimp
