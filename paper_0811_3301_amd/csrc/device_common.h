// Device helpers shared by the persistent second-pass and DTW kernels.
#pragma once

#include "internal.h"

namespace lbimp {

using u64 = unsigned long long;

__device__ __forceinline__ u64 make_key(float v, int c) {
    return ((u64)__float_as_uint(v) << 32) | (u64)(unsigned)c;
}

// Persistent work loop.  Items (a query and a batch of its pairs) are dealt to the one-wave
// blocks of the grid in a fixed stride -- block g takes items g, g + grid, g + 2*grid, ... --
// so no shared counter is contended.  With a fixed pair count per query the item maps to its
// query arithmetically; otherwise by binary search over the per-query item prefix.  Every
// block leaves the loop once its next item is past the total, so the grid always drains.
// Bucketed lists (pl.nb > 1; prefix over the nb * Q (bucket, query) slots, bucket-major):
// blocks are dealt to the 8 XCDs in turn (block g on XCD g % 8), so XCD x takes buckets x,
// x + 8, x + 16, ... and its blocks stride through the items of one bucket before the next;
// bk names the bucket of the last item.
// Contiguous form (lists that are not bucketed, on request): block g takes the items
// [g * total / grid, (g + 1) * total / grid) in order, so it finds its first query once and then
// steps to the next query when the current one's items are done.  Short items (a few
// microseconds each) then do not pay a dependent search of the prefix per item, and a block's
// consecutive items mostly share a query.
struct ItemCursor {
    long long next, stride, total;
    long long ipq;  // items per query when every query has the same pair count, else 0
    const long long *prefix;
    int64_t Q;
    int nb, bstep;
    int bk = 0;
    bool contig = false;
    long long end = 0;           // contiguous: one past the block's last item
    int64_t cq = 0;              // contiguous: query of the next item
    long long qlo = 0, qhi = 0;  // contiguous: items of query cq are [qlo, qhi)

    __device__ ItemCursor(const PairList &pl, const long long *prefix_, int64_t Q_, int batch,
                          bool contiguous = false)
        : next(blockIdx.x), stride(gridDim.x), prefix(prefix_), Q(Q_), nb(pl.nb), bstep(1) {
        if (!pl.cnt) {
            ipq = (pl.fixed + batch - 1) / batch;
            total = Q * ipq;
        } else {
            ipq = 0;
            total = prefix[(int64_t)nb * Q];
        }
        if (nb > 1 && gridDim.x >= 8 && gridDim.x % 8 == 0) {
            bk = (int)(blockIdx.x % 8);
            next = blockIdx.x / 8;
            stride = gridDim.x / 8;
            bstep = 8;
        } else if (nb > 1) {
            bk = 0;
        } else if (contiguous) {
            contig = true;
            next = total * (long long)blockIdx.x / (long long)gridDim.x;
            end = total * ((long long)blockIdx.x + 1) / (long long)gridDim.x;
            if (next < end) {
                cq = ipq ? next / ipq : slot_of(next, 0, Q);
                qlo = ipq ? cq * ipq : prefix[cq];
                qhi = ipq ? qlo + ipq : prefix[cq + 1];
            }
        }
    }

    // largest v in [lo, hi) with prefix[v] <= item
    __device__ int64_t slot_of(long long item, int64_t lo, int64_t hi) const {
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (prefix[mid] <= item)
                lo = mid;
            else
                hi = mid;
        }
        return lo;
    }

    __device__ bool get(int64_t &q, long long &b) {
        if (contig) {
            if (next >= end) return false;
            while (next >= qhi) {  // the next query with items (qhi reaches total by query Q - 1)
                ++cq;
                qlo = qhi;
                qhi = ipq ? qlo + ipq : prefix[cq + 1];
            }
            q = cq;
            b = next - qlo;
            ++next;
            return true;
        }
        if (nb > 1) {  // next is the item offset within bucket bk
            while (bk < nb) {
                const long long lo = prefix[(int64_t)bk * Q], range = prefix[(int64_t)(bk + 1) * Q] - lo;
                if (next < range) {
                    const long long item = lo + next;
                    next += stride;
                    const int64_t v = slot_of(item, (int64_t)bk * Q, (int64_t)(bk + 1) * Q);
                    q = v - (int64_t)bk * Q;
                    b = item - prefix[v];
                    return true;
                }
                next -= range;
                bk += bstep;
            }
            return false;
        }
        if (next >= total) return false;
        const long long item = next;
        next += stride;
        if (ipq) {
            q = item / ipq;
            b = item - q * ipq;
            return true;
        }
        q = slot_of(item, 0, Q);
        b = item - prefix[q];
        return true;
    }
};

__device__ __forceinline__ int pair_count(const PairList &pl, int64_t q, int bk = 0) {
    return pl.cnt ? pl.cnt[(int64_t)bk * pl.cq + q] : (int)pl.fixed;
}

__device__ __forceinline__ int pair_cand(const PairList &pl, int64_t q, long long j, int bk = 0) {
    return pl.list ? pl.list[q * pl.ldl + (int64_t)bk * pl.bs + j] : (int)(pl.base + j);
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
    if (thr && res && key < thr[q]) {
        int pos = atomicAdd(&rescnt[q], 1);
        res[q * ldres + pos] = key;
    }
}

__device__ __forceinline__ u64 current_threshold(int64_t q, const u64 *best, const u64 *thr) {
    if (best) return __hip_atomic_load(&best[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (thr) return thr[q];
    return kNoKey;
}


// Copy `count` values into LDS with one wave: dst[t] = value_at(t).  Eight loads per lane are
// issued before any store, so a staging pass costs a few memory latencies, not one per value.
template <class F>
__device__ __forceinline__ void stage_lds(float *dst, int count, F value_at) {
    const int lane = threadIdx.x & 63;
    for (int base = 0; base < count; base += 64 * 8) {
        float v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int t = base + r * 64 + lane;
            v[r] = t < count ? value_at(t) : 0.f;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int t = base + r * 64 + lane;
            if (t < count) dst[t] = v[r];
        }
    }
}

// Grid of a persistent kernel: as many one-wave blocks as fit on the chip at once.
template <class Kernel>
inline int persistent_grid(Kernel k, size_t lds, int num_cu) {
    // occupancy queries cost microseconds each; remember them per (kernel, LDS size, device) in a
    // fixed table, so that launching never allocates host memory
    struct Entry {
        const void *k;
        size_t lds;
        int device, per_cu;
    };
    constexpr int kCache = 512;
    static thread_local Entry cache[kCache];
    static thread_local int cached = 0;
    int device = 0;
    (void)hipGetDevice(&device);
    for (int i = 0; i < cached; ++i) {
        const Entry &e = cache[i];
        if (e.k == reinterpret_cast<const void *>(k) && e.lds == lds && e.device == device) return num_cu * e.per_cu;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64, lds) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 4;
    }
    if (cached < kCache) cache[cached++] = Entry{reinterpret_cast<const void *>(k), lds, device, per_cu};
    return num_cu * per_cu;
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
    const u64 *tkeys;  // [Q] abandon thresholds: best (k = 1) or thr (k > 1); always a valid array
    const float *S1;   // [Q][ldS] LB_Keogh^p of every pair (tightens the abandon bound), or nullptr
    int64_t ldS;
    // Row phases (lane-per-pair kernel only).  With row1 > 0 the launch runs rows [row0, row1)
    // and parks every pair still running there: its band row, LB_Keogh sum so far and candidate
    // go to slot s of `pool` (field f at pool[f * pool_cap + s], slots from the counter
    // *pool_ctr) and s is appended to park_list[q][*] (counts park_cnt[q]); a pair finding the
    // pool full runs on to the end.  With resume the pairs of pl are such slots, and the launch
    // continues them from row0.  row0 and row1 are multiples of the kernel's row group.
    int row0 = 0, row1 = 0;
    bool resume = false;
    float *pool = nullptr;
    int64_t pool_cap = 0;
    int *pool_ctr = nullptr;
    int *park_list = nullptr;
    int64_t ld_park = 0;
    int *park_cnt = nullptr;
};

// Lower bound of a pair's DTW_p once rows 0..i are done: the minimum of row i plus the
// LB_Keogh^p terms of the rows after i, which every remaining step of a path pays at least
// (a cell (r, j) costs d(x_r, y_j)^p >= d(x_r, [L_r, U_r])^p).  The tail is S1 (the sweep's
// sum over all rows) minus the rows already done.
// Rounding (u = 2^-24, D the exact DTW; every quantity below is at most D because LB_Keogh and
// any row minimum are):  the fp32 DTW is the rounded sum along some path of at most 2n - 1
// cells, each term carrying up to two roundings for p = 2, so it is at least D (1 - (2n + 3) u);
// the row minimum is such a partial sum, at most its exact value times (1 + (2n + 3) u); S1 and
// the running sum "done" carry at most n u S1 each, and S1 - done and the final add one u more.
// The computed bound is therefore at most D (1 + (4n + 8) u), and scaling it by
// 1 - (6n + 16) u keeps it at or below the fp32 DTW: abandoning on it changes no result.
__device__ __forceinline__ float cascade_bound(float rowmin, float s1, float done, float shrink) {
    return (rowmin + fmaxf(s1 - done, 0.f)) * shrink;
}
__host__ __device__ inline float cascade_shrink(int n) { return 1.f - (6.f * n + 16.f) * 5.9604645e-8f; }

// LB_Keogh^p term of one element against the envelope [lo, hi].
template <int P>
__device__ __forceinline__ float lbk_term(float x, float lo, float hi) {
    return pacc<P>(0.f, x - __builtin_amdgcn_fmed3f(x, lo, hi));
}

// Arguments of the register-state LB_Improved kernels (one instantiation per half-width).
struct LbiArgs {
    const float *rows;
    int64_t db_bytes;  // size of rows in bytes
    int n;
    QueryData qd;
    PairList pl;
    const float *S1;
    int64_t ldS;
    const long long *prefix;
    int64_t Q;
    int *ctr;
    const u64 *thr;
    int *list2;
    int64_t ldl2;
    int *cnt2;
    float *out_root;
    int pipeline;   // blocks loaded ahead in the register kernel: 0 or 1 (more registers, fewer exposed latencies)
    bool abandon;   // early abandoning: stop once the partial bound reaches the threshold (thr set)
    bool fused = false;     // register kernel only: LB_Keogh computed here (S1 not read), see k_lbi_reg
    int *cntk = nullptr;    // fused: per query, pairs whose LB_Keogh is below the threshold
    float *S1out = nullptr; // fused: LB_Keogh of each surviving pair, [q * ldS + c]
};

// Wave-per-pair LB_Improved for wide bands (n + w <= 2048, 2w + 1 larger than a lane's slice).
bool lbi_wave_supported(int n, int w);
hipError_t launch_lbi_wave(int p, int w, int num_cu, const LbiArgs &a, hipStream_t s);

hipError_t launch_lbi_reg_p1(int w, int num_cu, const LbiArgs &a, hipStream_t s);
hipError_t launch_lbi_reg_p2(int w, int num_cu, const LbiArgs &a, hipStream_t s);
hipError_t launch_lbi_reg_pinf(int w, int num_cu, const LbiArgs &a, hipStream_t s);

// Group-of-lanes-per-pair DTW (anti-diagonals in registers); batch = dtw_wave_batch(n, w).
int dtw_wave_batch(int n, int w);
hipError_t launch_dtw_wavereg(int p, int w, int num_cu, const DtwArgs &a, hipStream_t s);

// Group-per-pair DTW for 63 < w < 512: one pair per wave, several band positions per lane.
bool dtw_wavereg_wide_supported(int n, int w);
hipError_t launch_dtw_wavereg_wide(int p, int w, int num_cu, const DtwArgs &a, hipStream_t s);

// Lane-per-pair DTW of wide bands in strips of rows (ring: per-wave strip boundaries).
hipError_t launch_dtw_strip(int p, int w, int num_cu, const DtwArgs &a, float *ring, size_t ring_bytes,
                            hipStream_t s);

hipError_t launch_dtw_lane_p1(int w, int num_cu, const DtwArgs &a, hipStream_t s);
hipError_t launch_dtw_lane_p2(int w, int num_cu, const DtwArgs &a, hipStream_t s);
hipError_t launch_dtw_lane_pinf(int w, int num_cu, const DtwArgs &a, hipStream_t s);

}  // namespace lbimp
