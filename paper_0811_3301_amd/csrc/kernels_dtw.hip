// Second pruning pass (LB_Improved), banded DTW_p and result finalisation.
//
// Cited passages (Lemire, arXiv:0811.3301): DTW_p recursion and locality constraint (Sec. 4),
// projection H and LB_Keogh (Sec. 7), LB_Improved and Algorithm 3 (Sec. 8).
#include "device_common.h"

namespace lbimp {

// ------------------------------------------------------------------ LB_Improved (Sec. 8)
// Generic fallback for bands neither the register kernel nor the wave kernel takes (series
// longer than 2048 with w > 52): lane per (query, candidate) pair, WL pairs per wave.  For the candidate
// x: x' = H(x, y) = med3(x, L, U) (eq. of H), its envelope (U', L') with the same w, and the
// second term sum_i d(y_i, [L'_i, U'_i])^p.  The envelope of x' is streamed with van Herk /
// Gil-Werman blocks of K = 2w+1: walking e forward through block B keeps g = running max/min
// since the block start; the window of output i = e - w starts at s = e - K + 1, inside
// block B-1 at offset o+1 (or at B's start when o = K-1), whose suffix max/min h was stored
// by a backward walk over block B-1.  Only h (2(K+1) floats per lane) lives in LDS.
int lbi_batch(int n, int w) {
    if (w <= kLbiRegMaxW || lbi_wave_supported(n, w)) return 64;
    const size_t K = 2 * (size_t)w + 1;
    const size_t fixed = 3 * 4 * (size_t)n;
    if (fixed >= kLdsBudget) return 0;
    const size_t budget = kLdsBudget - fixed;
    int wl = 64;
    while (wl > 1 && 8 * (K + 1) * wl > budget) wl >>= 1;
    return 8 * (K + 1) * wl > budget ? 0 : wl;
}

template <int P>
__device__ __forceinline__ float lb_acc(float acc, float v, float lo, float hi) {
    return pacc<P>(acc, v - __builtin_amdgcn_fmed3f(v, lo, hi));
}

template <int P>
__global__ __launch_bounds__(64) void k_lbi(const float *__restrict__ rows, int n, int w, QueryData qd, PairList pl,
                                            const float *__restrict__ S1, int64_t ldS,
                                            const long long *__restrict__ prefix, int64_t Q, int *ctr, int WL,
                                            const u64 *__restrict__ thr, int *__restrict__ list2, int64_t ldl2,
                                            int *__restrict__ cnt2, float *__restrict__ out_root) {
    extern __shared__ float sm[];
    float *sU = sm, *sL = sm + n, *sY = sm + 2 * n;
    float *hmax = sm + 3 * n;
    const int K = 2 * w + 1;
    float *hmin = hmax + (size_t)(K + 1) * WL;
    const int lane = threadIdx.x;
    const int nblk = (n + w + K - 1) / K;
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(pl, prefix, Q, WL);
    while (items.get(q, b)) {
        if (q != cur_q) {
            __syncthreads();
            stage_lds(sU, n, [&](int i) { return qd.U[q * qd.ldq + i]; });
            stage_lds(sL, n, [&](int i) { return qd.L[q * qd.ldq + i]; });
            stage_lds(sY, n, [&](int i) { return qd.Y[q * qd.ldy + i]; });
            __syncthreads();
            cur_q = q;
        }
        const long long j = b * WL + lane;
        const bool active = lane < WL && j < pair_count(pl, q, items.bk);
        const int c = active ? pair_cand(pl, q, j, items.bk) : 0;
        const float *x = rows + (int64_t)c * n;
        const int hl = lane < WL ? lane : 0;
        if (lane < WL) {
            hmax[(size_t)K * WL + hl] = -kInf;
            hmin[(size_t)K * WL + hl] = kInf;
            for (int o = 0; o < K; ++o) {
                hmax[(size_t)o * WL + hl] = -kInf;
                hmin[(size_t)o * WL + hl] = kInf;
            }
        }
        float acc = 0.f;
        for (int B = 0; B < nblk; ++B) {
            const int e0 = B * K;
            float gmx = -kInf, gmn = kInf;
            const int oend = min(K, n + w - e0);
            for (int o = 0; o < oend; ++o) {
                const int e = e0 + o;
                if (e < n) {
                    float v = __builtin_amdgcn_fmed3f(x[e], sL[e], sU[e]);
                    gmx = fmaxf(gmx, v);
                    gmn = fminf(gmn, v);
                }
                if (e >= w) {
                    const float um = fmaxf(hmax[(size_t)(o + 1) * WL + hl], gmx);
                    const float lm = fminf(hmin[(size_t)(o + 1) * WL + hl], gmn);
                    acc = lb_acc<P>(acc, sY[e - w], lm, um);
                }
            }
            if (B + 1 < nblk) {
                float rmx = -kInf, rmn = kInf;
                for (int o = K - 1; o >= 0; --o) {
                    const int e = e0 + o;
                    if (e < n) {
                        float v = __builtin_amdgcn_fmed3f(x[e], sL[e], sU[e]);
                        rmx = fmaxf(rmx, v);
                        rmn = fminf(rmn, v);
                    }
                    if (lane < WL) {
                        hmax[(size_t)o * WL + hl] = rmx;
                        hmin[(size_t)o * WL + hl] = rmn;
                    }
                }
            }
        }
        const float s2 = pjoin<P>(active ? S1[q * ldS + c] : 0.f, acc);
        if (out_root && active) out_root[c] = root_p<P>(s2);
        if (thr) {
            const bool keep = active && make_key(s2, c) < thr[q];
            const u64 m = __ballot(keep);
            if (m) {
                int pos = 0;
                if (lane == 0) pos = atomicAdd(&cnt2[q], __popcll(m));
                pos = __shfl(pos, 0);
                if (keep) list2[q * ldl2 + pos + __popcll(m & ((1ull << lane) - 1ull))] = c;
            }
        }
    }
}

hipError_t launch_lbi(int p, const float *rows, int64_t db_bytes, int n, int w, QueryData qd, PairList pl, const float *S1,
                      int64_t ldS, const long long *prefix, int64_t Q, int *ctr, int num_cu,
                      const unsigned long long *thr, int *list2, int64_t ldl2, int *cnt2, float *out_root,
                      int pipeline, bool abandon, hipStream_t s, bool fused, int *cntk, float *S1out) {
    if (fused && w > kLbiRegMaxW) return hipErrorInvalidValue;  // only the register kernel computes LB_Keogh itself
    if (w <= kLbiRegMaxW || lbi_wave_supported(n, w)) {
        LbiArgs a{rows, db_bytes, n, qd, pl, S1, ldS, prefix, Q, ctr, thr, list2, ldl2, cnt2, out_root, pipeline,
                  abandon};
        a.fused = fused;
        a.cntk = cntk;
        a.S1out = S1out;
        if (w > kLbiRegMaxW) return launch_lbi_wave(p, w, num_cu, a, s);
        if (p == 1) return launch_lbi_reg_p1(w, num_cu, a, s);
        return p == 2 ? launch_lbi_reg_p2(w, num_cu, a, s) : launch_lbi_reg_pinf(w, num_cu, a, s);
    }
    const int WL = lbi_batch(n, w);
    const int K = 2 * w + 1;
    size_t lds = sizeof(float) * (3 * (size_t)n + 2 * (size_t)(K + 1) * WL);
#define LBIMP_LBI(PP)                                                                                             \
    hipLaunchKernelGGL(k_lbi<PP>, dim3(persistent_grid(k_lbi<PP>, lds, num_cu)), dim3(64), lds, s, rows, n, w, qd, pl, \
                       S1, ldS, prefix, Q, ctr, WL, thr, list2, ldl2, cnt2, out_root)
    if (p == 1)
        LBIMP_LBI(1);
    else if (p == 2)
        LBIMP_LBI(2);
    else
        LBIMP_LBI(kPInf);
#undef LBIMP_LBI
    return hipGetLastError();
}

// Wide bands: wave per pair along anti-diagonals d = i + j.  Cells of one anti-diagonal are
// independent; cell (i, d-i) needs (i-1, j) and (i, j-1) on d-1 and (i-1, j-1) on d-2.  Three
// rotating LDS rows indexed by i+1 hold diagonals d-2, d-1, d; the two entries just outside
// each diagonal's valid range are written +inf so later reads never see stale values.  Any
// path visits one of every two consecutive anti-diagonals, so their minimum bounds the result.
template <int P>
__global__ __launch_bounds__(64) void k_dtw_wave(const float *__restrict__ rows, int n, int w, QueryData qd,
                                                 PairList pl, const long long *__restrict__ prefix, int64_t Q,
                                                 int *ctr, u64 *best, const u64 *__restrict__ thr, u64 *res,
                                                 int64_t ldres, int *rescnt, int *abandoned, float *out_root,
                                                 bool abandon) {
    extern __shared__ float sm[];
    float *buf[3] = {sm, sm + n + 1, sm + 2 * n + 2};
    const int lane = threadIdx.x;
    int64_t q;
    long long b;
    ItemCursor items(pl, prefix, Q, 1);
    while (items.get(q, b)) {
        const bool valid = b < pair_count(pl, q, items.bk);
        if (!valid) continue;
        const int c = pair_cand(pl, q, b, items.bk);
        const float *sx = rows + (int64_t)c * n;
        const float *sy = qd.Y + q * qd.ldy;
        __syncthreads();
        for (int i = lane; i <= n; i += 64) {
            buf[0][i] = (i == 0) ? 0.f : kInf;  // diagonal -2: D(-1,-1) = 0
            buf[1][i] = kInf;                   // diagonal -1
            buf[2][i] = kInf;
        }
        __syncthreads();
        int a2 = 0, a1 = 1, a0 = 2;
        bool alive = true;
        float mprev = kInf;
        for (int d = 0; d <= 2 * n - 2; ++d) {
            const int lo = max(max(0, d - n + 1), (d - w + 1) >> 1);
            const int hi = min(min(n - 1, d), (d + w) >> 1);
            float *C = buf[a0];
            const float *Bm = buf[a1];
            const float *Am = buf[a2];
            float mcur = kInf;
            for (int i = lo + lane; i <= hi; i += 64) {
                const float dd = sx[i] - sy[d - i];
                const float m = fminf(fminf(Bm[i], Bm[i + 1]), Am[i]);
                const float v = pacc<P>(m, dd);
                C[i + 1] = v;
                mcur = fminf(mcur, v);
            }
            if (lane == 0) C[lo] = kInf;
            if (lane == 1 && hi + 2 <= n) C[hi + 2] = kInf;
            __syncthreads();
            if (abandon && (d & 7) == 7) {
                float mm = fminf(mcur, mprev);
                for (int off = 32; off > 0; off >>= 1) mm = fminf(mm, __shfl_xor(mm, off));
                int stop = lane == 0 && make_key(mm, c) >= current_threshold(q, best, thr);
                if (__shfl(stop, 0)) {  // one decision for the whole wave: the loop holds barriers
                    alive = false;
                    break;
                }
            }
            mprev = mcur;
            const int t = a2;
            a2 = a1;
            a1 = a0;
            a0 = t;
        }
        if (alive) {
            const float dfin = buf[a1][n];
            if (lane == 0) publish<P>(true, dfin, c, q, best, thr, res, ldres, rescnt, out_root);
        } else if (abandoned && lane == 0) {
            atomicAdd(&abandoned[q], 1);
        }
    }
}

int dtw_batch(int n, int w, bool low_latency) {
    if (w > kLaneMaxW) return low_latency ? 1 : 64;
    return low_latency ? dtw_wave_batch(n, w) : 64;
}

hipError_t launch_dtw(int p, const float *rows, int n, int w, QueryData qd, PairList pl, const long long *prefix,
                      int64_t Q, int *ctr, int num_cu, unsigned long long *best, const unsigned long long *thr,
                      unsigned long long *res, int64_t ldres, int *rescnt, int *abandoned, float *out_root,
                      bool abandon, bool low_latency, float *ring, size_t ring_bytes, const float *S1,
                      int64_t ldS, hipStream_t s, const DtwPhase *ph) {
    if (ph && (w > kLaneMaxW || low_latency)) return hipErrorInvalidValue;  // phases: lane-per-pair kernel only
    if (w <= kLaneMaxW || !low_latency || dtw_wavereg_wide_supported(n, w)) {
        const u64 *tkeys = best ? best : thr;
        if (!tkeys) return hipErrorInvalidValue;  // callers pass a threshold array, kNoKey-filled if unused
        DtwArgs a{rows, n, qd, pl, prefix, Q, ctr, best, thr, res, ldres, rescnt, abandoned, out_root, abandon, tkeys,
                  abandon && p != kPInf ? S1 : nullptr, ldS};  // the LB_Keogh tail bound sums p-th powers
        if (ph) {
            a.row0 = ph->row0;
            a.row1 = ph->row1;
            a.resume = ph->resume;
            a.pool = ph->pool;
            a.pool_cap = ph->pool_cap;
            a.pool_ctr = ph->pool_ctr;
            a.park_list = ph->park_list;
            a.ld_park = ph->ld_park;
            a.park_cnt = ph->park_cnt;
        }
        if (w > kLaneMaxW && low_latency) return launch_dtw_wavereg_wide(p, w, num_cu, a, s);
        if (w > kLaneMaxW) return launch_dtw_strip(p, w, num_cu, a, ring, ring_bytes, s);
        if (low_latency) return launch_dtw_wavereg(p, w, num_cu, a, s);
        if (p == 1) return launch_dtw_lane_p1(w, num_cu, a, s);
        return p == 2 ? launch_dtw_lane_p2(w, num_cu, a, s) : launch_dtw_lane_pinf(w, num_cu, a, s);
    }
    const size_t lds = sizeof(float) * (3 * (size_t)n + 3);
#define LBIMP_DTW_WAVE(PP)                                                                                          \
    hipLaunchKernelGGL(k_dtw_wave<PP>, dim3(persistent_grid(k_dtw_wave<PP>, lds, num_cu)), dim3(64), lds, s, rows, n, w, \
                       qd, pl, prefix, Q, ctr, best, thr, res, ldres, rescnt, abandoned, out_root, abandon)
    if (p == 1)
        LBIMP_DTW_WAVE(1);
    else if (p == 2)
        LBIMP_DTW_WAVE(2);
    else
        LBIMP_DTW_WAVE(kPInf);
#undef LBIMP_DTW_WAVE
    return hipGetLastError();
}

// ------------------------------------------------------------------ thresholds and results
// 64-entry bitonic sort in LDS of one query's first min(cnt, 64) keys; the threshold is the
// k-th smallest, with k = kq[q] when a per-query array is given.
__global__ __launch_bounds__(64) void k_kth_key(const u64 *__restrict__ res, int64_t ldres,
                                                const int *__restrict__ rescnt, int k, const int64_t *__restrict__ kq,
                                                u64 *__restrict__ thr) {
    __shared__ u64 keys[64];
    const int64_t q = blockIdx.x;
    const int cnt = min(rescnt[q], 64);
    const int kk = kq ? (int)kq[q] : k;
    keys[threadIdx.x] = threadIdx.x < cnt ? res[q * ldres + threadIdx.x] : kNoKey;
    __syncthreads();
    for (int size = 2; size <= 64; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (threadIdx.x < 32) {
                int t = threadIdx.x;
                int i = 2 * t - (t & (stride - 1));
                int j = i + stride;
                bool up = (i & size) == 0;
                u64 a = keys[i], bb = keys[j];
                if ((a > bb) == up) {
                    keys[i] = bb;
                    keys[j] = a;
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) thr[q] = (cnt >= kk) ? keys[kk - 1] : kNoKey;
}

hipError_t launch_kth_key(const unsigned long long *res, int64_t ldres, const int *rescnt, int64_t Q, int k,
                          const int64_t *kq, unsigned long long *thr, hipStream_t s) {
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kth_key, dim3((unsigned)Q), dim3(64), 0, s, res, ldres, rescnt, k, kq, thr);
    return hipGetLastError();
}

__device__ __forceinline__ float key_root(u64 key, int p) {
    float v = __uint_as_float((unsigned)(key >> 32));
    return p == 2 ? sqrtf(v) : v;
}

// Output row r holds ldo entries: the best key in entry 0, -1 / +inf in the others.
__global__ void k_finalize1(const u64 *__restrict__ best, int64_t Q, int p, int64_t *__restrict__ idx,
                            float *__restrict__ dist, const int64_t *__restrict__ qmap, int ldo) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const u64 key = best[q];
    const int64_t row = (qmap ? qmap[q] : q) * ldo;
    if (key == kNoKey) {
        idx[row] = -1;
        dist[row] = kInf;
    } else {
        idx[row] = (int64_t)(key & 0xffffffffu);
        dist[row] = key_root(key, p);
    }
    for (int r = 1; r < ldo; ++r) {
        idx[row + r] = -1;
        dist[row + r] = kInf;
    }
}

hipError_t launch_finalize1(const unsigned long long *best, int64_t Q, int p, int64_t *idx, float *dist,
                            const int64_t *qmap, int ldo, hipStream_t s) {
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize1, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, best, Q, p, idx, dist, qmap,
                       ldo);
    return hipGetLastError();
}

__global__ void k_gather_rows(const float *__restrict__ src, const int64_t *__restrict__ off, int n, int64_t total,
                              float *__restrict__ dst) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int64_t j = g / n;
    const int i = (int)(g - j * n);
    dst[g] = src[off[j] + i];
}

hipError_t launch_gather_rows(const float *src, const int64_t *off, int n, int64_t count, float *dst, hipStream_t s) {
    const int64_t total = count * n;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, off, n, total, dst);
    return hipGetLastError();
}

// k rounds of a block-wide minimum (k = kq[q] when a per-query array is given); each
// selected key is removed before the next round.  Entries k .. ldo-1 of the output row get
// -1 / +inf.
__global__ __launch_bounds__(256) void k_finalize_k(u64 *__restrict__ res, int64_t ldres,
                                                    const int *__restrict__ rescnt, int k,
                                                    const int64_t *__restrict__ kq, int ldo, int p,
                                                    int64_t *__restrict__ idx, float *__restrict__ dist,
                                                    const int64_t *__restrict__ qmap) {
    __shared__ u64 red[256];
    const int64_t q = blockIdx.x;
    const int cnt = rescnt[q];
    const int kk = kq ? (int)kq[q] : k;
    const int64_t row = (qmap ? qmap[q] : q) * ldo;
    u64 *r = res + q * ldres;
    for (int round = 0; round < kk; ++round) {
        u64 m = kNoKey;
        for (int t = threadIdx.x; t < cnt; t += 256) m = min(m, r[t]);
        red[threadIdx.x] = m;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + off]);
            __syncthreads();
        }
        const u64 best = red[0];
        __syncthreads();
        if (best != kNoKey) {
            for (int t = threadIdx.x; t < cnt; t += 256)
                if (r[t] == best) r[t] = kNoKey;
        }
        if (threadIdx.x == 0) {
            idx[row + round] = best == kNoKey ? -1 : (int64_t)(best & 0xffffffffu);
            dist[row + round] = best == kNoKey ? kInf : key_root(best, p);
        }
        __syncthreads();
    }
    for (int t = kk + threadIdx.x; t < ldo; t += 256) {
        idx[row + t] = -1;
        dist[row + t] = kInf;
    }
}

hipError_t launch_finalize_k(unsigned long long *res, int64_t ldres, const int *rescnt, int64_t Q, int k,
                             const int64_t *kq, int ldo, int p, int64_t *idx, float *dist, const int64_t *qmap,
                             hipStream_t s) {
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_k, dim3((unsigned)Q), dim3(256), 0, s, res, ldres, rescnt, k, kq, ldo, p, idx,
                       dist, qmap);
    return hipGetLastError();
}

// Between two chunks of a search over a database split into candidate ranges: keep the k
// smallest keys of res[q] (k = kq[q] when given), sorted, as its only entries, and make the
// k-th of them the threshold of the next chunk (no key if fewer than k).
__global__ __launch_bounds__(256) void k_res_shrink(u64 *__restrict__ res, int64_t ldres, int *__restrict__ rescnt,
                                                     int k, const int64_t *__restrict__ kq, u64 *__restrict__ thr) {
    __shared__ u64 red[256];
    __shared__ u64 kept[64];
    const int64_t q = blockIdx.x;
    const int cnt = rescnt[q];
    const int kk = kq ? (int)kq[q] : k;
    u64 *r = res + q * ldres;
    int got = 0;
    for (int round = 0; round < kk; ++round) {
        u64 m = kNoKey;
        for (int t = threadIdx.x; t < cnt; t += 256) m = min(m, r[t]);
        red[threadIdx.x] = m;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + off]);
            __syncthreads();
        }
        const u64 best = red[0];
        __syncthreads();
        if (best == kNoKey) break;
        for (int t = threadIdx.x; t < cnt; t += 256)
            if (r[t] == best) r[t] = kNoKey;
        if (threadIdx.x == 0) kept[round] = best;
        ++got;
        __syncthreads();
    }
    __syncthreads();
    for (int t = threadIdx.x; t < got; t += 256) r[t] = kept[t];
    if (threadIdx.x == 0) {
        rescnt[q] = got;
        thr[q] = got >= kk ? kept[kk - 1] : kNoKey;
    }
}

hipError_t launch_res_shrink(unsigned long long *res, int64_t ldres, int *rescnt, int64_t Q, int k, const int64_t *kq,
                             unsigned long long *thr, hipStream_t s) {
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_res_shrink, dim3((unsigned)Q), dim3(256), 0, s, res, ldres, rescnt, k, kq, thr);
    return hipGetLastError();
}

// tot[r][q] += cnt[rows[r]][q] and the counter is cleared, for the three list counts of a chunk.
__global__ void k_chunk_counts(int *__restrict__ counters, long long *__restrict__ tot, int64_t Q) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const int rows[3] = {0, 1, 4};  // cnt1, cnt2, cnt0
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        tot[r * Q + q] += counters[rows[r] * Q + q];
        counters[rows[r] * Q + q] = 0;
    }
}

hipError_t launch_chunk_counts(int *counters, long long *tot, int64_t Q, hipStream_t s) {
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_counts, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, counters, tot, Q);
    return hipGetLastError();
}

}  // namespace lbimp
