// Second pruning pass, LB_Improved (Sec. 8 of Lemire, arXiv:0811.3301), with the per-lane
// envelope state in registers: one instantiation per band half-width W.
#pragma once

#include <array>
#include <utility>

#include "device_common.h"

namespace lbimp {

// Lane per (query, candidate) pair, 64 pairs of one query per wave.  For candidate x:
// x' = H(x, y) = med3(x, L, U) (the projection of Sec. 7), the envelope (U', L') of x' with the
// same w, and S2 = S1 + sum_i d(y_i, [L'_i, U'_i])^p.
//
// The envelope of x' is streamed with van Herk / Gil-Werman blocks of K = 2W+1 positions e
// (aligned at 0).  Walking block B forward keeps g = running max/min from the block start; the
// window of output i = e - W starts at s = e - K + 1, which lies in block B-1 at offset o+1 (or
// at the start of block B when o = K-1, where the neutral entry h[K] applies), so the window
// value is max(h[o+1], g) with h the suffix max/min of block B-1, built by walking B-1
// backwards.  h lives in registers (compile-time offsets); x' of the current block is staged
// in LDS, transposed ([offset][pair]) so each lane reads its own column without bank
// conflicts.  The staging loads are coalesced: for pair j the wave reads K consecutive floats
// of row c_j, one per lane, and applies the clamp on the way in.
// Early abandoning (a.abandon, with a threshold): the bound only grows as terms are added, so a
// pair is pruned once S1 combined with the terms so far reaches the threshold key; the wave
// leaves the block loop when every one of its pairs has (a lane alone cannot skip work).
// Positions e >= n repeat x'[n-1]: every window of an output i < n that reaches past the end
// contains n-1, so the repeated value changes no maximum or minimum.
// For bands w >= 20 the LDS values (x' of the pair, y of the query) are read in groups of four
// offsets, one group ahead of the arithmetic that uses them (a scheduling barrier keeps them
// there), so the LDS latency is covered by a group of work instead of a few instructions
// (measured: 6% faster at w = 26, 5% slower at w = 13, where the compiler's own order is kept).
// In the last block (PARTIAL) offsets past olim (outputs past the series) add nothing; their x'
// repeat x'[n-1], which changes no running maximum or minimum.
template <int W>
constexpr int lbi_group() { return W >= 20 ? 4 : 1; }

template <int P, int W, bool FIRST, bool PARTIAL>
__device__ __forceinline__ void lbi_forward(float &acc, const float (&hx)[2 * W + 2], const float (&hn)[2 * W + 2],
                                            const float *stage, const float *yb, int olim, int lane) {
    constexpr int K = 2 * W + 1;
    constexpr int G = lbi_group<W>(), NG = (K + G - 1) / G;
    float gx = -kInf, gn = kInf;
    if constexpr (G == 1) {
#pragma unroll
        for (int o = 0; o < K; ++o) {
            if (!PARTIAL || o < olim) {
                const float v = stage[o * 65 + lane];
                gx = fmaxf(gx, v);
                gn = fminf(gn, v);
                if (!FIRST || o >= W) {  // in the first block, windows of o < W start before the series
                    const float um = fmaxf(hx[o + 1], gx);
                    const float lm = fminf(hn[o + 1], gn);
                    const float yv = yb[o - W];
                    const float d = yv - __builtin_amdgcn_fmed3f(yv, lm, um);
                    acc = pacc<P>(acc, d);
                }
            }
        }
        return;
    }
    float v[2][G], y[2][G];
    auto fetch = [&](int g, float (&vv)[G], float (&yy)[G]) {
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int o = g * G + t;
            if (o < K) {
                vv[t] = stage[o * 65 + lane];
                if (!FIRST || o >= W) yy[t] = yb[o - W];  // in the first block, windows of o < W start before the series
            }
        }
    };
    fetch(0, v[0], y[0]);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG) fetch(g + 1, v[(g + 1) & 1], y[(g + 1) & 1]);
        if constexpr (G > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int o = g * G + t;
            if (o < K) {
                const float x = v[g & 1][t];
                gx = fmaxf(gx, x);
                gn = fminf(gn, x);
                if (!FIRST || o >= W) {
                    const float um = fmaxf(hx[o + 1], gx);
                    const float lm = fminf(hn[o + 1], gn);
                    const float yv = y[g & 1][t];
                    float d = yv - __builtin_amdgcn_fmed3f(yv, lm, um);
                    if (PARTIAL) d = o < olim ? d : 0.f;
                    acc = pacc<P>(acc, d);
                }
            }
        }
    }
}

// Suffix maximum and minimum of the staged block, in place (hx[K], hn[K] stay neutral), with the
// LDS reads a group ahead as in the forward pass.
template <int W>
__device__ __forceinline__ void lbi_suffix(float (&hx)[2 * W + 2], float (&hn)[2 * W + 2], const float *stage, int lane) {
    constexpr int K = 2 * W + 1;
    constexpr int G = lbi_group<W>(), NG = (K + G - 1) / G;
    if constexpr (G == 1) {
#pragma unroll
        for (int o = K - 1; o >= 0; --o) {
            const float v = stage[o * 65 + lane];
            hx[o] = fmaxf(hx[o + 1], v);
            hn[o] = fminf(hn[o + 1], v);
        }
        return;
    }
    float v[2][G];
    auto fetch = [&](int g, float (&vv)[G]) {
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int o = K - 1 - (g * G + t);
            if (o >= 0) vv[t] = stage[o * 65 + lane];
        }
    };
    fetch(0, v[0]);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG) fetch(g + 1, v[(g + 1) & 1]);
        if constexpr (G > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int o = K - 1 - (g * G + t);
            if (o >= 0) {
                hx[o] = fmaxf(hx[o + 1], v[g & 1][t]);
                hn[o] = fminf(hn[o + 1], v[g & 1][t]);
            }
        }
    }
}

template <int P, int W, int DEPTH>
__global__ __launch_bounds__(64) void k_lbi_reg(LbiArgs a) {
    constexpr int K = 2 * W + 1;
    extern __shared__ float sm[];
    const int n = a.n;
    float *sY = sm;                   // [n]
    float *stage = sm + n;            // [K][65]
    unsigned *soff = reinterpret_cast<unsigned *>(stage + K * 65);  // [64]
    const int lane = threadIdx.x;
    const int nblk = (n + W + K - 1) / K;
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(a.pl, a.prefix, a.Q, 64);
    while (items.get(q, b)) {
        if (q != cur_q) {
            __syncthreads();
            const float *y = a.qd.Y + q * a.qd.ldy;
            stage_lds(sY, n, [&](int i) { return y[i]; });
            cur_q = q;
        }
        const float *Uq = a.qd.U + q * a.qd.ldq;
        const float *Lq = a.qd.L + q * a.qd.ldq;
        const long long j = b * 64 + lane;
        const bool active = j < pair_count(a.pl, q, items.bk);
        const int c = active ? pair_cand(a.pl, q, j, items.bk) : 0;
        const float s1 = active ? a.S1[q * a.ldS + c] : 0.f;
        const bool abandon = a.abandon && a.thr && !a.out_root;
        const u64 tq = a.thr ? a.thr[q] : kNoKey;
        float hx[K + 1], hn[K + 1];
#pragma unroll
        for (int o = 0; o <= K; ++o) {
            hx[o] = -kInf;
            hn[o] = kInf;
        }
        float acc = 0.f;
        // Bands with K <= 64 are software-pipelined (DEPTH 1): the raw values of the next block
        // are loaded into registers (one per pair) while the current block is processed, and
        // clamped into LDS once the stage is free.  The loads are buffer loads with a 32-bit byte
        // offset (one address register each), so the database must be below 2 GiB for this path.
        // Wider bands, larger databases and DEPTH 0 stage each block in batches of 16 loads.
        constexpr int D = K <= 64 ? DEPTH : 0;
        const bool pipe = D > 0 && a.db_bytes < 0x80000000ll;
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc((void *)a.rows, (short)0, pipe ? (int)a.db_bytes : 0, 0x00020000);
        // byte offsets of the 64 rows, read back from LDS (not hoisted across barriers, so they
        // do not pin 64 registers for the whole item)
        __syncthreads();
        soff[lane] = (unsigned)c * (unsigned)n * 4u;
        __syncthreads();
        // a block loaded ahead: the raw row values (one per pair) and the query envelope at the
        // lane's position, all requested together so that staging waits on one round trip that
        // the previous block's computation has covered
        float va[D >= 1 ? 64 : 1];
        float ua = 0.f, la = 0.f;
        auto load_block = [&](auto &v, float &u, float &l, int e0n) {
            const int er = min(e0n + lane, n - 1);
            u = Uq[er];
            l = Lq[er];
            const unsigned eb = (unsigned)er * 4u;
#pragma unroll
            for (int t = 0; t < (D >= 1 ? 64 : 1); ++t)
                v[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, soff[t] + eb, 0, 0));
        };
        auto stage_from = [&](const auto &v, float u, float l) {
            if (lane < K) {
#pragma unroll
                for (int t = 0; t < (D >= 1 ? 64 : 1); ++t) stage[lane * 65 + t] = __builtin_amdgcn_fmed3f(v[t], l, u);
            }
        };
        auto stage_batched = [&](int e0) {
#pragma unroll
            for (int r0 = 0; r0 < K; r0 += 64) {
                const int er = min(e0 + r0 + lane, n - 1);
                const float ur = Uq[er], lr = Lq[er];
#pragma unroll 1
                for (int j0 = 0; j0 < 64; j0 += 16) {
                    float v[16];
#pragma unroll
                    for (int t = 0; t < 16; ++t) v[t] = a.rows[(int64_t)__shfl(c, j0 + t) * n + er];
                    if (r0 + lane < K) {
#pragma unroll
                        for (int t = 0; t < 16; ++t)
                            stage[(r0 + lane) * 65 + j0 + t] = __builtin_amdgcn_fmed3f(v[t], lr, ur);
                    }
                }
            }
        };
        // forward pass of block B over the staged x', then (unless it is the last) the suffix
        // max/min of the block in place; true when every pair of the wave has been abandoned
        auto compute_block = [&](int B) -> bool {
            const int e0 = B * K;
            const float *yb = sY + e0;  // yb[o - W] = y[e - W]
            const int olim = n + W - e0;
            if (B == 0) {
                if (olim < K)
                    lbi_forward<P, W, true, true>(acc, hx, hn, stage, yb, olim, lane);
                else
                    lbi_forward<P, W, true, false>(acc, hx, hn, stage, yb, olim, lane);
            } else if (olim < K) {
                lbi_forward<P, W, false, true>(acc, hx, hn, stage, yb, olim, lane);
            } else {
                lbi_forward<P, W, false, false>(acc, hx, hn, stage, yb, olim, lane);
            }
            if (abandon && B + 1 < nblk && __ballot(active && make_key(pjoin<P>(s1, acc), c) < tq) == 0) return true;
            if (B + 1 < nblk) lbi_suffix<W>(hx, hn, stage, lane);
            return false;
        };
        if (D >= 1 && pipe) {
            load_block(va, ua, la, 0);
            for (int B = 0; B < nblk; ++B) {
                __syncthreads();  // the previous block's readers are done with the stage
                stage_from(va, ua, la);
                __syncthreads();
                if (B + 1 < nblk) load_block(va, ua, la, (B + 1) * K);
                if (compute_block(B)) break;
            }
        } else {
            for (int B = 0; B < nblk; ++B) {
                __syncthreads();
                stage_batched(B * K);
                __syncthreads();
                if (compute_block(B)) break;
            }
        }
        const float s2 = pjoin<P>(s1, acc);
        if (a.out_root && active) a.out_root[c] = root_p<P>(s2);
        if (a.thr) {
            const bool keep = active && make_key(s2, c) < a.thr[q];
            const u64 m = __ballot(keep);
            if (m) {
                int pos = 0;
                if (lane == 0) pos = atomicAdd(&a.cnt2[q], __popcll(m));
                pos = __shfl(pos, 0);
                if (keep) a.list2[q * a.ldl2 + pos + __popcll(m & ((1ull << lane) - 1ull))] = c;
            }
        }
    }
}

template <int P, int W>
static void lbi_reg_launch(int num_cu, const LbiArgs &a, hipStream_t s) {
    constexpr int K = 2 * W + 1;
    const size_t lds = sizeof(float) * ((size_t)a.n + (size_t)K * 65 + 64);
#define LBIMP_LBI_REG(DD) \
    hipLaunchKernelGGL((k_lbi_reg<P, W, DD>), dim3(persistent_grid(k_lbi_reg<P, W, DD>, lds, num_cu)), dim3(64), lds, s, a)
    if constexpr (K <= 64) {
        if (a.pipeline) {
            LBIMP_LBI_REG(1);
            return;
        }
    }
    LBIMP_LBI_REG(0);
#undef LBIMP_LBI_REG
}

using LbiRegFn = void (*)(int, const LbiArgs &, hipStream_t);

template <int P, int... Ws>
constexpr std::array<LbiRegFn, sizeof...(Ws)> lbi_reg_table(std::integer_sequence<int, Ws...>) {
    return {&lbi_reg_launch<P, Ws>...};
}

}  // namespace lbimp
