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
// backwards.  h lives in registers (compile-time offsets).  x' of the current block is staged
// in LDS one row per pair ([pair][S], S = 4 * odd >= K), so a lane reads four offsets of its
// own pair with one 16-byte read whose address is fixed per lane (no address arithmetic), and
// 16 lanes reading rows S floats apart touch disjoint banks.  The staging loads are coalesced:
// for pair j the wave reads K consecutive floats of row c_j, one per lane, and applies the clamp
// on the way in; lanes writing consecutive offsets of one row write disjoint banks.  The query
// values of the block's outputs are copied to an aligned row of S floats beside the stage and
// read four at a time by all lanes at once.  Each pass reads its next group of four offsets
// one group ahead of the arithmetic (a scheduling barrier keeps the reads there), so the LDS
// latency is covered by a group of work.
// Early abandoning (a.abandon, with a threshold): the bound only grows as terms are added, so a
// pair is pruned once S1 combined with the terms so far reaches the threshold key; the wave
// leaves the block loop when every one of its pairs has (a lane alone cannot skip work).
// Positions e >= n repeat x'[n-1]: every window of an output i < n that reaches past the end
// contains n-1, so the repeated value changes no maximum or minimum.
// In the last block (PARTIAL) the pass stops at olim (outputs past the series), a branch that is
// uniform over the wave, so a short last block costs only its own positions.
// Narrow bands stage KB consecutive blocks at once (as many as fit in the 64 lanes, at most
// four), so that the loads and clamps of a stage keep most lanes busy; block b of a stage sits at
// offset b * SK of a pair's row (SK = K rounded up to four, keeping the 16-byte reads aligned).
template <int W>
constexpr int lbi_blocks_per_stage() {
    constexpr int K = 2 * W + 1;
    return K > 32 ? 1 : (64 / K > 4 ? 4 : 64 / K);
}
template <int W>
constexpr int lbi_seg() { return (2 * W + 1 + 3) / 4 * 4; }
template <int W>
constexpr int lbi_stride() {
    constexpr int m = lbi_blocks_per_stage<W>() * lbi_seg<W>() / 4;
    return 4 * (m | 1);
}

template <int T>
__device__ __forceinline__ float f4get(const float4 &v) {
    if constexpr (T == 0) return v.x;
    if constexpr (T == 1) return v.y;
    if constexpr (T == 2) return v.z;
    return v.w;
}

// xs: this lane's staged row of x' (16-byte aligned); ys: the query values of the block's
// outputs, ys[o] = y[e - W] for offset o (read only where an output exists).  Fused (F): xs holds
// the raw row and us, ls the query envelope at the block's offsets; the clamp to the envelope is
// taken here, the LB_Keogh terms |x - x'|^p accumulate into s1 (positions past the series are
// staged so that their term is zero), and x' is written back over the raw row group by group for
// the suffix pass (which a last, partial block does not need).
template <int P, int W, bool FIRST, bool PARTIAL, bool F>
__device__ __forceinline__ void lbi_forward(float &acc, float &s1, const float (&hx)[2 * W + 2],
                                            const float (&hn)[2 * W + 2], float4 *xs, const float4 *ys,
                                            const float4 *us, const float4 *ls, int olim) {
    constexpr int K = 2 * W + 1;
    constexpr int NG = (K + 3) / 4;
    float gx = -kInf, gn = kInf;
    float4 xv[2], yv[2], uv, lv;  // F: the envelope of the current group only (registers are short)
    xv[0] = xs[0];
    yv[0] = ys[0];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if constexpr (F) {
            uv = us[g];
            lv = ls[g];
        }
        if (g + 1 < NG) {
            xv[(g + 1) & 1] = xs[g + 1];
            yv[(g + 1) & 1] = ys[g + 1];
        }
        __builtin_amdgcn_sched_barrier(0);
        float4 xo = xv[g & 1];  // F: this group's x'
        auto step = [&](auto tc) {
            constexpr int t = decltype(tc)::value;
            const int o = 4 * g + t;
            if (o < K) {
                if (PARTIAL && o >= olim) return false;  // uniform: the rest of the block is past the series
                float x = f4get<t>(xv[g & 1]);
                if constexpr (F) {
                    const float raw = x;
                    x = __builtin_amdgcn_fmed3f(raw, f4get<t>(lv), f4get<t>(uv));
                    s1 = pacc<P>(s1, raw - x);
                    if constexpr (t == 0) xo.x = x;
                    if constexpr (t == 1) xo.y = x;
                    if constexpr (t == 2) xo.z = x;
                    if constexpr (t == 3) xo.w = x;
                }
                gx = fmaxf(gx, x);
                gn = fminf(gn, x);
                if (!FIRST || o >= W) {  // in the first block, windows of o < W start before the series
                    // the first block's windows start at position 0: the running max/min alone
                    const float um = FIRST ? gx : fmaxf(hx[o + 1], gx);
                    const float lm = FIRST ? gn : fminf(hn[o + 1], gn);
                    const float yo = f4get<t>(yv[g & 1]);
                    const float d = yo - __builtin_amdgcn_fmed3f(yo, lm, um);
                    acc = pacc<P>(acc, d);
                }
            }
            return true;
        };
        if (!step(std::integral_constant<int, 0>{})) return;
        if (!step(std::integral_constant<int, 1>{})) return;
        if (!step(std::integral_constant<int, 2>{})) return;
        if (!step(std::integral_constant<int, 3>{})) return;
        if constexpr (F) xs[g] = xo;
    }
}

// Suffix maximum and minimum of the staged block, in place (hx[K], hn[K] stay neutral), reading
// the groups of four from the top, one group ahead (fused: clamping the raw row again).
template <int W, bool F>
__device__ __forceinline__ void lbi_suffix(float (&hx)[2 * W + 2], float (&hn)[2 * W + 2], const float4 *xs,
                                           const float4 *us, const float4 *ls) {
    constexpr int K = 2 * W + 1;
    constexpr int NG = (K + 3) / 4;
    float4 v[2], uv[2], lv[2];
    v[0] = xs[NG - 1];
    if constexpr (F) {
        uv[0] = us[NG - 1];
        lv[0] = ls[NG - 1];
    }
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int g = NG - 1 - gi;
        if (gi + 1 < NG) {
            v[(gi + 1) & 1] = xs[g - 1];
            if constexpr (F) {
                uv[(gi + 1) & 1] = us[g - 1];
                lv[(gi + 1) & 1] = ls[g - 1];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        auto step = [&](auto tc) {
            constexpr int t = decltype(tc)::value;
            const int o = 4 * g + t;
            if (o < K) {
                float x = f4get<t>(v[gi & 1]);
                if constexpr (F) x = __builtin_amdgcn_fmed3f(x, f4get<t>(lv[gi & 1]), f4get<t>(uv[gi & 1]));
                hx[o] = fmaxf(hx[o + 1], x);
                hn[o] = fminf(hn[o + 1], x);
            }
        };
        step(std::integral_constant<int, 3>{});
        step(std::integral_constant<int, 2>{});
        step(std::integral_constant<int, 1>{});
        step(std::integral_constant<int, 0>{});
    }
}

// F (fused): the list holds pass-0 survivors whose LB_Keogh has not been computed; the kernel
// stages raw rows, clamps them itself and sums LB_Keogh along the way (Algorithm 3's first bound,
// then its second, from one read of the row).  A pair counts in a.cntk[q] when its LB_Keogh
// alone stays below the threshold, and a surviving pair's LB_Keogh goes to a.S1out[q][c] for
// the DTW's abandon bound.  Early abandoning is off in this form (the counts need full sums).
template <int P, int W, int DEPTH, bool F>
__global__ __launch_bounds__(64) void k_lbi_reg(LbiArgs a) {
    constexpr int K = 2 * W + 1;
    extern __shared__ float sm[];
    const int n = a.n;
    constexpr int KB = lbi_blocks_per_stage<W>(), SK = lbi_seg<W>(), S = lbi_stride<W>();
    constexpr int SPAN = KB * K;      // positions staged together
    float *stage = sm;                // [64][S]: x' (raw x when F) of the stage's blocks, one row per pair
    float *ys = sm + 64 * S;          // [S]: y[e - W] of the stage's offsets
    float *us = ys + S;               // F: [S] U, then [S] L at the stage's offsets
    float *ls = us + (F ? S : 0);
    float *sY = ls + (F ? S : 0);     // [n]
    const int lane = threadIdx.x;
    const int nblk = (n + W + K - 1) / K;
    const int nsb = (nblk + KB - 1) / KB;
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(a.pl, a.prefix, a.Q, 64, true);  // contiguous: few query changes per block
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
        float s1 = (!F && active) ? a.S1[q * a.ldS + c] : 0.f;
        const bool abandon = a.abandon && a.thr && !a.out_root && !F;
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
        // byte offset of the lane's row; the loads of a block take row t's offset from lane t
        // into the scalar offset of the buffer load, so a load costs no vector instruction
        const unsigned roff = (unsigned)c * (unsigned)n * 4u;
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
                v[t] = __uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(rsrc, eb, __builtin_amdgcn_readlane(roff, t), 0));
        };
        // position l of a stage (block l / K, offset l % K) goes to offset dst_of(l) of a row
        auto dst_of = [&](int l) { return l / K * SK + l % K; };
        // F: a position past the series stages the clamped last value with an envelope of +-inf
        // (its clamp is then the identity and its LB_Keogh term zero); others stage the raw value
        auto stage_from = [&](const auto &v, float u, float l, int e0) {
            if (lane < SPAN) {
                const int dst = dst_of(lane);
                const bool tail = e0 + lane >= n;
                const float lo = (!F || tail) ? l : -kInf, hi = (!F || tail) ? u : kInf;
                if (F && e0 + SPAN <= n) {  // uniform: no position past the series, the raw row is staged as is
#pragma unroll
                    for (int t = 0; t < (D >= 1 ? 64 : 1); ++t) stage[t * S + dst] = v[t];
                } else {
#pragma unroll
                    for (int t = 0; t < (D >= 1 ? 64 : 1); ++t)
                        stage[t * S + dst] = __builtin_amdgcn_fmed3f(v[t], lo, hi);
                }
                ys[dst] = sY[min(max(e0 + lane - W, 0), n - 1)];
                if constexpr (F) {
                    us[dst] = tail ? kInf : u;
                    ls[dst] = tail ? -kInf : l;
                }
            }
        };
        auto stage_batched = [&](int e0) {
#pragma unroll
            for (int r0 = 0; r0 < SPAN; r0 += 64) {
                const int er = min(e0 + r0 + lane, n - 1);
                const float ur = Uq[er], lr = Lq[er];
                const int dst = dst_of(r0 + lane);
                const bool tail = e0 + r0 + lane >= n;
                const float lo = (!F || tail) ? lr : -kInf, hi = (!F || tail) ? ur : kInf;
                if (r0 + lane < SPAN) {
                    ys[dst] = sY[min(max(e0 + r0 + lane - W, 0), n - 1)];
                    if constexpr (F) {
                        us[dst] = tail ? kInf : ur;
                        ls[dst] = tail ? -kInf : lr;
                    }
                }
#pragma unroll 1
                for (int j0 = 0; j0 < 64; j0 += 16) {
                    float v[16];
#pragma unroll
                    for (int t = 0; t < 16; ++t) v[t] = a.rows[(int64_t)__shfl(c, j0 + t) * n + er];
                    if (r0 + lane < SPAN) {
#pragma unroll
                        for (int t = 0; t < 16; ++t)
                            stage[(j0 + t) * S + dst] = __builtin_amdgcn_fmed3f(v[t], lo, hi);
                    }
                }
            }
        };
        // forward pass of block B over the staged x', then (unless it is the last) the suffix
        // max/min of the block in place; true when every pair of the wave has been abandoned
        auto compute_block = [&](int B, int b) __attribute__((always_inline)) -> bool {
            const int olim = n + W - B * K;
            float4 *xs = reinterpret_cast<float4 *>(stage + lane * S + b * SK);
            const float4 *y4 = reinterpret_cast<const float4 *>(ys + b * SK);
            const float4 *u4 = reinterpret_cast<const float4 *>(us + b * SK);
            const float4 *l4 = reinterpret_cast<const float4 *>(ls + b * SK);
            if (B == 0) {
                if (olim < K)
                    lbi_forward<P, W, true, true, F>(acc, s1, hx, hn, xs, y4, u4, l4, olim);
                else
                    lbi_forward<P, W, true, false, F>(acc, s1, hx, hn, xs, y4, u4, l4, olim);
            } else if (olim < K) {
                lbi_forward<P, W, false, true, F>(acc, s1, hx, hn, xs, y4, u4, l4, olim);
            } else {
                lbi_forward<P, W, false, false, F>(acc, s1, hx, hn, xs, y4, u4, l4, olim);
            }
            if (abandon && B + 1 < nblk && __ballot(active && make_key(pjoin<P>(s1, acc), c) < tq) == 0) return true;
            if (B + 1 < nblk) lbi_suffix<W, false>(hx, hn, xs, u4, l4);  // x' is in the stage now
            return false;
        };
        // the blocks of stage sb in order; true when every pair of the wave has been abandoned
        auto run_stage = [&](int sb) __attribute__((always_inline)) -> bool {
            if constexpr (KB == 1) return compute_block(sb, 0);
#pragma unroll 1
            for (int b = 0; b < KB; ++b) {
                const int B = sb * KB + b;
                if (B >= nblk) break;
                if (compute_block(B, b)) return true;
            }
            return false;
        };
        if (D >= 1 && pipe) {
            load_block(va, ua, la, 0);
            for (int sb = 0; sb < nsb; ++sb) {
                __syncthreads();  // the previous stage's readers are done with it
                stage_from(va, ua, la, sb * SPAN);
                __syncthreads();
                if (sb + 1 < nsb) load_block(va, ua, la, (sb + 1) * SPAN);
                if (run_stage(sb)) break;
            }
        } else {
            for (int sb = 0; sb < nsb; ++sb) {
                __syncthreads();
                stage_batched(sb * SPAN);
                __syncthreads();
                if (run_stage(sb)) break;
            }
        }
        const float s2 = pjoin<P>(s1, acc);
        if (a.out_root && active) a.out_root[c] = root_p<P>(s2);
        if constexpr (F) {
            const u64 mk = __ballot(active && make_key(s1, c) < tq);
            if (lane == 0 && mk) atomicAdd(&a.cntk[q], __popcll(mk));
            if (active && make_key(s2, c) < tq) a.S1out[q * a.ldS + c] = s1;
        }
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
    const size_t lds = sizeof(float) * ((size_t)a.n + (a.fused ? 67 : 65) * (size_t)lbi_stride<W>());
#define LBIMP_LBI_REG(DD, FF)                                                                                     \
    hipLaunchKernelGGL((k_lbi_reg<P, W, DD, FF>), dim3(persistent_grid(k_lbi_reg<P, W, DD, FF>, lds, num_cu)), \
                       dim3(64), lds, s, a)
    if (a.fused) {  // one depth: blocks loaded ahead where they fit
        LBIMP_LBI_REG(K <= 64 ? 1 : 0, true);
        return;
    }
    if constexpr (K <= 64) {
        if (a.pipeline) {
            LBIMP_LBI_REG(1, false);
            return;
        }
    }
    LBIMP_LBI_REG(0, false);
#undef LBIMP_LBI_REG
}

using LbiRegFn = void (*)(int, const LbiArgs &, hipStream_t);

template <int P, int... Ws>
constexpr std::array<LbiRegFn, sizeof...(Ws)> lbi_reg_table(std::integer_sequence<int, Ws...>) {
    return {&lbi_reg_launch<P, Ws>...};
}

}  // namespace lbimp
