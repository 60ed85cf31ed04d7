// Database layout, warping envelopes, the LB_Keogh sweep, seed selection and compaction.
//
// Cited passages (Lemire, arXiv:0811.3301): envelope definition (Sec. 5), LB_Keogh and the
// projection H (Sec. 7), the first pruning test of Algorithms 2 and 3 (Sec. 7, Sec. 8).
#include "internal.h"

namespace lbimp {

// ------------------------------------------------------------------ database layout
// Tile t holds candidates [64t, 64t+64); float4 (t, i4, lane) holds elements 4*i4..4*i4+3 of
// candidate 64t+lane.  A wave reading one i4 of one tile touches 1 KB of contiguous memory.
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ rows, int64_t N, int n, int n4,
                                               float4 *__restrict__ il, int64_t total) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int lane = (int)(g & 63);
    int64_t r = g >> 6;
    int i4 = (int)(r % n4);
    int64_t t = r / n4;
    int64_t c = t * 64 + lane;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (c < N) {
        const float *x = rows + c * (int64_t)n;
        for (int k = 0; k < 4; ++k) {
            int i = i4 * 4 + k;
            if (i < n) v[k] = x[i];
        }
    }
    il[g] = make_float4(v[0], v[1], v[2], v[3]);
}

hipError_t launch_pack(const float *rows, int64_t N, int n, float4 *il, hipStream_t s) {
    int n4 = (n + 3) / 4;
    int64_t T = (N + 63) / 64;
    int64_t total = T * n4 * 64;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rows, N, n, n4, il, total);
    return hipGetLastError();
}

// ------------------------------------------------------------------ envelopes (Sec. 5)
// van Herk / Gil-Werman: with blocks of length K = 2w+1 aligned at 0, every window [s, e]
// (cut to the series) lies in one block or spans two neighbours.  g = running max/min from
// the block start, h = running max/min to the block end; the window value is
// max(h[s], g[e]) across a block boundary, g[e] when s starts its block, h[s] when the
// window is cut by the series end inside one block.
// Narrow bands (2w+1 <= kDirectWindow) take the window maximum and minimum of every output
// directly, one output per thread, from the series in LDS: the plain definition, with no
// serial walk.  keys0 / keys1 (optional) are set to "no key" and counts4 (optional, [kCounters][B])
// to 0 for the B real rows, so a search needs no separate fill launches for its best-so-far
// and threshold keys and its per-query counters.
constexpr int kDirectWindow = 128;
__global__ __launch_bounds__(256) void k_envelope(const float *__restrict__ y, int64_t B, int n, int w,
                                                   float *__restrict__ U, float *__restrict__ L, int ldo,
                                                   unsigned long long *__restrict__ keys0,
                                                   unsigned long long *__restrict__ keys1, int *__restrict__ counts4) {
    extern __shared__ float sm[];
    int64_t b = blockIdx.x;
    float *Ub = U + b * (int64_t)ldo;
    float *Lb = L + b * (int64_t)ldo;
    if (b >= B) {  // padding rows: an envelope that contains every value
        for (int i = threadIdx.x; i < ldo; i += blockDim.x) {
            Ub[i] = kInf;
            Lb[i] = -kInf;
        }
        return;
    }
    if (threadIdx.x == 0) {
        if (keys0) keys0[b] = kNoKey;
        if (keys1) keys1[b] = kNoKey;
    }
    if (counts4 && threadIdx.x < kCounters) counts4[threadIdx.x * B + b] = 0;
    const float *yb = y + b * (int64_t)n;
    float *gmax = sm, *gmin = sm + n, *hmax = sm + 2 * n, *hmin = sm + 3 * n;
    // The series is first copied into hmin by the whole block (coalesced), so the reads below
    // wait on LDS, not on global memory.  The backward walk reads hmin[i] before it overwrites
    // it, going down, and different threads walk disjoint blocks.
    for (int i = threadIdx.x; i < n; i += blockDim.x) hmin[i] = yb[i];
    __syncthreads();
    const int K = 2 * w + 1;
    if (K <= kDirectWindow) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int s = max(0, i - w), e = min(n - 1, i + w);
            float u = -kInf, l = kInf;
            for (int j = s; j <= e; ++j) {
                const float v = hmin[j];
                u = fmaxf(u, v);
                l = fminf(l, v);
            }
            Ub[i] = u;
            Lb[i] = l;
        }
        for (int i = n + threadIdx.x; i < ldo; i += blockDim.x) {
            Ub[i] = kInf;
            Lb[i] = -kInf;
        }
        return;
    }
    const int nb = (n + K - 1) / K;
    for (int blk = threadIdx.x; blk < nb; blk += blockDim.x) {
        int s = blk * K, e = min(n, s + K);
        float mx = -kInf, mn = kInf;
        for (int i = s; i < e; ++i) {
            float v = hmin[i];
            mx = fmaxf(mx, v);
            mn = fminf(mn, v);
            gmax[i] = mx;
            gmin[i] = mn;
        }
        mx = -kInf;
        mn = kInf;
        for (int i = e - 1; i >= s; --i) {
            float v = hmin[i];
            mx = fmaxf(mx, v);
            mn = fminf(mn, v);
            hmax[i] = mx;
            hmin[i] = mn;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int s = max(0, i - w), e = min(n - 1, i + w);
        int bs = s / K, be = e / K;
        float u, l;
        if (bs != be) {
            u = fmaxf(hmax[s], gmax[e]);
            l = fminf(hmin[s], gmin[e]);
        } else if (s == bs * K) {
            u = gmax[e];
            l = gmin[e];
        } else {
            u = hmax[s];
            l = hmin[s];
        }
        Ub[i] = u;
        Lb[i] = l;
    }
    for (int i = n + threadIdx.x; i < ldo; i += blockDim.x) {
        Ub[i] = kInf;
        Lb[i] = -kInf;
    }
}

hipError_t launch_envelope(const float *y, int64_t B, int64_t Bpad, int n, int w, float *U, float *L, int ldo,
                           hipStream_t s, unsigned long long *keys0, unsigned long long *keys1, int *counts4) {
    if (Bpad == 0) return hipSuccess;
    size_t lds = sizeof(float) * 4 * (size_t)n;
    hipLaunchKernelGGL(k_envelope, dim3((unsigned)Bpad), dim3(256), lds, s, y, B, n, w, U, L, ldo, keys0, keys1,
                       counts4);
    return hipGetLastError();
}

__global__ void k_pad_env(const float *__restrict__ U, const float *__restrict__ L, int64_t B, int n,
                          float *__restrict__ Ud, float *__restrict__ Ld, int ldo, int64_t total) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int64_t b = g / ldo;
    int i = (int)(g % ldo);
    bool in = b < B && i < n;
    Ud[g] = in ? U[b * n + i] : kInf;
    Ld[g] = in ? L[b * n + i] : -kInf;
}

hipError_t launch_pad_env(const float *U, const float *L, int64_t B, int64_t Bpad, int n, float *Ud, float *Ld,
                          int ldo, hipStream_t s) {
    int64_t total = Bpad * ldo;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_env, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, U, L, B, n, Ud, Ld, ldo,
                       total);
    return hipGetLastError();
}

// ------------------------------------------------------------------ LB_Keogh sweep (Sec. 7)
// d(x, [L, U]) = x - med3(x, L, U): zero inside the envelope, x - U above, x - L below.
template <int P>
__device__ __forceinline__ float lb_term(float acc, float x, float l, float u) {
    return pacc<P>(acc, x - __builtin_amdgcn_fmed3f(x, l, u));
}

// Block = 4 waves; wave -> CPL consecutive tiles (lane = candidate), block.y -> QG queries.
// The QG envelopes are staged through LDS in chunks of ICH float4 and read as broadcasts;
// every candidate value is read from HBM once per query group.
template <int P, int QG, int CPL, bool ROOT>
__global__ __launch_bounds__(256) void k_lbk_sweep(const float4 *__restrict__ il, int64_t T, int64_t N, int n4,
                                                    const float4 *__restrict__ Ue, const float4 *__restrict__ Le,
                                                    int ld4, int64_t Q, float *__restrict__ out, int64_t ldo,
                                                    bool pad_inf, unsigned long long *__restrict__ wmin, int64_t ldw,
                                                    unsigned gx, unsigned gy, int64_t cbase) {
    constexpr int ICH = 32;
    __shared__ float4 sU[QG][ICH];
    __shared__ float4 sL[QG][ICH];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // One-dimensional grid of gx (candidate tile groups) x gy (query groups) blocks.  Blocks
    // are dealt to the 8 XCDs in turn (block b on XCD b % 8); renumbering them so that logical
    // neighbours share an XCD, with query groups fastest, runs the query groups of one tile
    // group back to back on one XCD, where its L2 serves the tile to all of them.
    const unsigned nb = gx * gy, per = nb / 8, blk = blockIdx.x;
    const unsigned lid = blk < per * 8 ? (blk % 8) * per + blk / 8 : blk;
    const unsigned bx = lid / gy, by = lid % gy;
    const int64_t tile0 = ((int64_t)bx * 4 + wave) * CPL;
    const int64_t q0 = (int64_t)by * QG;
    float acc[QG][CPL];
#pragma unroll
    for (int a = 0; a < QG; ++a)
#pragma unroll
        for (int b = 0; b < CPL; ++b) acc[a][b] = 0.f;

    const float4 *src[CPL];
    bool tv[CPL];
#pragma unroll
    for (int b = 0; b < CPL; ++b) {
        tv[b] = tile0 + b < T;
        src[b] = il + ((tv[b] ? tile0 + b : 0) * n4) * 64 + lane;
    }

    for (int c0 = 0; c0 < n4; c0 += ICH) {
        const int len = min(ICH, n4 - c0);
        __syncthreads();
        // Staged rotated: element k of L sits in component k+1 and of U in k+3 (mod 4).  The
        // register quads of x, L and U start at even registers, so the three operands of each
        // med3 (x, L, U of element k) then fall in three different VGPR banks (a med3 reading
        // one bank three times issues slower).  med3 is symmetric, so the result is unchanged.
        for (int t = threadIdx.x; t < QG * ICH; t += 256) {
            int qq = t / ICH, ii = t % ICH;
            if (ii < len) {
                const float4 u = Ue[(q0 + qq) * ld4 + c0 + ii];
                const float4 l = Le[(q0 + qq) * ld4 + c0 + ii];
                sU[qq][ii] = make_float4(u.y, u.z, u.w, u.x);
                sL[qq][ii] = make_float4(l.w, l.x, l.y, l.z);
            }
        }
        __syncthreads();
        for (int ii = 0; ii < len; ++ii) {
            float4 xv[CPL];
#pragma unroll
            for (int b = 0; b < CPL; ++b) xv[b] = src[b][(int64_t)(c0 + ii) * 64];
#pragma unroll
            for (int a = 0; a < QG; ++a) {
                const float4 u = sU[a][ii], l = sL[a][ii];
#pragma unroll
                for (int b = 0; b < CPL; ++b) {
                    float r = acc[a][b];
                    r = lb_term<P>(r, xv[b].x, l.y, u.w);
                    r = lb_term<P>(r, xv[b].y, l.z, u.x);
                    r = lb_term<P>(r, xv[b].z, l.w, u.y);
                    r = lb_term<P>(r, xv[b].w, l.x, u.z);
                    acc[a][b] = r;
                }
            }
        }
    }
    if (wmin) {
        // smallest (value, index) key of this wave's candidates, per query: seed candidates
        const int64_t wid = (int64_t)bx * 4 + wave;
#pragma unroll
        for (int a = 0; a < QG; ++a) {
            unsigned long long k = kNoKey;
#pragma unroll
            for (int b = 0; b < CPL; ++b) {
                const int64_t c = (tile0 + b) * 64 + lane;
                if (tv[b] && c < N) {
                    unsigned long long kb =
                        ((unsigned long long)__float_as_uint(acc[a][b]) << 32) | (unsigned long long)(c + cbase);
                    k = kb < k ? kb : k;
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                unsigned hi = __shfl_xor((unsigned)(k >> 32), off);
                unsigned lo = __shfl_xor((unsigned)k, off);
                unsigned long long o = ((unsigned long long)hi << 32) | lo;
                k = o < k ? o : k;
            }
            if (lane == 0 && q0 + a < Q) wmin[(q0 + a) * ldw + wid] = k;
        }
    }
#pragma unroll
    for (int a = 0; a < QG; ++a) {
        const int64_t q = q0 + a;
        if (q >= Q) continue;
#pragma unroll
        for (int b = 0; b < CPL; ++b) {
            if (!tv[b]) continue;
            const int64_t c = (tile0 + b) * 64 + lane;
            if (c < N)
                out[q * ldo + c] = ROOT ? root_p<P>(acc[a][b]) : acc[a][b];
            else if (pad_inf && c < ldo)
                out[q * ldo + c] = kInf;
        }
    }
}

template <int P, int QG, int CPL, bool ROOT>
static hipError_t sweep_variant(const float4 *il, int64_t N, int n4, const float4 *Ue, const float4 *Le, int ld4,
                                int64_t Q, float *out, int64_t ldo, bool pad_inf, unsigned long long *wmin,
                                int64_t cbase, hipStream_t s) {
    int64_t T = (N + 63) / 64;
    const unsigned gx = (unsigned)((T + 4 * CPL - 1) / (4 * CPL)), gy = (unsigned)((Q + QG - 1) / QG);
    hipLaunchKernelGGL((k_lbk_sweep<P, QG, CPL, ROOT>), dim3(gx * gy), dim3(256), 0, s, il, T, N, n4, Ue, Le, ld4, Q,
                       out, ldo, pad_inf, wmin, (int64_t)gx * 4, gx, gy, cbase);
    return hipGetLastError();
}

// Sweep shapes: queries per block (QG) x candidate tiles per wave (CPL).  Shape 0 serves a
// single query (the HBM-bound form); the others trade LDS broadcast traffic (less with more
// tiles per wave) against waves in flight.
static void shape_of(int shape, int64_t Q, int &qg, int &cpl) {
    if (Q == 1) {
        qg = 1;
        cpl = 4;
        return;
    }
    switch (shape) {
        case 2: qg = 8; cpl = 4; break;
        case 3: qg = 32; cpl = 2; break;
        case 4: qg = 16; cpl = 4; break;
        case 5: qg = 8; cpl = 2; break;
        default: qg = 16; cpl = 2; break;
    }
}

int sweep_query_group(int shape, int64_t Q) {
    int qg, cpl;
    shape_of(shape, Q, qg, cpl);
    return qg;
}

int64_t sweep_waves(int shape, int64_t N, int64_t Q) {
    int qg, cpl;
    shape_of(shape, Q, qg, cpl);
    const int64_t T = (N + 63) / 64;
    return (T + 4 * cpl - 1) / (4 * cpl) * 4;
}

template <int P, bool ROOT>
static hipError_t sweep_p(int qg, int cpl, const float4 *il, int64_t N, int n4, const float4 *Ue, const float4 *Le,
                          int ld4, int64_t Q, float *out, int64_t ldo, bool pad_inf, unsigned long long *wmin,
                          int64_t cbase, hipStream_t s) {
#define LBIMP_SWEEP(QG, CPL) \
    if (qg == QG && cpl == CPL) \
        return sweep_variant<P, QG, CPL, ROOT>(il, N, n4, Ue, Le, ld4, Q, out, ldo, pad_inf, wmin, cbase, s);
    LBIMP_SWEEP(1, 4)
    LBIMP_SWEEP(16, 2)
    LBIMP_SWEEP(8, 4)
    LBIMP_SWEEP(32, 2)
    LBIMP_SWEEP(16, 4)
    LBIMP_SWEEP(8, 2)
#undef LBIMP_SWEEP
    return hipErrorInvalidValue;
}

hipError_t launch_lbk_sweep(int p, int shape, const float4 *il, int64_t N, int n4, const float4 *Ue,
                            const float4 *Le, int ld4, int64_t Q, float *out, int64_t ldo, bool pad_inf, bool root,
                            unsigned long long *wmin, hipStream_t s, int64_t cbase) {
    if (N == 0 || Q == 0) return hipSuccess;
    int qg, cpl;
    shape_of(shape, Q, qg, cpl);
    // query envelopes are padded by the caller to a multiple of sweep_query_group(shape, Q)
    if (p == 1)
        return root ? sweep_p<1, true>(qg, cpl, il, N, n4, Ue, Le, ld4, Q, out, ldo, pad_inf, wmin, cbase, s)
                    : sweep_p<1, false>(qg, cpl, il, N, n4, Ue, Le, ld4, Q, out, ldo, pad_inf, wmin, cbase, s);
    if (p == 2)
        return root ? sweep_p<2, true>(qg, cpl, il, N, n4, Ue, Le, ld4, Q, out, ldo, pad_inf, wmin, cbase, s)
                    : sweep_p<2, false>(qg, cpl, il, N, n4, Ue, Le, ld4, Q, out, ldo, pad_inf, wmin, cbase, s);
    // p = infinity: LB_Keogh_inf is its own root form
    return sweep_p<kPInf, false>(qg, cpl, il, N, n4, Ue, Le, ld4, Q, out, ldo, pad_inf, wmin, cbase, s);
}

// ------------------------------------------------------------------ seed selection
// Threshold seeding: the paper's scan starts from b = inf and tightens b in database order;
// a parallel pass instead computes the DTW of the candidates with the smallest LB_Keogh first.
// Each thread keeps its 4 smallest (value, index) keys of a contiguous range of entries; of the
// 1024 keys of the block one wave then takes the S with the smallest values (a radix select on
// the value bits).  Approximate top-S is enough: any threshold that is the
// DTW of some candidate is a valid (never too small) best-so-far.
template <bool FROM_KEYS>
__global__ __launch_bounds__(256) void k_select_seeds(float *__restrict__ S1, int64_t ldS, int64_t cstart, int64_t N,
                                                       const unsigned long long *__restrict__ wmin, int64_t nw,
                                                       int S, int *__restrict__ seeds) {
    __shared__ unsigned long long keys[1024];
    const int64_t q = blockIdx.x;
    float *row = S1 + q * ldS;
    unsigned long long top[4] = {kNoKey, kNoKey, kNoKey, kNoKey};
    const int64_t count = FROM_KEYS ? nw : N - cstart;
    // Thread t takes a contiguous range of entries, so that keys of equal value sit in the block's
    // key list in the order of their entries (below); eight are loaded before the first is
    // inserted, so a pass waits for memory once per eight loads.
    constexpr int U = 8;
    const int64_t per = (count + 255) / 256;
    const int64_t e0 = threadIdx.x * per, e1 = e0 + per < count ? e0 + per : count;
    for (int64_t c0 = e0; c0 < e1; c0 += U) {
        unsigned long long kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = c0 + u;
            const int64_t cc = c < e1 ? c : e1 - 1;
            const unsigned long long k =
                FROM_KEYS ? wmin[q * nw + cc]
                          : ((unsigned long long)__float_as_uint(row[cstart + cc]) << 32) |
                                (unsigned long long)(cstart + cc);
            kk[u] = c < e1 ? k : kNoKey;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned long long k = kk[u];
            if (k < top[3]) {
                top[3] = k;
#pragma unroll
                for (int a = 3; a > 0; --a) {
                    if (top[a] < top[a - 1]) {
                        unsigned long long t = top[a];
                        top[a] = top[a - 1];
                        top[a - 1] = t;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) keys[threadIdx.x * 4 + a] = top[a];
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    unsigned long long kv[16];
    unsigned hv[16];  // the value half of each key (values are >= 0, so their bits order them)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        kv[j] = keys[j * 64 + lane];
        hv[j] = (unsigned)(kv[j] >> 32);
    }
    // T = the S-th smallest value: the largest T with fewer than S values below it, bit by bit
    unsigned T = 0;
    for (int b = 31; b >= 0; --b) {
        const unsigned cand = T | (1u << b);
        int below = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) below += __popcll(__ballot(hv[j] < cand));
        if (below < S) T = cand;
    }
    // every key below T, then keys at T in list order until there are S: each thread's keys are
    // sorted and cover a contiguous range of entries, so equal values go to the earlier entry
    // (the smaller candidate index for the minima of the pass-0 scans and for S1 rows); the 1024
    // keys hold at least S at or below T, so exactly S are written
    int nlt = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) nlt += __popcll(__ballot(hv[j] < T));
    const unsigned long long lower = (1ull << lane) - 1ull;
    int lt = 0, eq = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const unsigned long long mlt = __ballot(hv[j] < T), meq = __ballot(hv[j] == T);
        int r = -1;
        if (hv[j] < T) r = lt + __popcll(mlt & lower);
        else if (hv[j] == T) r = nlt + eq + __popcll(meq & lower);
        if (r >= 0 && r < S) {
            const int c = kv[j] == kNoKey ? -1 : (int)(kv[j] & 0xffffffffu);
            seeds[q * S + r] = c;
            if (c >= 0) row[c] = kInf;  // its DTW is computed by the seeding stage
        }
        lt += __popcll(mlt);
        eq += __popcll(meq);
    }
}

hipError_t launch_select_seeds(float *S1, int64_t ldS, int64_t N, int64_t Q, int S, const unsigned long long *wmin,
                               int64_t nw, int *seeds, hipStream_t s, int64_t c0) {
    if (Q == 0 || S == 0) return hipSuccess;
    if (wmin)
        hipLaunchKernelGGL(k_select_seeds<true>, dim3((unsigned)Q), dim3(256), 0, s, S1, ldS, c0, N, wmin, nw, S,
                           seeds);
    else
        hipLaunchKernelGGL(k_select_seeds<false>, dim3((unsigned)Q), dim3(256), 0, s, S1, ldS, c0, N, wmin, nw, S,
                           seeds);
    return hipGetLastError();
}

// ------------------------------------------------------------------ compaction
// Strict test of Algorithms 2 and 3 on the (value, index) key: a candidate whose bound key is
// not below the threshold key can at best tie, and a tie goes to the smaller index.
// Each wave covers 64*CH candidates: one ballot per chunk, one atomicAdd per block (per bucket
// of the block when the list is bucketed: cntb given, buckets of bs candidates counted from c0).
__global__ __launch_bounds__(256) void k_compact(const float *__restrict__ S1, int64_t ldS, int64_t c0, int64_t N,
                                                  const unsigned long long *__restrict__ thr, int *__restrict__ list,
                                                  int64_t ldl, int *__restrict__ cnt, int64_t bs, int *__restrict__ cntb,
                                                  int64_t cq) {
    constexpr int CH = 16;
    __shared__ int wtot[4];
    __shared__ int wbase[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = blockIdx.y;
    const int64_t base = c0 + ((int64_t)blockIdx.x * 4 + wave) * 64 * CH;
    const unsigned long long t = thr[q];
    const float *row = S1 + q * ldS;
    // All CH loads are issued before the first test (a load under `c < N` would be a branch of
    // its own, waited on before its ballot); positions past N read the last value and are
    // masked out after.
    float v[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int64_t c = base + ch * 64 + lane;
        v[ch] = row[c < N ? c : N - 1];
    }
    unsigned long long masks[CH];
    int total = 0;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int64_t c = base + ch * 64 + lane;
        const unsigned long long k = ((unsigned long long)__float_as_uint(v[ch]) << 32) | (unsigned long long)c;
        masks[ch] = __ballot(c < N && k < t);
        total += __popcll(masks[ch]);
    }
    if (lane == 0) wtot[wave] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!cntb) {
            const int sum = wtot[0] + wtot[1] + wtot[2] + wtot[3];
            int pos = sum ? atomicAdd(&cnt[q], sum) : 0;
            for (int wv = 0; wv < 4; ++wv) {
                wbase[wv] = pos;
                pos += wtot[wv];
            }
        } else {
            // consecutive waves of one bucket share an atomic; list positions start at k * bs
            const int64_t blk0 = c0 + (int64_t)blockIdx.x * 4 * 64 * CH;
            int tot = 0;
            for (int wv = 0; wv < 4;) {
                const int64_t k = (blk0 + (int64_t)wv * 64 * CH - c0) / bs;
                int sum = 0, w2 = wv;
                while (w2 < 4 && (blk0 + (int64_t)w2 * 64 * CH - c0) / bs == k) sum += wtot[w2++];
                int pos = sum ? atomicAdd(&cntb[k * cq + q], sum) : 0;
                pos += (int)(k * bs);
                for (; wv < w2; ++wv) {
                    wbase[wv] = pos;
                    pos += wtot[wv];
                }
                tot += sum;
            }
            if (tot) atomicAdd(&cnt[q], tot);
        }
    }
    __syncthreads();
    if (total == 0) return;
    int pos = wbase[wave];
    const unsigned long long below = (1ull << lane) - 1ull;
    int *out = list + q * ldl;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        if ((masks[ch] >> lane) & 1ull) out[pos + __popcll(masks[ch] & below)] = (int)(base + ch * 64 + lane);
        pos += __popcll(masks[ch]);
    }
}

hipError_t launch_compact(const float *S1, int64_t ldS, int64_t N, int64_t Q, const unsigned long long *thr,
                          int *list, int64_t ldl, int *cnt, hipStream_t s, int64_t c0, int64_t bs, int *cntb) {
    if (N <= c0 || Q == 0) return hipSuccess;
    if (cntb && (bs <= 0 || bs % (64 * 16) != 0)) return hipErrorInvalidValue;  // a bucket is whole waves
    int64_t per_block = 4 * 64 * 16;
    dim3 grid((unsigned)((N - c0 + per_block - 1) / per_block), (unsigned)Q);
    hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, S1, ldS, c0, N, thr, list, ldl, cnt, bs, cntb, Q);
    return hipGetLastError();
}

int64_t compact_wave_span() { return 64 * 16; }

// ------------------------------------------------------------------ work-item prefix
__global__ __launch_bounds__(1024) void k_items_prefix(const int *__restrict__ cnt, int64_t fixed, int64_t Q,
                                                        int batch, long long *__restrict__ prefix) {
    // Inclusive scan of each wave's 64 item counts by lane shifts, then each wave adds the
    // totals of the waves before it: two barriers per 1024 queries.
    __shared__ long long wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) prefix[0] = 0;
    long long carry = 0;  // items of the queries before this chunk (the same in every thread)
    for (int64_t q0 = 0; q0 < Q; q0 += 1024) {
        const int64_t q = q0 + threadIdx.x;
        long long v = 0;
        if (q < Q) {
            const long long c = cnt ? (long long)cnt[q] : (long long)fixed;
            v = (c + batch - 1) / batch;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long t = __shfl_up(v, off);
            if (lane >= off) v += t;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        long long before = carry, chunk = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const long long t = wsum[w];
            if (w < wave) before += t;
            chunk += t;
        }
        if (q < Q) prefix[q + 1] = before + v;
        carry += chunk;
        __syncthreads();  // wsum is rewritten by the next chunk
    }
}

hipError_t launch_items_prefix(const int *cnt, int64_t fixed, int64_t Q, int batch, long long *prefix,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_items_prefix, dim3(1), dim3(1024), 0, s, cnt, fixed, Q, batch, prefix);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fills (kernels, not memsets)
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t count) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < count) p[g] = v;
}
__global__ void k_fill_i32(int *p, int v, int64_t count) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < count) p[g] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

__global__ void k_iota_i32(int *p, int64_t count) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < count) p[g] = (int)g;
}

hipError_t launch_iota_i32(int *p, int64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int v, int64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

}  // namespace lbimp
