// Second pruning pass, LB_Improved (Sec. 8 of Lemire, arXiv:0811.3301), for bands too wide
// to keep a lane's envelope state in registers: one wave per (query, candidate) pair.
//
// For candidate x: x' = H(x, y) = med3(x, L, U) (the projection of Sec. 7), its envelope
// U'_i = max x'[i-w .. i+w], L'_i = min (windows cut to [0, n)), and the second term
// sum_i d(y_i, [L'_i, U'_i])^p.  Since L' <= U', d = max(0, y - U') + max(0, L' - y) with
// at most one term non-zero, so the max envelope and the min envelope are handled in two
// passes that each add their own half.
//
// Envelope by van Herk / Gil-Werman with blocks of K = 2w+1 positions starting at 0: with g
// the running max from the block start and h the running max to the block end,
// U'_i = max(h[i-w], g[i+w]) (h of a negative position is neutral; positions >= n hold the
// neutral value, which every window reaching past n-1 also holds n-1 against).  Lane l owns
// positions [l*M, l*M + M); K > M, so a lane meets at most one block start.  g and h are
// lane-local scans joined by one segmented scan across the lanes (the carry stops at a block
// start), then written to LDS, where output i reads h[i-w] and g[i+w].
#include "device_common.h"

namespace lbimp {

namespace {

// Inclusive segmented scan across the wave with op(a, b) = max or min.  Lane l holds (v, f):
// f set means the running value restarts at this lane.  Forward scans combine lane l-d into
// lane l; backward scans lane l+d into lane l.
template <bool MAX, bool FORWARD>
__device__ __forceinline__ float seg_scan(float v, bool f, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float ov = FORWARD ? __shfl_up(v, d) : __shfl_down(v, d);
        const int of = FORWARD ? __shfl_up((int)f, d) : __shfl_down((int)f, d);
        const bool in = FORWARD ? lane >= d : lane + d < 64;
        if (in && !f) v = MAX ? fmaxf(v, ov) : fminf(v, ov);
        if (in) f = f || of;
    }
    return v;
}

// A per-lane value the compiler must treat as unknown here: comparisons against it are then
// made where they are used instead of being kept as lane masks across the whole pass.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// One pass over the max (MAX) or min envelope of x' (xraw[M] per lane; positions >= n take
// the neutral value); returns this lane's share of sum_i max(0, y_i - U'_i)^p (MAX) or
// max(0, L'_i - y_i)^p.  g and h live in LDS transposed: position l*M + j at j*64 + l, so
// the writes of a step and the reads of a step (lane l reads position l*M + j +- w, at lane
// l + q and slot r with q, r the same for every lane) touch 64 consecutive words.
template <int P, int M, bool MAX>
__device__ __forceinline__ float lbi_pass(const float (&xraw)[M], const float (&yv)[M], float *sg, float *sh,
                                          int w_in, int n, int lane, int rj_in) {
    constexpr float kNeutral = MAX ? -kInf : kInf;
    auto op = [](float a, float b) { return MAX ? fmaxf(a, b) : fminf(a, b); };
    const int p0 = lane * M;
    float xp[M];
    {
        const int valid = opaque(n - p0);
#pragma unroll
        for (int j = 0; j < M; ++j) xp[j] = j < valid ? xraw[j] : kNeutral;
    }
    int rj = opaque(rj_in);
    // lane summaries: before the block start (or the whole lane), and from it to the lane end
    float before = kNeutral, after = kNeutral;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const float v = xp[j];
        const bool b = j < rj;
        before = op(before, b ? v : kNeutral);
        after = op(after, b ? kNeutral : v);
    }
    const bool has_reset = rj < M;
    // forward carry: value entering this lane from the block that was open at its start
    const float fwd_out = seg_scan<MAX, true>(has_reset ? after : before, has_reset, lane);
    float cin = __shfl_up(fwd_out, 1);
    if (lane == 0) cin = kNeutral;
    // backward carry: value entering this lane's end from the lanes after it
    const float bwd_out = seg_scan<MAX, false>(before, has_reset, lane);
    float cback = __shfl_down(bwd_out, 1);
    if (lane == 63) cback = kNeutral;
    // g: running value from the block start (carry before the reset), written forward
    rj = opaque(rj);
    float run = cin;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        run = (j == rj) ? xp[j] : op(run, xp[j]);
        sg[j * 64 + lane] = run;
    }
    // h: running value to the block end (carry after the reset), written backward
    rj = opaque(rj);
    run = cback;
#pragma unroll
    for (int j = M - 1; j >= 0; --j) {
        run = op(run, xp[j]);
        sh[j * 64 + lane] = run;
        run = (j == rj) ? kNeutral : run;  // positions before the block start end their block here
    }
    __syncthreads();
    float acc = 0.f;
    // output i = p0 + j reads g at i + w and h at i - w; with w = qg*M + rg, position i + w
    // sits at lane + qg (+1 once rg + j reaches M) and slot (rg + j) mod M, and likewise for -w
    const int w = __builtin_amdgcn_readfirstlane(w_in);
    int rg = w % M, qg = w / M;
    int rh = (M - rg) % M, qh = -qg - (rg ? 1 : 0);
    const int hfrom = opaque(w - p0);  // h[i - w] exists for j >= w - p0
    const int valid = opaque(n - p0);  // outputs exist for j < n - p0
    const int top = M * 64 - 1;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const int ag = min(rg * 64 + qg + lane, top);
        const int ah = max(rh * 64 + qh + lane, 0);
        const float e = op(j >= hfrom ? sh[ah] : kNeutral, sg[ag]);
        float d = MAX ? fmaxf(yv[j] - e, 0.f) : fmaxf(e - yv[j], 0.f);
        d = j < valid ? d : 0.f;
        acc = pacc<P>(acc, d);
        if (++rg == M) rg = 0, ++qg;
        if (++rh == M) rh = 0, ++qh;
    }
    __syncthreads();  // the next pass overwrites sg and sh
    return acc;
}

}  // namespace

template <int P, int M>
__global__ __launch_bounds__(64) void k_lbi_wave(LbiArgs a, int w) {
    extern __shared__ float sm[];
    float *sg = sm, *sh = sm + 64 * M;  // [M][64] each
    // This lane's slice of the query envelope, [M][64] each: kept in LDS rather than registers
    // (each lane reads only its own column), which leaves room for a second wave per SIMD.
    float *sUq = sm + 2 * 64 * M, *sLq = sm + 3 * 64 * M;
    const int lane = threadIdx.x;
    const int n = a.n;
    const int K = 2 * w + 1;
    const int p0 = lane * M;
    const int rj = min(M, (p0 + K - 1) / K * K - p0);  // offset of the block start in this lane (M: none)
    int64_t cur_q = -1;
    float yv[M];
    int64_t q;
    long long b;
    ItemCursor items(a.pl, a.prefix, a.Q, 64);
    while (items.get(q, b)) {
        if (q != cur_q) {  // this lane's slice of the query envelope and series
            const float *Uq = a.qd.U + q * a.qd.ldq, *Lq = a.qd.L + q * a.qd.ldq, *yq = a.qd.Y + q * a.qd.ldy;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int i = min(p0 + j, n - 1);
                sUq[j * 64 + lane] = Uq[i];
                sLq[j * 64 + lane] = Lq[i];
                yv[j] = yq[i];
            }
            cur_q = q;
        }
        const long long j0 = b * 64;
        const int cnt = (int)min(64ll, (long long)pair_count(a.pl, q, items.bk) - j0);
        const int c_mine = lane < cnt ? pair_cand(a.pl, q, j0 + lane, items.bk) : 0;
        const float s1_mine = lane < cnt ? a.S1[q * a.ldS + c_mine] : 0.f;
        const bool abandon = a.abandon && a.thr && !a.out_root;
        const u64 tq = a.thr ? a.thr[q] : kNoKey;
        float s2_mine = 0.f;
        // rows are loaded one pair ahead of their use
        float xr[M];
        auto load_row = [&](int t) {
            const int c = __shfl(c_mine, t);
            const float *x = a.rows + (int64_t)c * n;
#pragma unroll
            for (int j = 0; j < M; ++j) xr[j] = x[min(p0 + j, n - 1)];
        };
        load_row(0);
        for (int t = 0; t < cnt; ++t) {
            float xp[M];
#pragma unroll
            for (int j = 0; j < M; ++j)
                xp[j] = __builtin_amdgcn_fmed3f(xr[j], sLq[j * 64 + lane], sUq[j * 64 + lane]);
            if (t + 1 < cnt) load_row(t + 1);
            float acc = lbi_pass<P, M, true>(xp, yv, sg, sh, w, n, lane, rj);
            if (abandon) {
                // early abandoning: the distances of y above the envelope of x' alone may already
                // take the bound of pair t to its threshold; the pass below it is then skipped
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) acc = pjoin<P>(acc, __shfl_xor(acc, off));
                const int ct = __shfl(c_mine, t);
                const float s1t = __shfl(s1_mine, t);
                if (make_key(pjoin<P>(s1t, acc), ct) >= tq) {
                    if (lane == t) s2_mine = acc;
                    continue;
                }
                acc = lane == 0 ? acc : (P == kPInf ? acc : 0.f);  // the sum so far, carried by lane 0
            }
            acc = pjoin<P>(acc, lbi_pass<P, M, false>(xp, yv, sg, sh, w, n, lane, rj));
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc = pjoin<P>(acc, __shfl_xor(acc, off));
            if (lane == t) s2_mine = acc;
        }
        const bool active = lane < cnt;
        const float s2 = pjoin<P>(s1_mine, s2_mine);
        if (a.out_root && active) a.out_root[c_mine] = root_p<P>(s2);
        if (a.thr) {
            const bool keep = active && make_key(s2, c_mine) < a.thr[q];
            const u64 m = __ballot(keep);
            if (m) {
                int pos = 0;
                if (lane == 0) pos = atomicAdd(&a.cnt2[q], __popcll(m));
                pos = __shfl(pos, 0);
                if (keep) a.list2[q * a.ldl2 + pos + __popcll(m & ((1ull << lane) - 1ull))] = c_mine;
            }
        }
    }
}

// Positions per lane for a band: the smallest supported M with 64 M >= n + w.
static int lbi_wave_m(int n, int w) {
    const int need = (n + w + 63) / 64;
    for (int m : {4, 8, 12, 16, 20, 24, 28, 32})
        if (m >= need) return m;
    return 0;
}

bool lbi_wave_supported(int n, int w) {
    const int m = lbi_wave_m(n, w);
    return m > 0 && 2 * w + 1 > m;
}

template <int P, int M>
static void lbi_wave_launch(int w, int num_cu, const LbiArgs &a, hipStream_t s) {
    const size_t lds = sizeof(float) * 4 * 64 * (size_t)M;
    hipLaunchKernelGGL((k_lbi_wave<P, M>), dim3(persistent_grid(k_lbi_wave<P, M>, lds, num_cu)), dim3(64), lds, s, a,
                       w);
}

template <int P>
static hipError_t lbi_wave_dispatch(int m, int w, int num_cu, const LbiArgs &a, hipStream_t s) {
    switch (m) {
        case 4: lbi_wave_launch<P, 4>(w, num_cu, a, s); break;
        case 8: lbi_wave_launch<P, 8>(w, num_cu, a, s); break;
        case 12: lbi_wave_launch<P, 12>(w, num_cu, a, s); break;
        case 16: lbi_wave_launch<P, 16>(w, num_cu, a, s); break;
        case 20: lbi_wave_launch<P, 20>(w, num_cu, a, s); break;
        case 24: lbi_wave_launch<P, 24>(w, num_cu, a, s); break;
        case 28: lbi_wave_launch<P, 28>(w, num_cu, a, s); break;
        case 32: lbi_wave_launch<P, 32>(w, num_cu, a, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lbi_wave(int p, int w, int num_cu, const LbiArgs &a, hipStream_t s) {
    if (!lbi_wave_supported(a.n, w)) return hipErrorInvalidValue;
    const int m = lbi_wave_m(a.n, w);
    if (p == 1) return lbi_wave_dispatch<1>(m, w, num_cu, a, s);
    if (p == 2) return lbi_wave_dispatch<2>(m, w, num_cu, a, s);
    return lbi_wave_dispatch<kPInf>(m, w, num_cu, a, s);
}

}  // namespace lbimp
