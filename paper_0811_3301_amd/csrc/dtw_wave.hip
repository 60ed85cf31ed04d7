// Banded DTW_p (Sec. 4 of Lemire, arXiv:0811.3301) with a group of lanes per pair: the band
// is swept along anti-diagonals held in registers, neighbours exchanged by DPP lane shifts.
// One pair costs about n dependent steps instead of n(2w+1), which is what a latency-bound
// stage (the seeding DTWs, a few per query) needs.
#include "device_common.h"

namespace lbimp {

// Cells (i, j) with |j - i| <= w.  Anti-diagonal d = i + j, band position u = j - i + w in
// [0, 2w].  Lane l of a group holds positions u = 2l (even) and 2l + 1 (odd); step t computes
// the even cell on diagonal de = 2t - (w & 1) and the odd cell on do = de + 1 (a position's
// parity fixes the parity of its diagonals).  The recursion, in prefix form:
//   even (de, 2l):   left (de-1, 2l-1) = odd of lane l-1, previous step (shift right)
//                    up   (de-1, 2l+1) = own odd, previous step
//                    diag (de-2, 2l)   = own even, previous step
//   odd  (do, 2l+1): left (do-1, 2l)   = own even, this step
//                    up   (do-1, 2l+2) = even of lane l+1, this step (shift left)
//                    diag (do-2, 2l+1) = own odd, previous step
// Both cells of a lane share i = (de - 2l + w) / 2; j = de - i and j + 1.  The pair's row x is
// staged in LDS padded with +inf and the query with -inf, so any cell outside the matrix costs
// +inf (x - y is +inf whichever side is out of range).  Lanes outside the band (2l > 2w for
// the even cell, 2l + 1 > 2w for the odd one) are forced to +inf, which also keeps groups of
// one wave from leaking into each other through the shifts.  The virtual cell (-1,-1) = 0 sits
// on diagonal -2 at u = w: the even slot of lane w/2 (w even) or the odd slot of lane
// (w-1)/2 (w odd), as the state of step -1.  The result D(n-1, n-1) is read from the same slot
// after step n-1.  Early abandoning: a path visits one of any two consecutive anti-diagonals,
// so min over both cells of all lanes bounds the result.
constexpr int kWavePad = 96;  // LDS padding of x and y on each side: |i - t|, |j - t| <= 64, +9 read ahead

// Lane shifts across the wave.  The lane without a source (lane 0 shifting right, lane 63
// shifting left) keeps `keep`: the callers pass the shift's previous result, whose value in that
// lane is the +inf it was set to before the first step, so no step spends an instruction
// refilling it.
__device__ __forceinline__ float dpp_shr1(float keep, float v) {  // lane l gets lane l-1
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(keep), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_shl1(float keep, float v) {  // lane l gets lane l+1
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(keep), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

template <int P>
__device__ __forceinline__ float cost_add(float d, float m) {
    return pacc<P>(m, d);
}

template <int P>
__global__ __launch_bounds__(64) void k_dtw_wavereg(DtwArgs a, int w, int LP) {
    extern __shared__ float sm[];
    const int n = a.n;
    const int span = n + 2 * kWavePad;
    float *ys = sm;                 // [span], ys[j + pad] = y[j], -inf outside
    float *xs = sm + span;          // [G][span], xs[g][i + pad] = x_g[i], +inf outside
    __shared__ int cand[64];
    const int lane = threadIdx.x;
    const int G = 64 / LP;
    const int g = lane / LP, l = lane % LP;
    float *xg = xs + g * span;
    const bool e_ok = 2 * l <= 2 * w;
    const bool o_ok = 2 * l + 1 <= 2 * w;
    const int slot_lane = w >> 1;   // lane (within the group) holding the start and end cells
    const bool slot_odd = (w & 1) != 0;
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(a.pl, a.prefix, a.Q, G);
    while (items.get(q, b)) {
        const long long jj = b * G + g;
        const int cl = jj < pair_count(a.pl, q, items.bk) ? pair_cand(a.pl, q, jj, items.bk) : -1;
        const bool active0 = cl >= 0;
        const int c = active0 ? cl : 0;
        __syncthreads();
        if (l == 0) cand[g] = cl;
        __syncthreads();
        if (q != cur_q) {
            const float *y = a.qd.Y + q * a.qd.ldy;
            stage_lds(ys, span, [&](int t) {
                const int j = t - kWavePad;
                return (j >= 0 && j < n) ? y[j] : -kInf;
            });
            cur_q = q;
        }
        // stage every group's row (+inf padded); all groups in one pass
        stage_lds(xs, G * span, [&](int t) {
            const int gg = t / span;
            const int i = t - gg * span - kWavePad;
            const int cg = cand[gg];
            return (cg >= 0 && i >= 0 && i < n) ? a.rows[(int64_t)cg * n + i] : kInf;
        });
        __syncthreads();
        const u64 *tq = a.tkeys + q;
        float E = kInf, O = kInf;  // state of step -1
        if (l == slot_lane) {
            if (slot_odd)
                O = 0.f;
            else
                E = 0.f;
        }
        // step t reads x[i] and y[j], y[j+1] with i = t + (w - (w&1))/2 - l, j = de - i
        const int i0 = (w - (w & 1)) / 2 - l;
        const int j0 = -(w & 1) - i0;
        const float *xp = xg + kWavePad + i0;
        const float *yp = ys + kWavePad + j0;
        bool alive = active0;
        float left = kInf, up = kInf;  // the shifted neighbours; +inf in lanes 0 and 63 throughout
        auto step = [&](float xi, float yj, float yj1) {
            left = dpp_shr1(left, O);
            float Ee = cost_add<P>(xi - yj, __builtin_fminf(__builtin_fminf(left, O), E));
            Ee = e_ok ? Ee : kInf;
            up = dpp_shl1(up, Ee);
            float Oo = cost_add<P>(xi - yj1, __builtin_fminf(__builtin_fminf(Ee, up), O));
            O = o_ok ? Oo : kInf;
            E = Ee;
        };
        // blocks of 8 steps: the 8 x and 9 y values of a block are read from LDS up front
        int t0 = 0;
        for (; t0 + 8 <= n; t0 += 8) {
            float xv[8], yv[9];
#pragma unroll
            for (int u = 0; u < 8; ++u) xv[u] = xp[t0 + u];
#pragma unroll
            for (int u = 0; u < 9; ++u) yv[u] = yp[t0 + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) step(xv[u], yv[u], yv[u + 1]);
            if (a.abandon) {
                float m = fminf(E, O);
                for (int off = LP >> 1; off > 0; off >>= 1) m = fminf(m, __shfl_xor(m, off));
                const u64 th = __hip_atomic_load(tq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (alive && make_key(m, c) >= th) alive = false;
                if (!__any(alive)) break;
            }
        }
        if (t0 + 8 > n)
            for (int t = t0; t < n; ++t) step(xp[t], yp[t], yp[t + 1]);
        const float dfin = slot_odd ? O : E;
        const bool owner = l == slot_lane;
        publish<P>(owner && alive, dfin, c, q, a.best, a.thr, a.res, a.ldres, a.rescnt, a.out_root);
        if (a.abandoned && owner && active0 && !alive) atomicAdd(&a.abandoned[q], 1);
    }
}

// Wide bands (63 < w < 64R): one pair per wave, lane l holding the R position pairs
// (2m, 2m+1) for m = lR + r, r < R.  The recursion is the one above with the neighbours
// inside a lane read directly: the even cell of position r takes its left value from the odd
// cell of r-1 (previous step), and only r = 0 takes it from lane l-1 (DPP shift right); the
// odd cell of r takes its up value from the even cell of r+1 (this step), and only r = R-1
// from lane l+1 (shift left).  Cell (r) of lane l sits at i = t + (w - (w&1))/2 - (lR + r):
// over a block of 8 steps a lane reads a window of R+7 x values and R+8 y values from LDS.
template <int P, int R>
__global__ __launch_bounds__(64) void k_dtw_wavereg_r(DtwArgs a, int w) {
    extern __shared__ float sm[];
    constexpr int pad = 64 * R + 32;
    const int n = a.n;
    const int span = n + 2 * pad;
    float *ys = sm;         // [span], ys[j + pad] = y[j], -inf outside
    float *xs = sm + span;  // [span], xs[i + pad] = x[i], +inf outside
    const int lane = threadIdx.x;
    const int mv = w >> 1;  // position pair holding the start and end cells
    const bool slot_odd = (w & 1) != 0;
    const int ibase = (w - (w & 1)) / 2;
    // x of (lane, r, step t) is x[ibase - (lane*R + r) + t]; y is y[-(w&1) - ibase + lane*R + r + t (+1)]
    const int xb = pad + ibase - (lane * R + R - 1);
    const int yb = pad - (w & 1) - ibase + lane * R;
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(a.pl, a.prefix, a.Q, 1);
    while (items.get(q, b)) {
        if (b >= pair_count(a.pl, q, items.bk)) continue;
        const int c = pair_cand(a.pl, q, b, items.bk);
        __syncthreads();
        if (q != cur_q) {
            const float *y = a.qd.Y + q * a.qd.ldy;
            stage_lds(ys, span, [&](int t) {
                const int j = t - pad;
                return (j >= 0 && j < n) ? y[j] : -kInf;
            });
            cur_q = q;
        }
        const float *xrow = a.rows + (int64_t)c * n;
        stage_lds(xs, span, [&](int t) {
            const int i = t - pad;
            return (i >= 0 && i < n) ? xrow[i] : kInf;
        });
        __syncthreads();
        const u64 *tq = a.tkeys + q;
        float E[R], O[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool here = lane * R + r == mv;
            E[r] = (here && !slot_odd) ? 0.f : kInf;  // state of step -1: D(-1,-1) = 0 on diagonal -2
            O[r] = (here && slot_odd) ? 0.f : kInf;
        }
        bool alive = true;
        float left0 = kInf, upl = kInf;  // the shifted neighbours; +inf in lanes 0 and 63 throughout
        // steps t0..t0+nb-1 from windows xw[k] = xs[xb + t0 + k], yw[k] = ys[yb + t0 + k]
        auto block = [&](int t0, int nb) {
            float xw[R + 7], yw[R + 8];
#pragma unroll
            for (int k = 0; k < R + 7; ++k) xw[k] = xs[xb + t0 + k];
#pragma unroll
            for (int k = 0; k < R + 8; ++k) yw[k] = ys[yb + t0 + k];
#pragma unroll
            for (int st = 0; st < 8; ++st) {
                if (st < nb) {
                    left0 = dpp_shr1(left0, O[R - 1]);
#pragma unroll
                    for (int r = R - 1; r >= 0; --r) {  // descending: O[r-1] still holds the previous step
                        const float left = (r == 0) ? left0 : O[r - 1];
                        const float m = __builtin_fminf(__builtin_fminf(left, O[r]), E[r]);
                        const float v = cost_add<P>(xw[R - 1 - r + st] - yw[r + st], m);
                        E[r] = 2 * (lane * R + r) <= 2 * w ? v : kInf;
                    }
                    upl = dpp_shl1(upl, E[0]);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float up = (r + 1 < R) ? E[r + 1] : upl;
                        const float m = __builtin_fminf(__builtin_fminf(E[r], up), O[r]);
                        const float v = cost_add<P>(xw[R - 1 - r + st] - yw[r + st + 1], m);
                        O[r] = 2 * (lane * R + r) + 1 <= 2 * w ? v : kInf;
                    }
                }
            }
        };
        int t0 = 0;
        for (; t0 + 8 <= n; t0 += 8) {
            block(t0, 8);
            if (a.abandon) {
                float m = kInf;
#pragma unroll
                for (int r = 0; r < R; ++r) m = fminf(m, fminf(E[r], O[r]));
                for (int off = 32; off > 0; off >>= 1) m = fminf(m, __shfl_xor(m, off));
                const u64 th = __hip_atomic_load(tq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (make_key(m, c) >= th) {
                    alive = false;
                    break;
                }
            }
        }
        if (alive && t0 < n) block(t0, n - t0);
        float dfin = kInf;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (lane * R + r == mv) dfin = slot_odd ? O[r] : E[r];
        const bool owner = lane == mv / R;
        publish<P>(owner && alive, dfin, c, q, a.best, a.thr, a.res, a.ldres, a.rescnt, a.out_root);
        if (a.abandoned && owner && !alive) atomicAdd(&a.abandoned[q], 1);
    }
}

// Position pairs per lane for a wide band (0: not supported, use the LDS kernel).
static int wave_r(int w) {
    for (int r : {2, 4, 8})
        if (w < 64 * r) return r;
    return 0;
}

bool dtw_wavereg_wide_supported(int n, int w) {
    const int r = wave_r(w);
    return r > 0 && sizeof(float) * 2 * (size_t)(n + 2 * (64 * r + 32)) <= kLdsBudget;
}

hipError_t launch_dtw_wavereg_wide(int p, int w, int num_cu, const DtwArgs &a, hipStream_t s) {
    if (w <= kLaneMaxW || !dtw_wavereg_wide_supported(a.n, w)) return hipErrorInvalidValue;
    const int r = wave_r(w);
    const size_t lds = sizeof(float) * 2 * (size_t)(a.n + 2 * (64 * r + 32));
#define LBIMP_WAVE_R(PP, RR)                                                                                    \
    hipLaunchKernelGGL((k_dtw_wavereg_r<PP, RR>), dim3(persistent_grid(k_dtw_wavereg_r<PP, RR>, lds, num_cu)), \
                       dim3(64), lds, s, a, w)
    if (p == 1) {
        if (r == 2) LBIMP_WAVE_R(1, 2);
        else if (r == 4) LBIMP_WAVE_R(1, 4);
        else LBIMP_WAVE_R(1, 8);
    } else if (p == 2) {
        if (r == 2) LBIMP_WAVE_R(2, 2);
        else if (r == 4) LBIMP_WAVE_R(2, 4);
        else LBIMP_WAVE_R(2, 8);
    } else {
        if (r == 2) LBIMP_WAVE_R(kPInf, 2);
        else if (r == 4) LBIMP_WAVE_R(kPInf, 4);
        else LBIMP_WAVE_R(kPInf, 8);
    }
#undef LBIMP_WAVE_R
    return hipGetLastError();
}

// Lanes per pair: the smallest power of two above w, widened until the staged rows fit in LDS.
static int wave_lanes(int n, int w) {
    int lp = 1;
    while (lp < w + 1) lp <<= 1;
    while (lp < 64 && sizeof(float) * (size_t)(n + 2 * kWavePad) * (1 + 64 / lp) > kLdsBudget) lp <<= 1;
    return lp;
}

int dtw_wave_batch(int n, int w) { return 64 / wave_lanes(n, w); }

hipError_t launch_dtw_wavereg(int p, int w, int num_cu, const DtwArgs &a, hipStream_t s) {
    if (w > kLaneMaxW) return hipErrorInvalidValue;
    const int LP = wave_lanes(a.n, w);
    const size_t lds = sizeof(float) * (size_t)(a.n + 2 * kWavePad) * (1 + 64 / LP);
    if (lds > kLdsBudget) return hipErrorInvalidValue;
#define LBIMP_WAVEREG(PP) \
    hipLaunchKernelGGL(k_dtw_wavereg<PP>, dim3(persistent_grid(k_dtw_wavereg<PP>, lds, num_cu)), dim3(64), lds, s, a, w, LP)
    if (p == 1)
        LBIMP_WAVEREG(1);
    else if (p == 2)
        LBIMP_WAVEREG(2);
    else
        LBIMP_WAVEREG(kPInf);
#undef LBIMP_WAVEREG
    return hipGetLastError();
}

}  // namespace lbimp
