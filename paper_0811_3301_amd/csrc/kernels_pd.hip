// Pass 0 of the search: the piecewise-sum lower bound of Sec. 9 (Lemire, arXiv:0811.3301), and
// LB_Keogh (Sec. 7) of the candidates that pass it, read row by row instead of swept.
//
// Every series is summarised by its sums over the d = 8 parts of the cover the paper chose
// (width floor(n/8), the last part taking the rest).  The distance of a candidate's sums to the
// box spanned by the sums of the query envelope bounds LB_Keogh_1 from below (a sum over a part
// of clamped differences is at most the sum of their absolute values); for p = 2 a part's
// distance squared is divided by its size, and for p = infinity the largest distance per element
// of a part is taken (power-mean inequality).  The scan reads 64 bytes per candidate (8 fp64
// sums) instead of the 4n bytes of the row.  Sums are formed in fp64, each part in index order,
// for the rows and the envelopes alike: rounding is monotone, so a candidate inside the
// envelope on a whole part keeps a zero distance there, and the bound is rounded down to fp32.
#include "device_common.h"

namespace lbimp {

// Part j of the cover covers [j*m, (j+1)*m) for j < 7 and [7*m, n) for the last, m = n / 8.
__device__ __forceinline__ void pd_part(int n, int j, int &a, int &b) {
    const int m = n / kPdParts;
    a = j * m;
    b = j + 1 < kPdParts ? (j + 1) * m : n;
}

// pd[c][j] = sum of row c over part j, one thread per (row, part).
__global__ __launch_bounds__(256) void k_pd_rows(const float *__restrict__ rows, int64_t N, int n,
                                                  double *__restrict__ pd) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N * kPdParts) return;
    const int64_t c = g / kPdParts;
    const int j = (int)(g - c * kPdParts);
    int a, b;
    pd_part(n, j, a, b);
    const float *x = rows + c * (int64_t)n;
    double s = 0.0;
    for (int i = a; i < b; ++i) s += (double)x[i];
    pd[g] = s;
}

hipError_t launch_pd_rows(const float *rows, int64_t N, int n, double *pd, hipStream_t s) {
    const int64_t total = N * kPdParts;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pd_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rows, N, n, pd);
    return hipGetLastError();
}

// qpd[q][0][j] = sum of U over part j, qpd[q][1][j] = sum of L (the envelopes of stride ldq).
__global__ __launch_bounds__(64) void k_pd_query(const float *__restrict__ U, const float *__restrict__ L, int ldq,
                                                  int64_t Q, int n, double *__restrict__ qpd) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Q * 2 * kPdParts) return;
    const int64_t q = g / (2 * kPdParts);
    const int r = (int)(g - q * 2 * kPdParts);
    const int side = r / kPdParts, j = r % kPdParts;
    int a, b;
    pd_part(n, j, a, b);
    const float *e = (side == 0 ? U : L) + q * (int64_t)ldq;
    double s = 0.0;
    for (int i = a; i < b; ++i) s += (double)e[i];
    qpd[g] = s;
}

hipError_t launch_pd_query(const float *U, const float *L, int ldq, int64_t Q, int n, double *qpd, hipStream_t s) {
    const int64_t total = Q * 2 * kPdParts;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pd_query, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, U, L, ldq, Q, n, qpd);
    return hipGetLastError();
}

// Bound of one candidate against one query, pow domain, fp64.
template <int P>
__device__ __forceinline__ double pd_bound(const double (&x)[kPdParts], const double *qu, const double *ql,
                                           const double (&inv)[kPdParts]) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < kPdParts; ++j) {
        const double d = fmax(fmax(x[j] - qu[j], ql[j] - x[j]), 0.0);
        if constexpr (P == 1)
            acc += d;
        else if constexpr (P == 2)
            acc += d * d * inv[j];
        else
            acc = fmax(acc, d * inv[j]);
    }
    return acc;
}

// Lane = candidate, block = 4 waves of 64 candidates x up to QG queries (blockIdx.y).  Writes
// out[q][c] (pow domain, or root form with ROOT), +inf for padding columns c in [N, ldo) when
// pad_inf, and, per query and wave, the smallest (bound, index) key of the wave's candidates.
template <int P, int QG, bool ROOT>
__global__ __launch_bounds__(256) void k_pd_scan(const double *__restrict__ pd, int64_t N, int n,
                                                  const double *__restrict__ qpd, int64_t Q, float *__restrict__ out,
                                                  int64_t ldo, bool pad_inf, unsigned long long *__restrict__ wmin,
                                                  int64_t ldw, int64_t cbase) {
    __shared__ double sq[QG][2 * kPdParts];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.y * QG;
    for (int t = threadIdx.x; t < QG * 2 * kPdParts; t += 256) {
        const int64_t q = q0 + t / (2 * kPdParts);
        sq[t / (2 * kPdParts)][t % (2 * kPdParts)] = q < Q ? qpd[q * 2 * kPdParts + t % (2 * kPdParts)] : 0.0;
    }
    const int64_t c = ((int64_t)blockIdx.x * 4 + wave) * 64 + lane;
    const bool valid = c < N;
    double x[kPdParts];
    const double4 *src = reinterpret_cast<const double4 *>(pd + (valid ? c : 0) * kPdParts);
    const double4 v0 = src[0], v1 = src[1];
    x[0] = v0.x, x[1] = v0.y, x[2] = v0.z, x[3] = v0.w;
    x[4] = v1.x, x[5] = v1.y, x[6] = v1.z, x[7] = v1.w;
    double inv[kPdParts];
#pragma unroll
    for (int j = 0; j < kPdParts; ++j) {
        int a, b;
        pd_part(n, j, a, b);
        inv[j] = b > a ? 1.0 / (double)(b - a) : 0.0;  // an empty part has zero distance
    }
    __syncthreads();
#pragma unroll 4
    for (int qq = 0; qq < QG; ++qq) {
        const int64_t q = q0 + qq;
        if (q >= Q) break;
        const double b = pd_bound<P>(x, sq[qq], sq[qq] + kPdParts, inv);
        float f = __double2float_rd(b);
        if (ROOT && P == 2) f = __double2float_rd(sqrt(b));
        if (valid)
            out[q * ldo + c] = f;
        else if (pad_inf && c < ldo)
            out[q * ldo + c] = kInf;
        if (wmin) {
            unsigned long long k = valid ? make_key(f, (int)(c + cbase)) : kNoKey;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned hi = __shfl_xor((unsigned)(k >> 32), off);
                const unsigned lo = __shfl_xor((unsigned)k, off);
                const unsigned long long o = ((unsigned long long)hi << 32) | lo;
                k = o < k ? o : k;
            }
            if (lane == 0) wmin[q * ldw + (int64_t)blockIdx.x * 4 + wave] = k;
        }
    }
}

int64_t pd_scan_waves(int64_t N) { return (N + 255) / 256 * 4; }

template <int P, bool ROOT>
static void pd_scan_launch(const double *pd, int64_t N, int n, const double *qpd, int64_t Q, float *out, int64_t ldo,
                           bool pad_inf, unsigned long long *wmin, int64_t cbase, hipStream_t s) {
    constexpr int QG = 16;
    const dim3 grid((unsigned)((N + 255) / 256), (unsigned)((Q + QG - 1) / QG));
    hipLaunchKernelGGL((k_pd_scan<P, QG, ROOT>), grid, dim3(256), 0, s, pd, N, n, qpd, Q, out, ldo, pad_inf, wmin,
                       pd_scan_waves(N), cbase);
}

hipError_t launch_pd_scan(int p, const double *pd, int64_t N, int n, const double *qpd, int64_t Q, float *out,
                          int64_t ldo, bool pad_inf, bool root, unsigned long long *wmin, hipStream_t s, int64_t cbase) {
    if (N == 0 || Q == 0) return hipSuccess;
    if (p == 1)
        pd_scan_launch<1, false>(pd, N, n, qpd, Q, out, ldo, pad_inf, wmin, cbase, s);
    else if (p == 2)
        root ? pd_scan_launch<2, true>(pd, N, n, qpd, Q, out, ldo, pad_inf, wmin, cbase, s)
             : pd_scan_launch<2, false>(pd, N, n, qpd, Q, out, ldo, pad_inf, wmin, cbase, s);
    else
        pd_scan_launch<kPInf, false>(pd, N, n, qpd, Q, out, ldo, pad_inf, wmin, cbase, s);
    return hipGetLastError();
}

// ------------------------------------------------------------------ LB_Keogh of the survivors
// One wave per item of G = 8 pairs of one query (the pass-0 survivors of list0).  The lanes walk
// a candidate's row together, 64 consecutive elements per load, with the query envelope in
// LDS; the G rows' loads of one 64-element chunk are issued before any is used.  The G per-lane
// sums are combined across the wave by a transposing butterfly -- at each of the steps 32, 16, 8
// a lane keeps half of its values and adds its partner's copies of them, so after three steps
// lane l holds pair l/8 summed over 8 lanes -- then three plain steps finish the sums: 10 lane
// exchanges instead of 6 per pair.  S1[q][c] receives LB_Keogh^p (the compaction that follows
// reads it, as do LB_Improved and the DTW).
constexpr int kGatherPairs = 8;

template <int P>
__global__ __launch_bounds__(64) void k_lbk_gather(const float *__restrict__ rows, int n, QueryData qd, PairList pl,
                                                    const long long *__restrict__ prefix, int64_t Q,
                                                    float *__restrict__ S1, int64_t ldS) {
    extern __shared__ float sm[];
    float *sU = sm, *sL = sm + n;
    const int lane = threadIdx.x;
    int64_t cur_q = -1;
    int64_t q;
    long long b;
    ItemCursor items(pl, prefix, Q, kGatherPairs);
    while (items.get(q, b)) {
        if (q != cur_q) {
            __syncthreads();
            stage_lds(sU, n, [&](int i) { return qd.U[q * qd.ldq + i]; });
            stage_lds(sL, n, [&](int i) { return qd.L[q * qd.ldq + i]; });
            __syncthreads();
            cur_q = q;
        }
        const int count = pair_count(pl, q, items.bk);
        int c[kGatherPairs];
        const float *x[kGatherPairs];
#pragma unroll
        for (int g = 0; g < kGatherPairs; ++g) {
            const long long j = b * kGatherPairs + g;
            c[g] = j < count ? pair_cand(pl, q, j, items.bk) : -1;
            x[g] = rows + (int64_t)(c[g] < 0 ? 0 : c[g]) * n;
        }
        float acc[kGatherPairs];
#pragma unroll
        for (int g = 0; g < kGatherPairs; ++g) acc[g] = 0.f;
        for (int i0 = 0; i0 < n; i0 += 64) {
            const int i = i0 + lane;
            const int ii = i < n ? i : n - 1;
            float v[kGatherPairs];
#pragma unroll
            for (int g = 0; g < kGatherPairs; ++g) v[g] = x[g][ii];
            const float u = sU[ii], l = sL[ii];
#pragma unroll
            for (int g = 0; g < kGatherPairs; ++g)
                if (i < n) acc[g] = pacc<P>(acc[g], v[g] - __builtin_amdgcn_fmed3f(v[g], l, u));
        }
        float v4[4], v2[2];
        {
            const bool up = lane & 32;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float send = up ? acc[t] : acc[t + 4], keep = up ? acc[t + 4] : acc[t];
                v4[t] = pjoin<P>(keep, __shfl_xor(send, 32));
            }
        }
        {
            const bool up = lane & 16;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const float send = up ? v4[t] : v4[t + 2], keep = up ? v4[t + 2] : v4[t];
                v2[t] = pjoin<P>(keep, __shfl_xor(send, 16));
            }
        }
        const bool up = lane & 8;
        float v1 = pjoin<P>(up ? v2[1] : v2[0], __shfl_xor(up ? v2[0] : v2[1], 8));
        v1 = pjoin<P>(v1, __shfl_xor(v1, 4));
        v1 = pjoin<P>(v1, __shfl_xor(v1, 2));
        v1 = pjoin<P>(v1, __shfl_xor(v1, 1));
        // lanes 8g .. 8g+7 now hold the sum of pair g
        int cm = -1;
#pragma unroll
        for (int g = 0; g < kGatherPairs; ++g)
            if ((lane >> 3) == g) cm = c[g];
        if ((lane & 7) == 0 && cm >= 0) S1[q * ldS + cm] = v1;
    }
}

int lbk_gather_batch() { return kGatherPairs; }

hipError_t launch_lbk_gather(int p, const float *rows, int n, QueryData qd, PairList pl, const long long *prefix,
                             int64_t Q, int num_cu, float *S1, int64_t ldS, hipStream_t s) {
    const size_t lds = sizeof(float) * 2 * (size_t)n;
#define LBIMP_GATHER(PP)                                                                                              \
    hipLaunchKernelGGL(k_lbk_gather<PP>, dim3(persistent_grid(k_lbk_gather<PP>, lds, num_cu)), dim3(64), lds, s, rows, \
                       n, qd, pl, prefix, Q, S1, ldS)
    if (p == 1)
        LBIMP_GATHER(1);
    else if (p == 2)
        LBIMP_GATHER(2);
    else
        LBIMP_GATHER(kPInf);
#undef LBIMP_GATHER
    return hipGetLastError();
}

}  // namespace lbimp
