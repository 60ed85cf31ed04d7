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

// ------------------------------------------------------------------ pass 0 on the fine cover
// The same bound on the cover of kPdFine = 32 parts (width floor(n/32), the last part taking the
// rest), evaluated in fp32 as the first pass of a search: on smooth series the sums over short
// parts lose little against LB_Keogh, at 32 terms per pair instead of n.  The sums are formed in
// fp64 and rounded to nearest fp32, so each differs from the exact sum by at most u = 2^-24 of
// its size; the distance of a part is 1-Lipschitz in its three sums, so it exceeds the exact one
// by at most u (|P(x)_j| + |P(L)_j| + |P(U)_j|) plus the rounding of the subtraction.  Every part
// gives up 4u of that sum (for p = 1 once for the whole series), and the total is shrunk by a
// few units of rounding, so the result stays below the exact bound of Sec. 9 and hence below
// LB_Keogh.
__device__ __forceinline__ void pdf_part(int n, int j, int &a, int &b) {
    const int m = n / kPdFine;
    a = j * m;
    b = j + 1 < kPdFine ? (j + 1) * m : n;
}

constexpr float kPdfEps = 4.f * 5.9604645e-8f;  // 4u

// Minimum of v over the wave, returned to every lane: DPP steps within quads, half-rows and rows,
// then row broadcasts carry the minimum to lane 63, which is read back.  No LDS round trips.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_min_step(float v) {
    const int o = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xf, false);
    return fminf(v, __int_as_float(o));
}
__device__ __forceinline__ float wave_min(float v) {
    v = dpp_min_step<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
    v = dpp_min_step<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
    v = dpp_min_step<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_min_step<0x140, 0xf>(v);  // row_mirror
    v = dpp_min_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_min_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// pdf: [ceil(N/64)][kPdFine/4][64] float4 -- candidate 64t + l, parts 4g..4g+3 at [t][g][l].
// One thread per (tile, group, lane); padding candidates get zeros.
__global__ __launch_bounds__(256) void k_pdf_rows(const float *__restrict__ rows, int64_t N, int n,
                                                   float4 *__restrict__ pdf) {
    constexpr int G = kPdFine / 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tiles = (N + 63) / 64;
    if (t >= tiles * G * 64) return;
    const int lane = (int)(t % 64), g = (int)((t / 64) % G);
    const int64_t c = (t / (64 * G)) * 64 + lane;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (c < N) {
        const float *x = rows + c * (int64_t)n;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int a, b;
            pdf_part(n, 4 * g + r, a, b);
            double sum = 0.0;
            for (int i = a; i < b; ++i) sum += (double)x[i];
            v[r] = (float)sum;
        }
    }
    pdf[t] = make_float4(v[0], v[1], v[2], v[3]);
}

hipError_t launch_pdf_rows(const float *rows, int64_t N, int n, float4 *pdf, hipStream_t s) {
    const int64_t total = (N + 63) / 64 * (kPdFine / 4) * 64;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pdf_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rows, N, n, pdf);
    return hipGetLastError();
}

// qpf[q]: P(U) [kPdFine], P(L) [kPdFine], the margins e_j = 4u (|P(U)_j| + |P(L)_j|) [kPdFine],
// then their total and padding (kPdfQuery floats).  One thread per (query, part).
__global__ __launch_bounds__(64) void k_pdf_query(const float *__restrict__ U, const float *__restrict__ L, int ldq,
                                                   int64_t Q, int n, float *__restrict__ qpf) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Q * kPdFine) return;
    const int64_t q = g / kPdFine;
    const int j = (int)(g % kPdFine);
    int a, b;
    pdf_part(n, j, a, b);
    double su = 0.0, sl = 0.0;
    for (int i = a; i < b; ++i) {
        su += (double)U[q * ldq + i];
        sl += (double)L[q * ldq + i];
    }
    const float fu = (float)su, fl = (float)sl;
    float *o = qpf + q * kPdfQuery;
    o[j] = fu;
    o[kPdFine + j] = fl;
    const float e = kPdfEps * (fabsf(fu) + fabsf(fl));
    o[2 * kPdFine + j] = e;
    // the total of the margins, summed by lane order within the part's wave slice
    float tot = e;
#pragma unroll
    for (int off = 1; off < kPdFine; off <<= 1) tot += __shfl_xor(tot, off, kPdFine);
    if (j == 0) o[3 * kPdFine] = tot * (1.f + 64.f * 5.9604645e-8f);
}

hipError_t launch_pdf_query(const float *U, const float *L, int ldq, int64_t Q, int n, float *qpf, hipStream_t s) {
    const int64_t total = Q * kPdFine;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pdf_query, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, U, L, ldq, Q, n, qpf);
    return hipGetLastError();
}

// Two candidates per lane (tiles 2v and 2v + 1 of wave v), block = 4 waves x up to QG queries
// (blockIdx.y), the query sums in LDS read as broadcasts and shared by both candidates.  Writes
// out[q][c] (pow domain, or root form with ROOT) and, per query and wave, the smallest (bound,
// index) key of the wave's 128 candidates.
template <int P, int QG, bool ROOT>
__global__ __launch_bounds__(256) void k_pdf_scan(const float4 *__restrict__ pdf, int64_t N, int n,
                                                   const float *__restrict__ qpf, int64_t Q, float *__restrict__ out,
                                                   int64_t ldo, unsigned long long *__restrict__ wmin, int64_t ldw,
                                                   int64_t cbase) {
    constexpr int G = kPdFine / 4;
    __shared__ float4 sq[QG][kPdfQuery / 4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.y * QG;
    for (int t = threadIdx.x; t < QG * kPdfQuery / 4; t += 256) {
        const int64_t q = q0 + t / (kPdfQuery / 4);
        sq[t / (kPdfQuery / 4)][t % (kPdfQuery / 4)] =
            q < Q ? reinterpret_cast<const float4 *>(qpf + q * kPdfQuery)[t % (kPdfQuery / 4)]
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int64_t v = (int64_t)blockIdx.x * 4 + wave;  // this wave's index among the scan's waves
    const int64_t tiles = (N + 63) / 64;
    float x[2][kPdFine];
    float sx[2] = {0.f, 0.f};  // sums of |P(x)_j|
    int64_t c[2];
    bool valid[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t tile = 2 * v + h;
        c[h] = tile * 64 + lane;
        valid[h] = c[h] < N;
        const int64_t tl = tile < tiles ? tile : 0;  // a tile past the end loads tile 0 (unused)
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const float4 w4 = pdf[(tl * G + g) * 64 + lane];
            x[h][4 * g] = w4.x, x[h][4 * g + 1] = w4.y, x[h][4 * g + 2] = w4.z, x[h][4 * g + 3] = w4.w;
            sx[h] += fabsf(w4.x) + fabsf(w4.y) + fabsf(w4.z) + fabsf(w4.w);
        }
    }
    // 1 / part size: every part but the last has floor(n/32) elements (an empty part has zero
    // distance)
    const int m = n / kPdFine;
    const float inv_m = m > 0 ? 1.f / (float)m : 0.f;
    const float inv_last = 1.f / (float)(n - (kPdFine - 1) * m);
    __syncthreads();
#pragma unroll 2
    for (int qq = 0; qq < QG; ++qq) {
        const int64_t q = q0 + qq;
        if (q >= Q) break;
        const float *sqf = reinterpret_cast<const float *>(sq[qq]);
        float acc[2] = {0.f, 0.f};
#pragma unroll
        for (int j = 0; j < kPdFine; ++j) {
            const float hi = sqf[j], lo = sqf[kPdFine + j];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float d = x[h][j] - __builtin_amdgcn_fmed3f(x[h][j], lo, hi);
                if constexpr (P == 1) {
                    acc[h] += fabsf(d);
                } else {
                    // this part's margin: 4u (|P(x)_j| + |P(U)_j| + |P(L)_j|)
                    const float ds = fmaxf(fabsf(d) - fmaf(kPdfEps, fabsf(x[h][j]), sqf[2 * kPdFine + j]), 0.f);
                    const float inv = j + 1 < kPdFine ? inv_m : inv_last;
                    if constexpr (P == 2)
                        acc[h] = fmaf(ds * inv, ds, acc[h]);
                    else
                        acc[h] = fmaxf(acc[h], ds * inv);
                }
            }
        }
        float f[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if constexpr (P == 1)
                f[h] = fmaxf(fmaf(acc[h], -64.f * 5.9604645e-8f, acc[h]) - fmaf(kPdfEps, sx[h], sqf[3 * kPdFine]), 0.f);
            else
                f[h] = acc[h] * (1.f - 64.f * 5.9604645e-8f);
            if (ROOT && P == 2) f[h] = sqrtf(f[h]) * (1.f - 4.f * 5.9604645e-8f);
            if (valid[h]) out[q * ldo + c[h]] = f[h];
        }
        if (wmin) {
            // the wave's smallest bound, then the smallest index holding it: the first tile's
            // candidates precede the second's, and within a tile the lowest lane comes first
            const float m = wave_min(fminf(valid[0] ? f[0] : kInf, valid[1] ? f[1] : kInf));
            const unsigned long long b0 = __ballot(valid[0] && f[0] == m), b1 = __ballot(valid[1] && f[1] == m);
            if (lane == 0) {
                unsigned long long k = kNoKey;
                if (b0)
                    k = make_key(m, (int)(2 * v * 64 + __ffsll(b0) - 1 + cbase));
                else if (b1)
                    k = make_key(m, (int)((2 * v + 1) * 64 + __ffsll(b1) - 1 + cbase));
                wmin[q * ldw + v] = k;
            }
        }
    }
}

int64_t pdf_scan_waves(int64_t N) { return (N + 511) / 512 * 4; }

template <int P, bool ROOT>
static void pdf_scan_launch(const float4 *pdf, int64_t N, int n, const float *qpf, int64_t Q, float *out, int64_t ldo,
                            unsigned long long *wmin, int64_t cbase, hipStream_t s) {
    constexpr int QG = 16;
    const dim3 grid((unsigned)((N + 511) / 512), (unsigned)((Q + QG - 1) / QG));
    hipLaunchKernelGGL((k_pdf_scan<P, QG, ROOT>), grid, dim3(256), 0, s, pdf, N, n, qpf, Q, out, ldo, wmin,
                       pdf_scan_waves(N), cbase);
}

hipError_t launch_pdf_scan(int p, const float4 *pdf, int64_t N, int n, const float *qpf, int64_t Q, float *out,
                           int64_t ldo, bool root, unsigned long long *wmin, hipStream_t s, int64_t cbase) {
    if (N == 0 || Q == 0) return hipSuccess;
    if (p == 1)
        pdf_scan_launch<1, false>(pdf, N, n, qpf, Q, out, ldo, wmin, cbase, s);
    else if (p == 2)
        root ? pdf_scan_launch<2, true>(pdf, N, n, qpf, Q, out, ldo, wmin, cbase, s)
             : pdf_scan_launch<2, false>(pdf, N, n, qpf, Q, out, ldo, wmin, cbase, s);
    else
        pdf_scan_launch<kPInf, false>(pdf, N, n, qpf, Q, out, ldo, wmin, cbase, s);
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
