// Internal declarations shared by the kernel translation units and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbimp.h"
#include "pnorm.h"

namespace lbimp {

constexpr int kWave = 64;
constexpr float kInf = __builtin_huge_valf();
constexpr unsigned long long kNoKey = ~0ull;  // larger than every (distance, index) key
constexpr size_t kLdsBudget = 65536;          // dynamic LDS per workgroup used by any kernel
constexpr int kLaneMaxW = 63;                 // widest band (half-width) of the lane-per-pair DTW
// rows per group of the lane-per-pair DTW (its unit of early abandoning and of row phases)
constexpr int lane_rows(int w) { return w <= 32 ? 8 : w <= 53 ? 6 : 4; }
constexpr int kLbiRegMaxW = 52;               // widest band of the register-state LB_Improved
constexpr int kCounters = 5;                  // per-query counters of a search: cnt1, cnt2, rescnt, abandoned, cnt0
constexpr int kPdParts = 8;                   // parts d of the piecewise-sum cover (Sec. 9)
constexpr int kPdFine = 32;                   // parts of the fine cover of the fp32 first pass
constexpr int kPdfQuery = 3 * kPdFine + 4;    // floats per query of the fine cover's query table
constexpr int kPdfMinN = 64;                  // shortest series with a fine-cover table

// Launch wrappers.  Every pointer is device memory; all launches go to `s`.
// Each returns hipSuccess or the launch error.

// Copy [B][n] envelopes into rows of stride ldo padded with U = +inf, L = -inf (columns >= n
// and rows in [B, Bpad)), the layout the LB_Keogh sweep reads.
hipError_t launch_pad_env(const float *U, const float *L, int64_t B, int64_t Bpad, int n, float *Ud, float *Ld,
                          int ldo, hipStream_t s);

// Row-major [N][n] -> 64-candidate interleaved tiles [T][n4][64] of float4 (zero padded).
hipError_t launch_pack(const float *rows, int64_t N, int n, float4 *il, hipStream_t s);

// Envelope of B series (rows of length n) into rows of stride ldo; rows b in [B, Bpad) and
// columns i in [n, ldo) are filled with U = +inf, L = -inf when ldo > n or Bpad > B.
// keys0 / keys1, when given, receive "no key" in their first B entries; counts4 ([kCounters][B]),
// when given, receives 0 in all its entries.
hipError_t launch_envelope(const float *y, int64_t B, int64_t Bpad, int n, int w, float *U, float *L, int ldo,
                           hipStream_t s, unsigned long long *keys0 = nullptr, unsigned long long *keys1 = nullptr,
                           int *counts4 = nullptr);

// LB_Keogh^p of every interleaved candidate against Q padded envelopes (stride ld4 float4).
// Writes out[q*ldo + c] for c < N (and +inf for c in [N, ldo) when pad_inf).  root: take the
// p-th root (public output) instead of leaving the pow-domain value.
// wmin (optional, nn search only): wmin[q][v] = smallest (S1, index) key over the candidates of
// sweep wave v, v < sweep_waves(N, Q).
// shape: tiling variant (0 = default); rows of Ue/Le must be padded to a multiple of
// sweep_query_group(shape, Q) queries.  cbase is added to the candidate index of the wmin keys
// (a sweep over a chunk of a database: il, N and out are the chunk's).
hipError_t launch_lbk_sweep(int p, int shape, const float4 *il, int64_t N, int n4, const float4 *Ue,
                            const float4 *Le, int ld4, int64_t Q, float *out, int64_t ldo, bool pad_inf, bool root,
                            unsigned long long *wmin, hipStream_t s, int64_t cbase = 0);
int sweep_query_group(int shape, int64_t Q);
int64_t sweep_waves(int shape, int64_t N, int64_t Q);

// Per query: pick S candidates of small first-pass sum into seeds[q][0..S) and set their S1
// entries to +inf.  From the whole S1 row (wmin == nullptr), or from the nw per-wave minima of
// the sweep (one candidate per sweep wave).  S <= 64, S <= number of sources.  Candidates are
// [c0, N) and indexed globally: S1 may be a chunk's buffer shifted back by c0.
hipError_t launch_select_seeds(float *S1, int64_t ldS, int64_t N, int64_t Q, int S, const unsigned long long *wmin,
                               int64_t nw, int *seeds, hipStream_t s, int64_t c0 = 0);

// list[q][*] <- candidates c0 <= c < N with key(S1[q][c], c) < thr[q]; cnt[q] += number kept.
// Bucketed (cntb given): candidate c goes to bucket k = (c - c0) / bs, at list[q][k * bs + pos]
// with pos counted in cntb[k * Q + q]; bs must be a multiple of compact_wave_span().
hipError_t launch_compact(const float *S1, int64_t ldS, int64_t N, int64_t Q, const unsigned long long *thr,
                          int *list, int64_t ldl, int *cnt, hipStream_t s, int64_t c0 = 0, int64_t bs = 0,
                          int *cntb = nullptr);
int64_t compact_wave_span();

// prefix[0] = 0, prefix[q+1] = prefix[q] + ceil(count_q / batch), count_q = cnt[q] or `fixed`.
hipError_t launch_items_prefix(const int *cnt, int64_t fixed, int64_t Q, int batch, long long *prefix,
                               hipStream_t s);

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count, hipStream_t s);
hipError_t launch_fill_i32(int *p, int v, int64_t count, hipStream_t s);
hipError_t launch_iota_i32(int *p, int64_t count, hipStream_t s);  // p[i] = i

// Piecewise sums (Sec. 9) over the kPdParts parts of the cover, in fp64: pd [N][kPdParts] of
// the rows of a database; qpd [Q][2][kPdParts] of query envelopes (U sums, then L sums).
hipError_t launch_pd_rows(const float *rows, int64_t N, int n, double *pd, hipStream_t s);
hipError_t launch_pd_query(const float *U, const float *L, int ldq, int64_t Q, int n, double *qpd, hipStream_t s);
// Pass 0: the piecewise-sum bound of every candidate against Q queries into out[q][c] (pow
// domain, or root form with root), +inf in padding columns [N, ldo) when pad_inf; with wmin,
// the smallest (bound, index) key of every 64 candidates, wmin[q][v] for v < pd_scan_waves(N).
int64_t pd_scan_waves(int64_t N);
hipError_t launch_pd_scan(int p, const double *pd, int64_t N, int n, const double *qpd, int64_t Q, float *out,
                          int64_t ldo, bool pad_inf, bool root, unsigned long long *wmin, hipStream_t s,
                          int64_t cbase = 0);

// The same bound on the fine cover (kPdFine parts, fp32, with rounding margins that keep it below
// the exact bound): pdf [ceil(N/64)][kPdFine/4][64] float4 interleaved sums of a database's
// rows; qpf [Q][kPdfQuery] the query envelopes' sums and margins.  The scan writes out[q][c] and
// the per-wave minima wmin[q][v] of 128 candidates each (v < pdf_scan_waves(N)); the fine table is
// addressed by 64-candidate tiles, so a chunk's cbase must be a multiple of 64.
int64_t pdf_scan_waves(int64_t N);
hipError_t launch_pdf_rows(const float *rows, int64_t N, int n, float4 *pdf, hipStream_t s);
hipError_t launch_pdf_query(const float *U, const float *L, int ldq, int64_t Q, int n, float *qpf, hipStream_t s);
hipError_t launch_pdf_scan(int p, const float4 *pdf, int64_t N, int n, const float *qpf, int64_t Q, float *out,
                           int64_t ldo, bool root, unsigned long long *wmin, hipStream_t s, int64_t cbase);

// Pair list description for the persistent second-pass and DTW kernels.
// Bucketed lists (nb > 1): the candidates of each query are split by index range into nb
// buckets; bucket k of query q holds its pairs at list[q * ldl + k * bs + j] and counts them in
// cnt[k * cq + q].  The persistent kernels then walk the work bucket by bucket, each bucket on
// one XCD, so that the rows of a bucket, read by the pairs of every query, stay in that XCD's L2.
struct PairList {
    const int *list;     // [Q][ldl] candidate ids, or nullptr for "candidate = base + position"
    int64_t ldl;
    const int *cnt;      // [Q] counts ([nb][cq] when bucketed), or nullptr for `fixed` pairs per query
    int64_t fixed;
    int64_t base = 0;
    int nb = 1;          // buckets
    int64_t bs = 0;      // list entries per bucket
    int64_t cq = 0;      // row stride of the bucketed counts (the query count)
};

struct QueryData {
    const float *Y;      // [Q][ldy] queries
    int64_t ldy;
    const float *U, *L;  // [Q][ldq] envelopes (only the second pass reads them)
    int64_t ldq;
};

// Second pass.  S2 = S1[q][c] + sum_i d(y_i, env(H(x_c, y)))^p.  With thr: survivors with
// key(S2, c) < thr[q] are appended to list2/cnt2.  With out_root: out_root[c] = S2^(1/p)
// (single query).  prefix: items of `lbi_batch(n, w)` pairs; 0 means the per-lane envelope
// state of this (n, w) does not fit in LDS.  The kernels read prefix (launch_items_prefix
// over pl.cnt) only when pl.cnt is set; a fixed count per query maps items arithmetically.
// abandon: stop a pair's sum once it reaches the threshold (register and wave-per-pair kernels;
// only with thr and without out_root).  fused (w <= kLbiRegMaxW, with thr): S1 is not read; the
// kernel computes each pair's LB_Keogh from its row, counts per query in cntk the pairs whose
// LB_Keogh alone is below the threshold, and writes a survivor's LB_Keogh to S1out[q*ldS + c].
int lbi_batch(int n, int w);
hipError_t launch_lbi(int p, const float *rows, int64_t db_bytes, int n, int w, QueryData qd, PairList pl, const float *S1,
                      int64_t ldS, const long long *prefix, int64_t Q, int *ctr, int num_cu,
                      const unsigned long long *thr, int *list2, int64_t ldl2, int *cnt2, float *out_root,
                      int pipeline, bool abandon, hipStream_t s, bool fused = false, int *cntk = nullptr,
                      float *S1out = nullptr);

// LB_Keogh^p of the pairs of pl (the pass-0 survivors), reading each candidate's row: S1[q][c]
// receives the bound.  Items hold lbk_gather_batch() pairs; prefix is launch_items_prefix over
// pl.cnt.
int lbk_gather_batch();
hipError_t launch_lbk_gather(int p, const float *rows, int n, QueryData qd, PairList pl, const long long *prefix,
                             int64_t Q, int num_cu, float *S1, int64_t ldS, hipStream_t s);

// Banded DTW over a pair list.  best (k = 1): per-query best key, updated by atomicMin and used
// for early abandoning.  thr/res/rescnt (k > 1): keys below thr[q] are appended to res[q].
// out_root (single query): out_root[c] = DTW_p.  abandon=false computes every DTW in full.
// low_latency: a group of lanes per pair (few pairs, each finished quickly) instead of a lane
// per pair (many pairs, highest throughput).  Items hold dtw_batch(n, w, low_latency) pairs;
// prefix (launch_items_prefix over pl.cnt) is read only when pl.cnt is set.
// S1 (optional, [Q][ldS]): LB_Keogh^p of every pair against the query envelope qd.U/qd.L; the
// lane-per-pair kernels then abandon on the row minimum plus the LB_Keogh terms still to come.
// Lane-per-pair DTW of bands wider than kLaneMaxW keeps a per-wave ring of strip boundaries
// in `ring` (device scratch of at least dtw_strip_scratch(p, n, w, num_cu) bytes; 0 bytes
// when the band is narrow enough or low_latency is set).
int dtw_batch(int n, int w, bool low_latency);
bool dtw_wavereg_wide_supported(int n, int w);  // group-per-pair kernel for 63 < w (low_latency)
size_t dtw_strip_scratch(int p, int n, int w, int num_cu);
// Row phases of the lane-per-pair DTW (w <= kLaneMaxW, not low_latency): see DtwArgs.
struct DtwPhase {
    int row0, row1;
    bool resume;
    float *pool;
    int64_t pool_cap;
    int *pool_ctr;
    int *park_list;
    int64_t ld_park;
    int *park_cnt;
};
hipError_t launch_dtw(int p, const float *rows, int n, int w, QueryData qd, PairList pl, const long long *prefix,
                      int64_t Q, int *ctr, int num_cu, unsigned long long *best, const unsigned long long *thr,
                      unsigned long long *res, int64_t ldres, int *rescnt, int *abandoned, float *out_root,
                      bool abandon, bool low_latency, float *ring, size_t ring_bytes, const float *S1,
                      int64_t ldS, hipStream_t s, const DtwPhase *ph = nullptr);

// k-th smallest key of res[q][0..min(rescnt[q], 64)) into thr[q] (kNoKey if fewer than k), with
// k = kq[q] when kq (device [Q]) is given.
hipError_t launch_kth_key(const unsigned long long *res, int64_t ldres, const int *rescnt, int64_t Q, int k,
                          const int64_t *kq, unsigned long long *thr, hipStream_t s);

// 1-NN outputs from best keys, or k-NN outputs by selecting the k smallest of res[q] (k = kq[q]
// when kq is given).  Query q writes output row qmap[q] (or q when qmap is null) of ldo entries;
// entries past its k get idx -1 and dist +inf.
hipError_t launch_finalize1(const unsigned long long *best, int64_t Q, int p, int64_t *idx, float *dist,
                            const int64_t *qmap, int ldo, hipStream_t s);
hipError_t launch_finalize_k(unsigned long long *res, int64_t ldres, const int *rescnt, int64_t Q, int k,
                             const int64_t *kq, int ldo, int p, int64_t *idx, float *dist, const int64_t *qmap,
                             hipStream_t s);

// Between chunks of a search: res[q] keeps its k smallest keys, sorted (k = kq[q] when given),
// rescnt[q] their number, thr[q] the k-th (no key if fewer).
hipError_t launch_res_shrink(unsigned long long *res, int64_t ldres, int *rescnt, int64_t Q, int k, const int64_t *kq,
                             unsigned long long *thr, hipStream_t s);
// tot ([3][Q]) += the chunk's counts cnt1, cnt2, cnt0 of counters ([kCounters][Q]), which are cleared.
hipError_t launch_chunk_counts(int *counters, long long *tot, int64_t Q, hipStream_t s);

// dst[j][i] = src[off[j] + i] for j < count, i < n (gathers equal-length rows of a packed array).
hipError_t launch_gather_rows(const float *src, const int64_t *off, int n, int64_t count, float *dst, hipStream_t s);

}  // namespace lbimp
