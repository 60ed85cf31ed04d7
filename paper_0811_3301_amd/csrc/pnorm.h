// The l_p aggregation of Sec. 2 for the exponents the kernels take: p = 1 and p = 2 sum p-th
// powers, p = infinity takes a maximum (DTW_inf of the Sec. 4 recursion, LB_Keogh_inf of Sec. 7).
// Every distance and bound on the path stays in this "pow" domain -- sums of |d|^p, or maxima
// of |d| -- and the root is taken only for reported values.
#pragma once

#include <hip/hip_runtime.h>

#include "lbimp.h"

namespace lbimp {

constexpr int kPInf = LBIMP_P_INF;  // template value of p = infinity

// acc combined with |d|^p: acc + |d|, acc + d*d (one fma), or max(acc, |d|).
template <int P>
__device__ __forceinline__ float pacc(float acc, float d) {
    if constexpr (P == 1)
        return acc + fabsf(d);
    else if constexpr (P == 2)
        return fmaf(d, d, acc);
    else
        return fmaxf(acc, fabsf(d));
}

// Two pow-domain partial results of disjoint index sets combined: a sum, or a maximum.
template <int P>
__device__ __forceinline__ float pjoin(float a, float b) {
    if constexpr (P == kPInf)
        return fmaxf(a, b);
    else
        return a + b;
}

// Root form of a pow-domain value.
template <int P>
__device__ __forceinline__ float root_p(float v) {
    if constexpr (P == 2)
        return sqrtf(v);
    else
        return v;
}

}  // namespace lbimp
