"""Plain fp64 reference of every quantity on the search path (TEST INFRASTRUCTURE ONLY).

Each function follows a definition of Lemire, "Faster Retrieval with a Two-Pass
Dynamic-Time-Warping Lower Bound" (arXiv:0811.3301); the passage is named in its
docstring.  Indices are 0-based here; the paper counts from 1.

Exponents: ``p`` is a positive integer or ``math.inf``.  Quantities in the
"pow" domain (``*_pow``) are p-th powers (sums of |.|^p); for p = inf they are
maxima.  Root-form functions return the paper's distances.

Nothing here is blocked, fused or reordered beyond the definitions; speed is not
a goal.  Inputs are widened to float64 before any arithmetic.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

INF = math.inf


# ---------------------------------------------------------------- helpers
def _as64(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


def _pow_abs(d, p):
    """|d|^p elementwise (p a positive integer); for p = inf just |d|."""
    d = np.abs(d)
    if p == INF:
        return d
    if p == 1:
        return d
    if p == 2:
        return d * d
    return d ** p


def _combine(values, p):
    """Sum of p-th powers, or the maximum for p = inf (the l_p aggregation, Sec. 2)."""
    values = np.asarray(values, dtype=np.float64)
    if values.size == 0:
        return 0.0
    return float(values.max()) if p == INF else float(values.sum())


def root(v: float, p) -> float:
    """Undo the p-th power of a pow-domain value."""
    if p == INF or p == 1:
        return float(v)
    if p == 2:
        return math.sqrt(v)
    return float(v) ** (1.0 / p)


def effective_band(n: int, w: int) -> int:
    """w >= n means no locality constraint (Sec. 4); the widest useful band is n-1."""
    if w < 0:
        raise ValueError("the locality constraint w must be >= 0")
    return min(int(w), max(n - 1, 0))


# ---------------------------------------------------------------- l_p (Sec. 2)
def lp_distance(x, y, p) -> float:
    """||x - y||_p = (sum |x_i - y_i|^p)^(1/p); max |x_i - y_i| for p = inf (Sec. 2)."""
    x, y = _as64(x), _as64(y)
    return root(_combine(_pow_abs(x - y, p), p), p)


# ---------------------------------------------------------------- envelopes (Sec. 5)
def envelope_naive(y, w):
    """U_i = max{y_k : |k-i| <= w}, L_i = min{...}, windows cut to the series (Sec. 5)."""
    y = _as64(y)
    n = y.size
    U = np.empty(n)
    L = np.empty(n)
    for i in range(n):
        lo, hi = max(0, i - w), min(n - 1, i + w)
        U[i] = y[lo:hi + 1].max()
        L[i] = y[lo:hi + 1].min()
    return U, L


def envelope_stream(y, w):
    """Streaming envelope with two monotone double-ended queues (Algorithm 1, Sec. 6).

    Index queues ``u`` (candidates for the window maximum, values decreasing from
    front to back) and ``l`` (for the minimum) are updated once per new sample.
    A single comparison of y_i with y_{i-1} decides which queue loses its back
    element, so at most 3n value comparisons are made in total.

    The output for position m is written once every sample of its window
    [m-w, m+w] has been pushed, i.e. before sample m+w+1 is processed: one step
    later than the printed listing, whose emission would precede the push of the
    window's last sample.  Returns (U, L, number of value comparisons).
    """
    y = _as64(y)
    n = y.size
    U = np.full(n, np.nan)
    L = np.full(n, np.nan)
    if n == 0:
        return U, L, 0
    comps = 0
    u = deque([0])
    l = deque([0])
    for i in range(1, n):
        m = i - 1 - w                    # every sample of m's window is already queued
        if m >= 0:
            U[m] = y[u[0]]
            L[m] = y[l[0]]
        comps += 1
        if y[i] > y[i - 1]:
            u.pop()                      # y_{i-1} can no longer be a window maximum
            while u:
                comps += 1
                if y[i] > y[u[-1]]:
                    u.pop()
                else:
                    break
        else:
            l.pop()                      # y_{i-1} can no longer be a window minimum
            while l:
                comps += 1
                if y[i] < y[l[-1]]:
                    l.pop()
                else:
                    break
        u.append(i)
        l.append(i)
        # the next emitted window is [i-2w, i]: drop an index that just left it
        if u[0] == i - 2 * w - 1:
            u.popleft()
        elif l[0] == i - 2 * w - 1:
            l.popleft()
    for m in range(max(0, n - 1 - w), n):
        while u[0] < m - w:
            u.popleft()
        while l[0] < m - w:
            l.popleft()
        U[m] = y[u[0]]
        L[m] = y[l[0]]
    return U, L, comps


# ---------------------------------------------------------------- projection and LB_Keogh (Sec. 7)
def projection(x, U, L):
    """H(x,y)_i: U_i if x_i >= U_i, L_i if x_i <= L_i, else x_i  (Sec. 7, eq. of H)."""
    x, U, L = _as64(x), _as64(U), _as64(L)
    H = x.copy()
    H[x >= U] = U[x >= U]
    low = (x <= L) & ~(x >= U)
    H[low] = L[low]
    return H


def dist_to_interval(v, lo, hi):
    """d(v, [lo, hi]) for each coordinate: v-hi above, lo-v below, 0 inside (Sec. 2 set distance)."""
    v, lo, hi = _as64(v), _as64(lo), _as64(hi)
    return np.where(v > hi, v - hi, np.where(v < lo, lo - v, 0.0))


def lb_keogh_pow(x, U, L, p) -> float:
    """LB_Keogh_p(x,y)^p = ||x - H(x,y)||_p^p with (U, L) the envelope of y (Sec. 7)."""
    x = _as64(x)
    return _combine(_pow_abs(x - projection(x, U, L), p), p)


def lb_keogh(x, U, L, p) -> float:
    return root(lb_keogh_pow(x, U, L, p), p)


# ---------------------------------------------------------------- LB_Improved (Sec. 8)
def lb_improved_pow(x, y, U, L, w, p) -> float:
    """LB_Improved_p(x,y)^p = LB_Keogh_p(x,y)^p + LB_Keogh_p(y, H(x,y))^p, 1 <= p < inf (Sec. 8).

    The second term measures y against the envelope (same w) of the projection
    x' = H(x,y) of the candidate onto the envelope (U, L) of the query.

    p = inf: the paper defines LB_Improved for finite p only.  Theorem 1 (Sec. 5) states
    DTW_inf(x,y) >= max(||x - h||_inf, NDTW_inf(h,y)) for the same h, and applied again to
    (y, h) it gives NDTW_inf(h,y) >= LB_Keogh_inf(y, h); so the bound for p = inf is the
    maximum of the two LB_Keogh terms (the p-th-power sum becomes a maximum, as in l_inf).
    """
    x, y = _as64(x), _as64(y)
    xp = projection(x, U, L)
    Up, Lp = envelope_naive(xp, w)
    first, second = lb_keogh_pow(x, U, L, p), lb_keogh_pow(y, Up, Lp, p)
    return max(first, second) if p == INF else first + second


def lb_improved(x, y, U, L, w, p) -> float:
    return root(lb_improved_pow(x, y, U, L, w, p), p)


# ---------------------------------------------------------------- piecewise sums P_d (Sec. 9)
def pd_cover(n: int, d: int):
    """The cover of Sec. 9: C_j = [j*m, (j+1)*m) for j < d-1 and C_{d-1} = [(d-1)*m, n), with
    m = floor(n/d) (0-based, half-open).  When n < d the first d-1 parts are empty."""
    m = n // d
    return [(j * m, (j + 1) * m) for j in range(d - 1)] + [((d - 1) * m, n)]


def piecewise_sums(x, cover) -> np.ndarray:
    """P_d(x) = (sum_{i in C_j} x_i)_j (Sec. 9)."""
    x = _as64(x)
    return np.array([x[a:b].sum() for a, b in cover])


def pd_bound_pow(x, U, L, p, d=8) -> float:
    """Distance of P_d(x) to the box [P_d(L), P_d(U)] spanned by the envelope of the query
    (Sec. 9), a lower bound of LB_Keogh: sum_j d(P_d(x)_j, [P_d(L)_j, P_d(U)_j]) for p = 1.

    For p = 1 this is the bound the paper states.  For other p the term of part j is
    d_j^p / |C_j|^(p-1) (and max_j d_j / |C_j| for p = inf): d_j <= sum_{i in C_j} d(x_i, [L_i, U_i])
    (the sum of the clamped differences of one sign), and (sum over |C| terms)^p <= |C|^(p-1)
    times the sum of their p-th powers (power-mean inequality); an empty part adds nothing."""
    cover = pd_cover(len(_as64(x)), d)
    px, pu, pl = piecewise_sums(x, cover), piecewise_sums(U, cover), piecewise_sums(L, cover)
    dj = dist_to_interval(px, pl, pu)
    size = np.array([b - a for a, b in cover], dtype=np.float64)
    live = size > 0
    if p == INF:
        return float(np.max(dj[live] / size[live])) if live.any() else 0.0
    return float(np.sum(dj[live] ** p / size[live] ** (p - 1)))


def pd_bound_pow_many(X, U, L, p, d=8) -> np.ndarray:
    """pd_bound_pow of every row of X (the same formula, one row per vector lane)."""
    X = _as64(X)
    cover = pd_cover(X.shape[1], d)
    px = np.stack([X[:, a:b].sum(axis=1) for a, b in cover], axis=1)
    pu, pl = piecewise_sums(U, cover), piecewise_sums(L, cover)
    dj = np.where(px > pu, px - pu, np.where(px < pl, pl - px, 0.0))
    size = np.array([b - a for a, b in cover], dtype=np.float64)
    live = size > 0
    if p == INF:
        return (dj[:, live] / size[live]).max(axis=1) if live.any() else np.zeros(X.shape[0])
    return (dj[:, live] ** p / size[live] ** (p - 1)).sum(axis=1)


# ---------------------------------------------------------------- DTW_p (Sec. 4)
def dtw_pow(x, y, w, p) -> float:
    """DTW_p(x,y)^p by dynamic programming over the band |i-j| <= w (Sec. 4 recursion).

    The paper recurses over suffixes; reversing every path gives the equivalent
    prefix form D(i,j) = |x_i - y_j|^p + min(D(i-1,j), D(i,j-1), D(i-1,j-1))
    with D(-1,-1) = 0 and every other out-of-range or out-of-band cell infinite.
    For p = inf the sum becomes a maximum.
    """
    x, y = _as64(x), _as64(y)
    n = x.size
    if y.size != n:
        raise ValueError("equal lengths required")
    if n == 0:
        return 0.0
    D = np.full((n + 1, n + 1), INF)           # D[i+1][j+1] holds cell (i, j)
    D[0, 0] = 0.0
    for i in range(n):
        for j in range(max(0, i - w), min(n - 1, i + w) + 1):
            c = abs(x[i] - y[j])
            best = min(D[i, j + 1], D[i + 1, j], D[i, j])
            if p == INF:
                D[i + 1, j + 1] = max(c, best)
            else:
                D[i + 1, j + 1] = (c if p == 1 else c ** p) + best
    return float(D[n, n])


def dtw(x, y, w, p) -> float:
    return root(dtw_pow(x, y, w, p), p)


def dtw_pow_many(X, y, w, p) -> np.ndarray:
    """dtw_pow of every row of X against y: the same recursion, one candidate per vector lane."""
    X, y = _as64(X), _as64(y)
    N, n = X.shape
    prev = np.full((N, n + 1), INF)            # row i-1, column j+1 holds cell (i-1, j)
    prev[:, 0] = 0.0                           # D(-1,-1) = 0
    for i in range(n):
        cur = np.full((N, n + 1), INF)
        for j in range(max(0, i - w), min(n - 1, i + w) + 1):
            c = np.abs(X[:, i] - y[j])
            best = np.minimum(np.minimum(prev[:, j + 1], cur[:, j]), prev[:, j])
            if p == INF:
                cur[:, j + 1] = np.maximum(c, best)
            else:
                cur[:, j + 1] = (c if p == 1 else c ** p) + best
        prev = cur
    return prev[:, n].copy()


def step_paths(n: int, w: int):
    """Every monotone step path from (0,0) to (n-1,n-1) with |i-j| <= w, as lists of cells.

    Steps are (1,0), (0,1), (1,1).  Exponential in n: for n <= 6 only.
    """
    if n <= 0:
        return
    stack = [[(0, 0)]]
    while stack:
        path = stack.pop()
        i, j = path[-1]
        if i == n - 1 and j == n - 1:
            yield path
            continue
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            a, b = i + di, j + dj
            if a < n and b < n and abs(a - b) <= w:
                stack.append(path + [(a, b)])


def dtw_enumerate(x, y, w, p) -> float:
    """Minimum over every step path inside the band of its l_p cost (brute force, p-th power).

    Every minimal warping path (Sec. 4) is such a path, and extra matches only add
    non-negative cost, so the minimum over step paths is DTW_p^p.
    """
    x, y = _as64(x), _as64(y)
    best = INF
    for path in step_paths(x.size, w):
        cost = _combine([_pow_abs(x[i] - y[j], p) for i, j in path], p)
        best = min(best, cost)
    return float(best)


# ---------------------------------------------------------------- nearest neighbours
def key_order(d_pow: np.ndarray):
    """Candidate order by (distance, index): ties go to the smaller index."""
    d_pow = np.asarray(d_pow)
    return np.lexsort((np.arange(d_pow.size), d_pow))


def nn_bruteforce(y, DB, w, p, k=1):
    """The k nearest candidates under DTW_p by computing every distance (the definition).

    Returns (indices, DTW_p distances, all pow-domain distances).
    """
    DB = _as64(DB)
    if DB.shape[0] == 0:
        return np.full(k, -1), np.full(k, INF), np.zeros(0)
    w = effective_band(DB.shape[1], w)
    D = dtw_pow_many(DB, y, w, p)
    order = key_order(D)[:k]
    return order, np.array([root(D[c], p) for c in order]), D


def nn_sequential(y, DB, w, p, improved: bool):
    """Sequential 1-NN scan in database order (Algorithm 2, or Algorithm 3 if ``improved``).

    Bounds and the best-so-far ``b`` are kept as p-th powers (the tests against b
    are unchanged by the monotone map t -> t^p).  A candidate is examined further
    only while its bound is strictly below b, and b is replaced only by a strictly
    smaller distance, so the first candidate in database order wins a tie.
    Returns (index, DTW_p, counters) with counters for the pruning passes and the
    value comparisons made outside the DTW.
    """
    y, DB = _as64(y), _as64(DB)
    N, n = DB.shape
    w = effective_band(n, w)
    U, L, env_comps = envelope_stream(y, w)
    b, best = INF, -1
    cnt = dict(pruned_keogh=0, pruned_improved=0, dtw=0, comparisons=env_comps)
    for c in range(N):
        x = DB[c]
        beta = 0.0
        xp = x.copy()
        for i in range(n):
            cnt["comparisons"] += 1
            if x[i] > U[i]:
                beta += _pow_abs(x[i] - U[i], p)
                xp[i] = U[i]
            else:
                cnt["comparisons"] += 1
                if x[i] < L[i]:
                    beta += _pow_abs(L[i] - x[i], p)
                    xp[i] = L[i]
        if not beta < b:
            cnt["pruned_keogh"] += 1
            continue
        if improved:
            Up, Lp, ec = envelope_stream(xp, w)
            cnt["comparisons"] += ec
            for i in range(n):
                cnt["comparisons"] += 1
                if y[i] > Up[i]:
                    beta += _pow_abs(y[i] - Up[i], p)
                else:
                    cnt["comparisons"] += 1
                    if y[i] < Lp[i]:
                        beta += _pow_abs(Lp[i] - y[i], p)
            if not beta < b:
                cnt["pruned_improved"] += 1
                continue
        t = dtw_pow(x, y, w, p)
        cnt["dtw"] += 1
        if t < b:
            b, best = t, c
    return best, root(b, p), cnt
