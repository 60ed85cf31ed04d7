"""Pin checks for the oracle: each takes the function under test as an argument.

The oracle tests call these with the oracle's own functions; the mutation tests
call them with copies that carry a planted mistake and expect a failure.  Every
check compares against something other than the oracle itself: values the paper
prints, closed forms, invariants proved in the paper, a library routine for a
special case, or brute-force enumeration.
"""
from __future__ import annotations

import math
import os

import numpy as np
from scipy.ndimage import maximum_filter1d, minimum_filter1d

from oracle import reference as R

INF = math.inf
PS = (1, 2, 3, INF)


def _rel_close(a, b, tol=1e-9):
    return abs(a - b) <= tol * max(1.0, abs(a), abs(b))


def root(v, p):
    return v if p in (1, INF) else v ** (1.0 / p)


def load_golden(path):
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, cite, p, ws, x, y, val = [f.strip() for f in line.split("|")]
            rows.append(dict(name=name, cite=cite, p=INF if p == "inf" else int(p),
                             ws=[int(v) for v in ws.split(",")],
                             x=[float(v) for v in x.split(",")], y=[float(v) for v in y.split(",")],
                             value=float(val)))
    return rows


def check_golden(dtw_pow, golden_dir):
    rows = load_golden(os.path.join(golden_dir, "paper_examples.txt"))
    assert len(rows) >= 10
    for r in rows:
        for w in r["ws"]:
            got = dtw_pow(r["x"], r["y"], w, r["p"])
            assert _rel_close(got, r["value"], 1e-12), (r["name"], w, got, r["value"])


def check_enumeration(dtw_pow, seed=0, trials=400):
    """DP against the minimum over all step paths, n <= 6, every w, p in {1,2,3,inf}."""
    g = np.random.default_rng(seed)
    for t in range(trials):
        n = int(g.integers(1, 7))
        w = int(g.integers(0, n + 1))
        p = PS[t % 4]
        if t % 2:
            x, y = g.integers(-3, 4, n).astype(float), g.integers(-3, 4, n).astype(float)
        else:
            x, y = g.standard_normal(n), g.standard_normal(n)
        want = R.dtw_enumerate(x, y, w, p)
        got = dtw_pow(x, y, w, p)
        assert _rel_close(got, want, 1e-12), (x, y, w, p, got, want)


def check_xyz_family(dtw_pow):
    """App. B: X=0^(2m+1), Y=0^m e 0^m, Z=0 e^(2m-1) 0 at w=m-1 give |e|, 0, (2m-1)^(1/p)|e|."""
    for m in range(1, 6):
        n = 2 * m + 1
        for eps in (0.5, -1.25, 3.0):
            X = [0.0] * n
            Y = [0.0] * m + [eps] + [0.0] * m
            Z = [0.0] + [eps] * (2 * m - 1) + [0.0]
            for p in (1, 2, 3):
                w = m - 1
                assert _rel_close(root(dtw_pow(X, Y, w, p), p), abs(eps)), (m, eps, p)
                assert _rel_close(dtw_pow(Y, Z, w, p), 0.0), (m, eps, p)
                assert _rel_close(root(dtw_pow(X, Z, w, p), p), (2 * m - 1) ** (1.0 / p) * abs(eps)), (m, eps, p)


def check_w0_is_lp(dtw_pow, seed=1):
    """Sec. 4: with w = 0 the DTW is the l_p distance."""
    g = np.random.default_rng(seed)
    for t in range(60):
        n = int(g.integers(1, 40))
        x, y = g.standard_normal(n), g.standard_normal(n)
        p = PS[t % 4]
        want = R._combine(np.abs(x - y) ** (1 if p == INF else p), p)
        assert _rel_close(dtw_pow(x, y, 0, p), want), (n, p)


def check_order_and_monotonicity(dtw_pow, seed=2):
    """DTW <= l_p (Sec. 4), non-increasing in w (Sec. 4), symmetric (App. B),
    and DTW_q <= DTW_p <= (2n-2)^(1/p-1/q) DTW_q for p < q (App. A proposition)."""
    g = np.random.default_rng(seed)
    for t in range(40):
        n = int(g.integers(2, 24))
        x = np.cumsum(g.standard_normal(n))
        y = np.cumsum(g.standard_normal(n))
        for p in (1, 2, INF):
            prev = INF
            lp = R._combine(np.abs(x - y) ** (1 if p == INF else p), p)
            for w in range(0, n + 1):
                d = dtw_pow(x, y, w, p)
                assert d <= lp * (1 + 1e-12)
                assert d <= prev * (1 + 1e-12), (n, p, w)
                assert _rel_close(d, dtw_pow(y, x, w, p))
                prev = d
        w = int(g.integers(0, n))
        vals = {p: root(dtw_pow(x, y, w, p), p) for p in (1, 2, 3, INF)}
        for p, q in ((1, 2), (1, 3), (2, 3), (1, INF), (2, INF), (3, INF)):
            e = 1.0 / p - (0.0 if q == INF else 1.0 / q)
            assert vals[q] <= vals[p] * (1 + 1e-12), (p, q)
            assert vals[p] <= (2 * n - 2) ** e * vals[q] * (1 + 1e-12), (p, q)


def check_value_separated_and_constant(dtw_pow, seed=3):
    """Prop. 1: x >= c >= y gives DTW_1 = ||x-y||_1; App. A lemma: constant y gives ||x-y||_p;
    App. A: translation invariance DTW(x+b, z+b) = DTW(x, z)."""
    g = np.random.default_rng(seed)
    for t in range(60):
        n = int(g.integers(1, 30))
        w = int(g.integers(0, n + 1))
        c = g.standard_normal()
        x = c + np.abs(g.standard_normal(n))
        y = c - np.abs(g.standard_normal(n))
        if t % 2:
            x, y = y, x
        assert _rel_close(dtw_pow(x, y, w, 1), np.abs(x - y).sum()), (n, w)
        yc = np.full(n, c)
        for p in PS:
            want = R._combine(np.abs(x - yc) ** (1 if p == INF else p), p)
            assert _rel_close(dtw_pow(x, yc, w, p), want), (n, w, p)
        z = np.cumsum(g.standard_normal(n))
        s = 4.0 * g.standard_normal()
        for p in PS:
            assert _rel_close(dtw_pow(x + s, z + s, w, p), dtw_pow(x, z, w, p), 1e-9), (n, w, p)


def check_weak_triangle(dtw_pow, seed=4):
    """App. B theorem: DTW(x,y) + DTW(y,z) >= DTW(x,z) / min(2w+1, n)^(1/p)."""
    g = np.random.default_rng(seed)
    for t in range(80):
        n = int(g.integers(1, 16))
        w = int(g.integers(0, n + 1))
        x, y, z = (np.cumsum(g.standard_normal(n)) for _ in range(3))
        for p in PS:
            a = root(dtw_pow(x, y, w, p), p)
            b = root(dtw_pow(y, z, w, p), p)
            c = root(dtw_pow(x, z, w, p), p)
            k = min(2 * w + 1, n)
            fac = 1.0 if p == INF else k ** (1.0 / p)
            assert a + b >= c / fac * (1 - 1e-12), (n, w, p)


def check_envelope(envelope, seed=5):
    """Sec. 5 definition via SciPy's windowed max/min (edge-replicating windows equal cut windows)."""
    g = np.random.default_rng(seed)
    for t in range(300):
        n = int(g.integers(1, 50))
        w = int(g.integers(0, n + 3))
        y = g.integers(-3, 4, n).astype(float) if t % 2 else g.standard_normal(n)
        U, L = envelope(y, w)[:2]
        size = 2 * w + 1
        assert np.array_equal(U, maximum_filter1d(y, size=size, mode="nearest")), (y, w)
        assert np.array_equal(L, minimum_filter1d(y, size=size, mode="nearest")), (y, w)


def check_lb_chain(lb_keogh_pow, lb_improved_pow, dtw_pow, seed=6):
    """LB_Keogh <= LB_Improved <= DTW (Sec. 7 and Sec. 8 corollaries); the LB_Keogh error
    bound DTW - LB_Keogh <= ||max(U-y, y-L)||_p (Sec. 7 corollary); at w = 0 all three equal l_p;
    for value-separated series with p = 1 the LB_Keogh error is exactly ||H - y||_1 (Sec. 5)."""
    g = np.random.default_rng(seed)
    strict = 0
    for t in range(150):
        n = int(g.integers(1, 40))
        w = int(g.integers(0, max(1, n // 2) + 1))
        x = np.cumsum(g.standard_normal(n))
        y = np.cumsum(g.standard_normal(n))
        U, L = R.envelope_naive(y, w)
        for p in PS:
            k = lb_keogh_pow(x, U, L, p)
            i = lb_improved_pow(x, y, U, L, w, p)
            d = dtw_pow(x, y, w, p)
            assert k <= i * (1 + 1e-12) + 1e-12, (n, w, p)
            assert i <= d * (1 + 1e-12) + 1e-12, (n, w, p, i, d)
            strict += i > k * (1 + 1e-9)
            gap = np.maximum(U - y, y - L)
            err = root(R._combine(gap if p == INF else gap ** p, p), p)
            assert root(d, p) - root(k, p) <= err * (1 + 1e-9) + 1e-12
        U0, L0 = R.envelope_naive(y, 0)
        for p in (1, 2, INF):
            lp = R._combine(np.abs(x - y) if p == INF else np.abs(x - y) ** p, p)
            assert _rel_close(lb_keogh_pow(x, U0, L0, p), lp)
            assert _rel_close(lb_improved_pow(x, y, U0, L0, 0, p), lp)
        c = g.standard_normal()
        xs, ys = c + np.abs(g.standard_normal(n)), c - np.abs(g.standard_normal(n))
        Us, Ls = R.envelope_naive(ys, w)
        H = R.projection(xs, Us, Ls)
        assert _rel_close(dtw_pow(xs, ys, w, 1) - lb_keogh_pow(xs, Us, Ls, 1), np.abs(H - ys).sum(), 1e-9)
    assert strict > 50, "LB_Improved should be strictly tighter on many random pairs"


def check_theorem1_general_h(dtw_pow, seed=7):
    """Theorem 1 with any h between x and the envelope of y, bounded below through LB_Keogh:
    DTW_p(x,y)^p >= ||x-h||_p^p + LB_Keogh_p(y, h)^p (LB_Improved is the case h = H(x,y))."""
    g = np.random.default_rng(seed)
    for t in range(120):
        n = int(g.integers(1, 30))
        w = int(g.integers(0, n + 1))
        x = np.cumsum(g.standard_normal(n))
        y = np.cumsum(g.standard_normal(n))
        U, L = R.envelope_naive(y, w)
        lam = g.uniform(0, 1, n)
        H = R.projection(x, U, L)
        h = H + lam * (x - H)                   # anywhere between x_i and its projection
        Uh, Lh = R.envelope_naive(h, w)
        for p in (1, 2, 3):
            lhs = dtw_pow(x, y, w, p)
            rhs = np.sum(np.abs(x - h) ** p) + R.lb_keogh_pow(y, Uh, Lh, p)
            assert lhs >= rhs * (1 - 1e-12) - 1e-12, (n, w, p)


def check_lemma1(seed=8):
    """Lemma 1: b in [a, c] implies (c-a)^p >= (c-b)^p + (b-a)^p."""
    g = np.random.default_rng(seed)
    for _ in range(1000):
        a, c = sorted(g.standard_normal(2) * 5)
        b = g.uniform(a, c)
        for p in (1, 2, 3, 4):
            assert (c - a) ** p >= ((c - b) ** p + (b - a) ** p) * (1 - 1e-12)


def check_pd_bound(pd_bound_pow, pd_cover, seed=21):
    """P_d (Sec. 9): the cover is d disjoint parts of width floor(n/d), the last taking the rest;
    d(P_d(x), [P_d(L), P_d(U)]) <= LB_Keogh <= DTW (Sec. 9 chain, extended to p = 2 and inf);
    d = n reduces to LB_Keogh exactly (one element per part); candidates entirely above the
    envelope reduce it to LB_Keogh_1 exactly for p = 1 (every clamped difference has one sign)."""
    g = np.random.default_rng(seed)
    for n in (1, 2, 5, 7, 8, 9, 16, 100, 131):
        for d in (1, 3, 8, n):
            cover = pd_cover(n, d)
            m = n // d
            assert len(cover) == d and cover[-1][1] == n
            assert all(b - a == m for a, b in cover[:-1]) and cover[-1][1] - cover[-1][0] == n - (d - 1) * m
            assert all(cover[j][1] == cover[j + 1][0] for j in range(d - 1)) and cover[0][0] == 0
    for t in range(120):
        n = int(g.integers(1, 60))
        w = int(g.integers(0, n + 1))
        d = int(g.integers(1, 12))
        x = np.cumsum(g.standard_normal(n))
        y = np.cumsum(g.standard_normal(n))
        U, L = R.envelope_naive(y, w)
        for p in PS:
            b = pd_bound_pow(x, U, L, p, d)
            k = R.lb_keogh_pow(x, U, L, p)
            assert -1e-12 <= b <= k * (1 + 1e-12) + 1e-12, (n, w, d, p, b, k)
            assert k <= R.dtw_pow(x, y, w, p) * (1 + 1e-12) + 1e-12
            assert _rel_close(pd_bound_pow(x, U, L, p, n), k, 1e-12), (n, w, p)
        above = U + np.abs(g.standard_normal(n)) + 0.1
        assert _rel_close(pd_bound_pow(above, U, L, 1, d), R.lb_keogh_pow(above, U, L, 1), 1e-12)
