"""The tightened abandon bound of the DTW kernels never exceeds the DTW computed in fp32.

After rows 0..i the kernels bound a pair's DTW_p from below by
    (min of row i + max(S1 - sum_{r<=i} lbk_r, 0)) * (1 - (6n + 16) * 2^-24)
with S1 the LB_Keogh^p sum of the first pass (any summation order) and lbk_r the LB_Keogh^p
term of row r.  This test replays that arithmetic in IEEE float32 (numpy) next to a float32
DTW_p with the kernels' cell order, over random walks, white noise and near-flat series, with
S1 summed in several orders, and checks the bound at every row.  (A check of fp32 rounding
margins; the DTW itself is pinned elsewhere against the oracle.)"""
import numpy as np
import pytest

from paper_0811_3301_amd import gen

F = np.float32


def _env(y, w):
    n = len(y)
    U = np.array([y[max(0, i - w):i + w + 1].max() for i in range(n)], dtype=F)
    L = np.array([y[max(0, i - w):i + w + 1].min() for i in range(n)], dtype=F)
    return U, L


def _lbk_terms(x, U, L, p):
    d = (x - np.minimum(np.maximum(x, L), U)).astype(F)
    return np.abs(d) if p == 1 else (d * d).astype(F)


def _dtw_rows_f32(x, y, w, p):
    """float32 DTW_p rows (prefix form), cell by cell in the kernels' order; returns row minima and final."""
    n = len(x)
    inf = F(np.inf)
    prev = np.full(n, inf, dtype=F)
    rowmins = []
    for i in range(n):
        cur = np.full(n, inf, dtype=F)
        for j in range(max(0, i - w), min(n, i + w + 1)):
            up = prev[j]
            diag = prev[j - 1] if j > 0 else (F(0) if i == 0 else inf)
            if i == 0 and j == 0:
                diag = F(0)
            left = cur[j - 1] if j > 0 else inf
            m = min(diag, up, left)
            d = F(x[i] - y[j])
            cur[j] = F(m + abs(d)) if p == 1 else F(np.fma(d, d, m) if hasattr(np, "fma") else F(m + F(d * d)))
        rowmins.append(cur.min())
        prev = cur
    return np.array(rowmins, dtype=F), prev[n - 1]


def _sums(t):
    """S1 in several float32 summation orders."""
    yield F(np.sum(t, dtype=F))
    acc = F(0)
    for v in t[::-1]:
        acc = F(acc + v)
    yield acc
    acc = F(0)
    for v in t:
        acc = F(acc + v)
    yield acc
    yield F(np.sum(t.reshape(-1, 4).T.reshape(-1), dtype=F)) if len(t) % 4 == 0 else F(np.sum(t, dtype=F))


CASES = [("walk", 32, 3), ("walk", 64, 8), ("noise", 48, 5), ("flat", 40, 4), ("walk", 96, 20),
         ("flat", 1024, 8), ("walk", 1024, 16), ("flat", 4096, 3)]


@pytest.mark.parametrize("kind,n,w", CASES)
@pytest.mark.parametrize("p", [1, 2])
def test_bound_never_exceeds_fp32_dtw(kind, n, w, p):
    r = gen.rng(900, 0, n, w, p)
    shrink = F(1.0 - (6.0 * n + 16.0) * 5.9604645e-8)
    worst = 0.0
    for trial in range(12 if n < 200 else 2):
        if kind == "walk":
            x, y = gen.random_walk(2, n, r)
        elif kind == "noise":
            x, y = gen.white_noise(2, n, r)
        else:  # near-flat: x close to y, where bound and DTW nearly meet
            y = gen.random_walk(1, n, r)[0]
            x = y + 1e-4 * r.standard_normal(n)
        x, y = x.astype(F), y.astype(F)
        U, L = _env(y, w)
        t = _lbk_terms(x, U, L, p)
        rowmins, final = _dtw_rows_f32(x, y, w, p)
        for S1 in _sums(t):
            done = F(0)
            for i in range(n):
                done = F(done + t[i])
                rem = max(F(S1 - done), F(0))
                bound = F(F(rowmins[i] + rem) * shrink)
                assert bound <= final, (kind, n, w, p, trial, i, bound, final)
                if final > 0:
                    worst = max(worst, float(bound / final))
    assert worst <= 1.0
