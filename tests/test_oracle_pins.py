"""Oracle pins (CPU): the Python and C oracles against the paper's values, closed forms,
invariants, a library special case and brute-force path enumeration."""
import math

import numpy as np
import pytest

from oracle import native
from oracle import reference as R
from tests import oracle_pins as P

DTW_IMPLS = {"python": R.dtw_pow, "python_many": lambda x, y, w, p: float(
    R.dtw_pow_many(np.atleast_2d(np.asarray(x, float)), y, w, p)[0]), "c": native.dtw_pow}


@pytest.fixture(params=sorted(DTW_IMPLS))
def dtw_impl(request):
    return DTW_IMPLS[request.param]


def test_golden_examples(dtw_impl, golden_dir):
    P.check_golden(dtw_impl, golden_dir)


def test_enumeration(dtw_impl):
    P.check_enumeration(dtw_impl)


def test_xyz_family(dtw_impl):
    P.check_xyz_family(dtw_impl)


def test_w0_is_lp(dtw_impl):
    P.check_w0_is_lp(dtw_impl)


def test_order_and_monotonicity(dtw_impl):
    P.check_order_and_monotonicity(dtw_impl)


def test_value_separated_and_constant(dtw_impl):
    P.check_value_separated_and_constant(dtw_impl)


def test_weak_triangle(dtw_impl):
    P.check_weak_triangle(dtw_impl)


def test_step_path_counts_are_central_delannoy():
    # central Delannoy numbers: sum_k C(m,k) C(m+k,k) with m = n-1
    for n in range(1, 7):
        m = n - 1
        want = sum(math.comb(m, k) * math.comb(m + k, k) for k in range(m + 1))
        assert sum(1 for _ in R.step_paths(n, n)) == want
    assert [sum(1 for _ in R.step_paths(n, n)) for n in range(1, 7)] == [1, 3, 13, 63, 321, 1683]


def test_step_paths_respect_band():
    for n in range(1, 7):
        for w in range(n + 1):
            for path in R.step_paths(n, w):
                assert path[0] == (0, 0) and path[-1] == (n - 1, n - 1)
                assert all(abs(i - j) <= w for i, j in path)
                assert all((a - i, b - j) in ((1, 0), (0, 1), (1, 1)) for (i, j), (a, b) in zip(path, path[1:]))


def test_minimal_path_length_bound():
    # App. A: a minimal warping path has at most 2n-2 matches (n > 1); the optimal step
    # path under strictly positive costs is minimal, so its length obeys the same bound.
    g = np.random.default_rng(11)
    for _ in range(50):
        n = int(g.integers(2, 7))
        x, y = g.standard_normal(n), g.standard_normal(n)
        best, best_len = math.inf, None
        for path in R.step_paths(n, n):
            c = sum(abs(x[i] - y[j]) + 1e-9 for i, j in path)
            if c < best:
                best, best_len = c, len(path)
        assert best_len <= 2 * n - 2 or n == 1


def test_envelope_naive():
    P.check_envelope(R.envelope_naive)


def test_envelope_stream():
    P.check_envelope(R.envelope_stream)


def test_envelope_c():
    P.check_envelope(native.envelope)


def test_envelope_stream_comparison_count():
    # Sec. 6: at most 3n comparisons between data values
    g = np.random.default_rng(12)
    for t in range(300):
        n = int(g.integers(1, 200))
        w = int(g.integers(0, n + 2))
        y = g.integers(-2, 3, n).astype(float) if t % 3 == 0 else np.cumsum(g.standard_normal(n))
        assert R.envelope_stream(y, w)[2] <= 3 * n


def test_envelope_special_cases():
    y = np.array([3.0, -1.0, 2.0, 5.0, 0.0])
    U, L, _ = R.envelope_stream(y, 0)
    assert np.array_equal(U, y) and np.array_equal(L, y)
    for w in (4, 5, 100):
        U, L, _ = R.envelope_stream(y, w)
        assert np.all(U == 5.0) and np.all(L == -1.0)
    U, L, _ = R.envelope_stream(np.array([2.5]), 3)
    assert U[0] == 2.5 and L[0] == 2.5


def test_lb_chain_python():
    P.check_lb_chain(R.lb_keogh_pow, R.lb_improved_pow, R.dtw_pow)


def test_lb_c_matches_python():
    g = np.random.default_rng(13)
    for t in range(20):
        n = int(g.integers(1, 60))
        w = int(g.integers(0, n + 1))
        X = np.cumsum(g.standard_normal((7, n)), axis=1)
        y = np.cumsum(g.standard_normal(n))
        U, L = R.envelope_naive(y, w)
        for p in (1, 2, 3, math.inf):
            s1, s2 = native.lb_many(X, y, w, p)
            for c in range(7):
                assert P._rel_close(s1[c], R.lb_keogh_pow(X[c], U, L, p), 1e-12)
                assert P._rel_close(s2[c], R.lb_improved_pow(X[c], y, U, L, w, p), 1e-12)


def test_theorem1_general_h():
    P.check_theorem1_general_h(R.dtw_pow)


def test_lemma1():
    P.check_lemma1()


def test_projection_in_envelope():
    g = np.random.default_rng(14)
    for _ in range(50):
        n = int(g.integers(1, 40))
        w = int(g.integers(0, n))
        x, y = g.standard_normal(n) * 2, g.standard_normal(n)
        U, L = R.envelope_naive(y, w)
        H = R.projection(x, U, L)
        assert np.all(H <= U) and np.all(H >= L)
        inside = (x < U) & (x > L)
        assert np.array_equal(H[inside], x[inside])


def test_c_dtw_matches_python_large():
    g = np.random.default_rng(15)
    for n, w in ((128, 13), (256, 26), (97, 200), (64, 0)):
        X = np.cumsum(g.standard_normal((5, n)), axis=1)
        y = np.cumsum(g.standard_normal(n))
        for p in (1, 2):
            a = native.dtw_pow_many(X, y, w, p)
            b = R.dtw_pow_many(X, y, R.effective_band(n, w), p)
            assert np.allclose(a, b, rtol=1e-12, atol=0)


def test_pd_bound():
    P.check_pd_bound(R.pd_bound_pow, R.pd_cover)


def test_pd_bound_many_matches_rows():
    g = np.random.default_rng(22)
    for n, w, d in ((50, 5, 8), (7, 3, 8), (131, 13, 8), (64, 0, 4), (256, 26, 32), (100, 10, 32)):
        X = np.cumsum(g.standard_normal((30, n)), axis=1)
        U, L = R.envelope_naive(np.cumsum(g.standard_normal(n)), w)
        for p in (1, 2, math.inf):
            many = R.pd_bound_pow_many(X, U, L, p, d)
            for c in range(X.shape[0]):
                assert P._rel_close(many[c], R.pd_bound_pow(X[c], U, L, p, d), 1e-12)


def test_pd_fine_cover():
    """The 32-part cover of the fp32 first pass: P_32 <= LB_Keogh <= DTW for every p; for p = 1
    on nested covers (n a multiple of 32) refining the 8 parts into 32 never lowers the bound,
    since the distance of a sum over a union of parts is at most the sum of the parts' distances;
    and n = 32 (one element per part) gives LB_Keogh exactly."""
    g = np.random.default_rng(23)
    for t in range(40):
        n = int(g.choice([64, 96, 128, 256, 100, 131]))
        w = int(g.integers(0, n // 4 + 1))
        x = np.cumsum(g.standard_normal(n))
        y = np.cumsum(g.standard_normal(n))
        U, L = R.envelope_naive(y, w)
        for p in (1, 2, math.inf):
            b32 = R.pd_bound_pow(x, U, L, p, 32)
            k = R.lb_keogh_pow(x, U, L, p)
            assert -1e-12 <= b32 <= k * (1 + 1e-12) + 1e-12, (n, w, p)
        if n % 32 == 0:
            assert R.pd_bound_pow(x, U, L, 1, 32) >= R.pd_bound_pow(x, U, L, 1, 8) * (1 - 1e-12) - 1e-12
    x = np.cumsum(g.standard_normal(32))
    U, L = R.envelope_naive(np.cumsum(g.standard_normal(32)), 3)
    for p in (1, 2, math.inf):
        assert P._rel_close(R.pd_bound_pow(x, U, L, p, 32), R.lb_keogh_pow(x, U, L, p), 1e-12)
