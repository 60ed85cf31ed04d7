"""Planted mistakes (CPU only): copies of the oracle with one plausible error each must
fail at least one pin, which shows the pins constrain the oracle."""
import math

import numpy as np
import pytest

from oracle import reference as R
from tests import oracle_pins as P

INF = math.inf


def _dtw_variant(mistake):
    def dtw_pow(x, y, w, p):
        x, y = np.asarray(x, float), np.asarray(y, float)
        n = x.size
        D = np.full((n + 1, n + 1), INF)
        D[0, 0] = 0.0
        for i in range(n):
            lo, hi = max(0, i - w), min(n - 1, i + w)
            if mistake == "band_off_by_one":
                lo, hi = max(0, i - w + 1), min(n - 1, i + w - 1)
            for j in range(lo, hi + 1):
                c = abs(x[i] - y[j])
                if mistake == "cost_same_index":
                    c = abs(x[i] - y[i])
                if mistake == "no_diagonal":
                    best = min(D[i, j + 1], D[i + 1, j])
                    if i == 0 and j == 0:
                        best = 0.0
                elif mistake == "wrong_diag_index":
                    best = min(D[i, j + 1], D[i + 1, j], D[i, j + 1 if j + 1 <= n else j])
                    if i == 0 and j == 0:
                        best = 0.0
                else:
                    best = min(D[i, j + 1], D[i + 1, j], D[i, j])
                if mistake == "sum_instead_of_max" and p == INF:
                    D[i + 1, j + 1] = c + best
                elif p == INF:
                    D[i + 1, j + 1] = max(c, best)
                elif mistake == "power_missing":
                    D[i + 1, j + 1] = c + best
                else:
                    D[i + 1, j + 1] = c ** p + best
        return float(D[n, n])
    return dtw_pow


DTW_CHECKS = [
    lambda f, g: P.check_golden(f, g),
    lambda f, g: P.check_enumeration(f),
    lambda f, g: P.check_xyz_family(f),
    lambda f, g: P.check_w0_is_lp(f),
    lambda f, g: P.check_order_and_monotonicity(f),
    lambda f, g: P.check_value_separated_and_constant(f),
]


def _fails_some(checks, fn, golden_dir):
    for chk in checks:
        try:
            chk(fn, golden_dir)
        except (AssertionError, IndexError, ValueError):
            return True
    return False


def test_unmutated_variant_passes(golden_dir):
    assert not _fails_some(DTW_CHECKS, _dtw_variant(None), golden_dir)


@pytest.mark.parametrize("mistake", ["band_off_by_one", "cost_same_index", "no_diagonal", "wrong_diag_index",
                                     "sum_instead_of_max", "power_missing"])
def test_dtw_mistakes_are_caught(mistake, golden_dir):
    assert _fails_some(DTW_CHECKS, _dtw_variant(mistake), golden_dir)


def _envelope_printed_index(y, w):
    """Algorithm 1 with the emission one step early (as printed): must be caught."""
    y = np.asarray(y, float)
    n = y.size
    U, L, _ = R.envelope_stream(y, w)
    U2, L2 = U.copy(), L.copy()
    # emulate writing position m before sample m+w is pushed: the window misses its last sample
    for m in range(n):
        lo, hi = max(0, m - w), min(n - 1, m + w - 1) if m + w <= n - 1 else n - 1
        if hi >= lo:
            U2[m], L2[m] = y[lo:hi + 1].max(), y[lo:hi + 1].min()
    return U2, L2


def _envelope_half_window(y, w):
    return R.envelope_naive(y, max(0, w - 1))


@pytest.mark.parametrize("env", [_envelope_printed_index, _envelope_half_window])
def test_envelope_mistakes_are_caught(env):
    with pytest.raises(AssertionError):
        P.check_envelope(env)


def _lbk_swapped(x, U, L, p):
    x = np.asarray(x, float)
    H = np.where(x >= U, L, np.where(x <= L, U, x))
    return float(np.sum(np.abs(x - H) ** p))


def _lbi_envelope_of_x(x, y, U, L, w, p):
    # mistake: envelope of the raw candidate instead of its projection
    Ux, Lx = R.envelope_naive(x, w)
    return R.lb_keogh_pow(x, U, L, p) + R.lb_keogh_pow(y, Ux, Lx, p)


def _lbi_wrong_operand(x, y, U, L, w, p):
    # mistake: second pass measures x (not y) against the envelope of the projection
    xp = R.projection(x, U, L)
    Up, Lp = R.envelope_naive(xp, w)
    return R.lb_keogh_pow(x, U, L, p) + R.lb_keogh_pow(x, Up, Lp, p)


def _lbi_dropped_term(x, y, U, L, w, p):
    return R.lb_keogh_pow(x, U, L, p)


def _lbi_inf_sum(x, y, U, L, w, p):
    # mistake: for p = inf the two LB_Keogh terms added, as the p-th powers are for finite p
    xp = R.projection(x, U, L)
    Up, Lp = R.envelope_naive(xp, w)
    return R.lb_keogh_pow(x, U, L, p) + R.lb_keogh_pow(y, Up, Lp, p)


@pytest.mark.parametrize("lbk,lbi", [(_lbk_swapped, R.lb_improved_pow), (R.lb_keogh_pow, _lbi_envelope_of_x),
                                     (R.lb_keogh_pow, _lbi_wrong_operand), (R.lb_keogh_pow, _lbi_dropped_term),
                                     (R.lb_keogh_pow, _lbi_inf_sum)])
def test_lb_mistakes_are_caught(lbk, lbi):
    with pytest.raises(AssertionError):
        P.check_lb_chain(lbk, lbi, R.dtw_pow)


def _pd_unscaled(x, U, L, p, d=8):
    # mistake: the p-th powers of the part distances summed without the 1/|C|^(p-1) factor
    cover = R.pd_cover(len(x), d)
    px, pu, pl = (R.piecewise_sums(v, cover) for v in (x, U, L))
    dj = R.dist_to_interval(px, pl, pu)
    return float(np.max(dj)) if p == R.INF else float(np.sum(dj ** p))


def _pd_swapped(x, U, L, p, d=8):
    # mistake: the box taken from the upper envelope at its lower side
    return R.pd_bound_pow(x, L, U, p, d)


def _cover_ceil(n, d):
    # mistake: parts of width ceil(n/d), which overrun the series for the last parts
    m = -(-n // d)
    return [(j * m, min(n, (j + 1) * m)) for j in range(d - 1)] + [(min(n, (d - 1) * m), n)]


def _pd_with_ceil_cover(x, U, L, p, d=8):
    cover = _cover_ceil(len(x), d)
    px, pu, pl = (R.piecewise_sums(v, cover) for v in (x, U, L))
    dj = R.dist_to_interval(px, pl, pu)
    size = np.array([max(b - a, 1) for a, b in cover], dtype=float)
    return float(np.max(dj / size)) if p == R.INF else float(np.sum(dj ** p / size ** (p - 1)))


@pytest.mark.parametrize("fn,cover", [(_pd_unscaled, R.pd_cover), (_pd_swapped, R.pd_cover),
                                      (_pd_with_ceil_cover, _cover_ceil)])
def test_pd_mistakes_are_caught(fn, cover):
    with pytest.raises(AssertionError):
        P.check_pd_bound(fn, cover)
