"""The App. B triangle-inequality experiment on the device: 100,000 triples (x, y, z) of
100-sample series, unconstrained DTW_1 and DTW_2 (w >= n), the statistic
C(x, y, z) = DTW_p(x, z) / (DTW_p(x, y) + DTW_p(y, z)) and the share of triples with C > 1.

All 300,000 distances of each p come from lbimp_dtw_pairs.  Checked: a seeded sample of
triples against the fp64 oracle, distance by distance and violation by violation (a decision
may differ only where C is within the distance tolerance of 1); the weak triangle inequality
of App. B, C <= min(2w+1, n)^(1/p), on every triple; no violation on white noise; and the
random-walk violation shares near the paper's 20% (DTW_1) and 15% (DTW_2).
"""
import numpy as np
import pytest
import torch

from oracle import native
from paper_0811_3301_amd import gen
from tests.test_gpu_parity import L, ctx, _say, f32, rt, to_dev  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu

COUNT, N_LEN = 100_000, 100
PAPER_SHARE = {1: 0.20, 2: 0.15}


def _triple_distances(L, ctx, X, Y, Z, p):
    Xd, Yd, Zd = to_dev(X), to_dev(Y), to_dev(Z)
    w = N_LEN  # unconstrained
    dxy = L.lbimp_dtw_pairs(ctx, Xd, Yd, w, p).cpu().numpy().astype(np.float64)
    dyz = L.lbimp_dtw_pairs(ctx, Yd, Zd, w, p).cpu().numpy().astype(np.float64)
    dxz = L.lbimp_dtw_pairs(ctx, Xd, Zd, w, p).cpu().numpy().astype(np.float64)
    return dxy, dyz, dxz


@pytest.mark.parametrize("p", [1, 2])
def test_triangle_random_walk_full_size(L, ctx, p):
    _say(f"triangle experiment, random walks, 100000 triples, p={p}")
    X, Y, Z = (f32(a).astype(np.float64) for a in gen.triangle_triples(COUNT, N_LEN, "random_walk"))
    dxy, dyz, dxz = _triple_distances(L, ctx, X, Y, Z, p)
    C = dxz / (dxy + dyz)
    assert np.all(C <= N_LEN ** (1.0 / p) * (1 + 1e-5))  # weak triangle inequality, min(2w+1, n) = n
    share = float(np.mean(C > 1))
    _say(f"  violation share {share:.4f} (paper: {PAPER_SHARE[p]:.2f})")
    assert abs(share - PAPER_SHARE[p]) < 0.05
    sample = gen.rng(6, 9, p).choice(COUNT, 300, replace=False)
    flips = 0
    for t in sample:
        o = [rt(native.dtw_pow(a[t], b[t], N_LEN - 1, p), p) for a, b in ((X, Y), (Y, Z), (X, Z))]
        for g, want in zip((dxy[t], dyz[t], dxz[t]), o):
            assert abs(g - want) <= 1e-5 * max(want, 1e-3), (t, g, want)
        c_orc = o[2] / (o[0] + o[1])
        if (c_orc > 1) != (C[t] > 1):
            assert abs(c_orc - 1) <= 3e-5, (t, c_orc, C[t])
            flips += 1
    assert flips <= 3


def test_triangle_white_noise_has_no_violation(L, ctx):
    _say("triangle experiment, white noise, 100000 triples, p=1 and p=2")
    X, Y, Z = (f32(a).astype(np.float64) for a in gen.triangle_triples(COUNT, N_LEN, "white_noise"))
    for p in (1, 2):
        dxy, dyz, dxz = _triple_distances(L, ctx, X, Y, Z, p)
        assert np.sum(dxz > dxy + dyz) == 0, p
