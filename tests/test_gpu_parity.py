"""GPU parity: every C-ABI entry point against the fp64 oracle on the same seeded inputs.

The oracle sees the float32-rounded inputs widened to float64 (what the device sees).
Distances: |gpu - oracle| <= 1e-5 * max(oracle, 1e-3 * ||x - y||_p) (relative error with a
floor for values near 0).  Nearest-neighbour indices: equal to the oracle's, unless the
oracle's distance of the device's pick is within that tolerance of the minimum (a tie).
Envelopes are exact (max/min of the inputs).
"""
import os

import numpy as np
import pytest
import torch

from oracle import native
from oracle import reference as R
from paper_0811_3301_amd import gen

pytestmark = pytest.mark.gpu

RTOL = 1e-5
INF = float("inf")


def rt(v, p):
    """Root form of pow-domain values: v^(1/p); for p = 1 and p = inf the value itself."""
    v = np.asarray(v, dtype=np.float64)
    return v if p in (1, INF) else v ** (1.0 / p)


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def L():
    from paper_0811_3301_amd import lbimp
    lbimp.load()
    return lbimp


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Ctx(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def f32(a):
    return np.asarray(a, dtype=np.float32)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(f32(a))).cuda()


def lp_scale(X, y, p):
    d = np.abs(X - y[None, :])
    return d.max(axis=1) if p == INF else (d ** p).sum(axis=1) ** (1.0 / p)


def assert_close(gpu, orc, scale, what):
    gpu, orc, scale = np.asarray(gpu, np.float64), np.asarray(orc, np.float64), np.asarray(scale, np.float64)
    tol = RTOL * np.maximum(np.abs(orc), 1e-3 * scale) + 1e-30
    err = np.abs(gpu - orc)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first {bad[:5]}: gpu {gpu[bad[:5]]} oracle {orc[bad[:5]]}"
    return float(np.max(err / np.maximum(np.abs(orc), 1e-30))) if orc.size else 0.0


def walks(count, n, seed):
    return f32(gen.random_walk(count, n, gen.rng(500, 0, seed))).astype(np.float64)


# ------------------------------------------------------------------ envelopes
@pytest.mark.parametrize("B,n,w", [(3, 1, 0), (2, 2, 1), (4, 63, 5), (4, 64, 0), (5, 65, 64), (2, 100, 200),
                                   (3, 257, 26), (2, 300, 63), (2, 1024, 205),
                                   (1, 4096, 409)])
def test_envelope(L, ctx, B, n, w):
    _say(f"envelope B={B} n={n} w={w}")
    Y = walks(B, n, n + w)
    U, Lo = L.lbimp_envelope(ctx, to_dev(Y), w)
    U, Lo = U.cpu().numpy(), Lo.cpu().numpy()
    for b in range(B):
        Uo, Loo = R.envelope_naive(Y[b], R.effective_band(n, w))
        assert np.array_equal(U[b].astype(np.float64), Uo)
        assert np.array_equal(Lo[b].astype(np.float64), Loo)


# ------------------------------------------------------------------ LB_Keogh
@pytest.mark.parametrize("N,n", [(1, 1), (63, 7), (64, 128), (65, 131), (1000, 256)])
@pytest.mark.parametrize("p", [1, 2, INF])
def test_lb_keogh(L, ctx, N, n, p):
    _say(f"lb_keogh N={N} n={n} p={p}")
    X = walks(N, n, 1)
    y = walks(1, n, 2)[0]
    w = max(0, n // 10)
    Uo, Lo = R.envelope_naive(y, w)
    lb = L.lbimp_lb_keogh(ctx, to_dev(X), to_dev(Uo), to_dev(Lo), p).cpu().numpy()
    s1, _ = native.lb_many(X, y, w, p)
    assert_close(lb, rt(s1, p), lp_scale(X, y, p), "lb_keogh")


@pytest.mark.parametrize("Q", [1, 3, 17, 40])
@pytest.mark.parametrize("p", [1, 2, INF])
@pytest.mark.parametrize("shape", [0, 2, 3, 4, 5])
def test_db_lb_keogh(L, ctx, Q, p, shape):
    N, n, w = 777, 96, 9
    _say(f"db_lb_keogh Q={Q} p={p} shape={shape}")
    X = walks(N, n, 3)
    Ys = walks(Q, n, 4)
    db = L.Db(ctx, to_dev(X))
    env = [R.envelope_naive(Ys[q], w) for q in range(Q)]
    U = to_dev(np.stack([e[0] for e in env]))
    Lo = to_dev(np.stack([e[1] for e in env]))
    L.lbimp_ctx_set_option(ctx, "sweep_shape", shape)
    try:
        lb = L.lbimp_db_lb_keogh(ctx, db, U, Lo, p).cpu().numpy()
    finally:
        L.lbimp_ctx_set_option(ctx, "sweep_shape", 0)
    for q in range(Q):
        s1, _ = native.lb_many(X, Ys[q], w, p)
        assert_close(lb[q], rt(s1, p), lp_scale(X, Ys[q], p), f"db_lb_keogh q={q}")
    db.close()


# ------------------------------------------------------------------ LB_Improved
@pytest.mark.parametrize("N,n,w", [(70, 32, 3), (130, 128, 13), (65, 256, 26), (40, 512, 51), (20, 1024, 205),
                                   (10, 50, 100), (9, 5, 0), (130, 300, 80), (70, 129, 128), (66, 512, 53),
                                   (65, 1000, 300), (12, 1500, 400), (5, 2100, 60), (70, 17, 1), (70, 45, 5),
                                   (70, 97, 10), (70, 64, 15), (70, 63, 16), (70, 200, 20), (70, 100, 31)])
@pytest.mark.parametrize("p", [1, 2, INF])
def test_lb_improved(L, ctx, N, n, w, p):
    _say(f"lb_improved N={N} n={n} w={w} p={p}")
    X = walks(N, n, 5)
    y = walks(1, n, 6)[0]
    wb = R.effective_band(n, w)
    Uo, Lo = R.envelope_naive(y, wb)
    lb = L.lbimp_lb_improved(ctx, to_dev(X), to_dev(y), to_dev(Uo), to_dev(Lo), w, p).cpu().numpy()
    _, s2 = native.lb_many(X, y, wb, p)
    assert_close(lb, rt(s2, p), lp_scale(X, y, p), "lb_improved")


# ------------------------------------------------------------------ DTW
@pytest.mark.parametrize("N,n,w", [(70, 1, 0), (70, 2, 1), (130, 64, 0), (130, 128, 13), (65, 256, 26),
                                   (33, 512, 51), (20, 300, 63), (10, 200, 64), (8, 512, 102), (4, 97, 500),
                                   (3, 1024, 205), (67, 77, 2), (45, 33, 7), (66, 4096, 31), (5, 40, 40),
                                   (130, 300, 80), (70, 129, 128), (65, 66, 65)])
@pytest.mark.parametrize("p", [1, 2, INF])
@pytest.mark.parametrize("group", [0, 1])
def test_dtw_band(L, ctx, N, n, w, p, group):
    _say(f"dtw_band N={N} n={n} w={w} p={p} group_per_pair={group}")
    X = walks(N, n, 7)
    y = walks(1, n, 8)[0]
    L.lbimp_ctx_set_option(ctx, "dtw_group_per_pair", group)
    try:
        d = L.lbimp_dtw_band(ctx, to_dev(X), to_dev(y), w, p).cpu().numpy()
    finally:
        L.lbimp_ctx_set_option(ctx, "dtw_group_per_pair", 0)
    D = native.dtw_pow_many(X, y, R.effective_band(n, w), p)
    assert_close(d, rt(D, p), lp_scale(X, y, p), "dtw_band")


def test_paper_worked_examples_through_the_abi(L, ctx, golden_dir):
    """The DTW values the paper prints (tests/golden/paper_examples.txt: Sec. 4 and App. A,
    including the DTW_inf examples) computed by lbimp_dtw_band, for every exponent the device
    takes (p = 3 lines are oracle-only)."""
    _say("paper worked examples through lbimp_dtw_band")
    done = 0
    for line in open(os.path.join(golden_dir, "paper_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, _, ptxt, wtxt, xtxt, ytxt, want = [f.strip() for f in line.split("|")]
        p = INF if ptxt == "inf" else int(ptxt)
        if p not in (1, 2, INF):
            continue
        x = np.array([float(v) for v in xtxt.split(",")])
        y = np.array([float(v) for v in ytxt.split(",")])
        for w in (int(v) for v in wtxt.split(",")):
            for group in (0, 1):
                L.lbimp_ctx_set_option(ctx, "dtw_group_per_pair", group)
                try:
                    d = float(L.lbimp_dtw_band(ctx, to_dev(x[None, :]), to_dev(y), w, p).cpu()[0])
                finally:
                    L.lbimp_ctx_set_option(ctx, "dtw_group_per_pair", 0)
                expect = float(rt(float(want), p))
                assert abs(d - expect) <= 1e-6 * max(1.0, expect), (name, w, group, d, expect)
                done += 1
    assert done >= 40


@pytest.mark.parametrize("N,n,w", [(70, 100, 99), (65, 64, 5), (40, 128, 13), (33, 300, 80), (20, 1000, 205),
                                   (9, 2000, 1500), (5, 7, 100), (1, 1, 0)])
@pytest.mark.parametrize("p", [1, 2, INF])
def test_dtw_pairs(L, ctx, N, n, w, p):
    """DTW of N independent pairs (row c of x against row c of y), each with its own query."""
    _say(f"dtw_pairs N={N} n={n} w={w} p={p}")
    X = walks(N, n, 30)
    Y = walks(N, n, 31)
    d = L.lbimp_dtw_pairs(ctx, to_dev(X), to_dev(Y), w, p).cpu().numpy()
    wb = R.effective_band(n, w)
    D = np.array([native.dtw_pow(X[c], Y[c], wb, p) for c in range(N)])
    scale = np.array([lp_scale(X[c][None, :], Y[c], p)[0] for c in range(N)])
    assert_close(d, rt(D, p), scale, "dtw_pairs")


# ------------------------------------------------------------------ piecewise-sum bound (Sec. 9)
@pytest.mark.parametrize("N,n", [(1, 1), (63, 7), (300, 8), (65, 131), (1000, 256), (70, 1000)])
@pytest.mark.parametrize("p", [1, 2, INF])
def test_db_pd_bound(L, ctx, N, n, p):
    _say(f"db_pd_bound N={N} n={n} p={p}")
    X = walks(N, n, 32)
    Ys = walks(3, n, 33)
    w = max(0, n // 10)
    db = L.Db(ctx, to_dev(X))
    env = [R.envelope_naive(Ys[q], w) for q in range(3)]
    lb = L.lbimp_db_pd_bound(ctx, db, to_dev(np.stack([e[0] for e in env])), to_dev(np.stack([e[1] for e in env])),
                             p).cpu().numpy()
    for q in range(3):
        want = rt(R.pd_bound_pow_many(X, env[q][0], env[q][1], p), p)
        assert_close(lb[q], want, lp_scale(X, Ys[q], p), f"pd_bound q={q}")
        s1, _ = native.lb_many(X, Ys[q], w, p)
        assert np.all(lb[q] <= rt(s1, p) * (1 + 1e-6) + 1e-6)  # below LB_Keogh
    db.close()


@pytest.mark.parametrize("N,n", [(300, 64), (65, 131), (1000, 256), (70, 1000), (129, 100)])
@pytest.mark.parametrize("p", [1, 2, INF])
def test_db_pd_bound_fine(L, ctx, N, n, p):
    """The 32-part cover in fp32: never above the oracle's exact bound on the same cover (the
    rounding margins), within a few parts per million of it, and below LB_Keogh."""
    _say(f"db_pd_bound fine N={N} n={n} p={p}")
    X = walks(N, n, 52)
    Ys = walks(3, n, 53)
    w = max(0, n // 10)
    db = L.Db(ctx, to_dev(X))
    env = [R.envelope_naive(Ys[q], w) for q in range(3)]
    L.lbimp_ctx_set_option(ctx, "pd_fine", 1)
    try:
        lb = L.lbimp_db_pd_bound(ctx, db, to_dev(np.stack([e[0] for e in env])),
                                 to_dev(np.stack([e[1] for e in env])), p).cpu().numpy().astype(np.float64)
    finally:
        L.lbimp_ctx_set_option(ctx, "pd_fine", 0)
    for q in range(3):
        want = rt(R.pd_bound_pow_many(X, env[q][0], env[q][1], p, d=32), p)
        scale = lp_scale(X, Ys[q], p)
        assert np.all(lb[q] <= want), f"fine bound above the exact one, q={q}"
        assert np.all(want - lb[q] <= 2e-5 * scale + 1e-6), f"fine bound too loose, q={q}"
        s1, _ = native.lb_many(X, Ys[q], w, p)
        assert np.all(lb[q] <= rt(s1, p) * (1 + 1e-6) + 1e-6)  # below LB_Keogh
    db.close()


def test_db_pd_bound_fine_short_series(L, ctx):
    """No 32-part sums below 64 samples: the fine bound is refused, the 8-part one works."""
    X = walks(50, 40, 54)
    db = L.Db(ctx, to_dev(X))
    U = to_dev(X[:1])
    L.lbimp_ctx_set_option(ctx, "pd_fine", 1)
    try:
        with pytest.raises(L.LbimpError):
            L.lbimp_db_pd_bound(ctx, db, U, U, 1)
    finally:
        L.lbimp_ctx_set_option(ctx, "pd_fine", 0)
    L.lbimp_db_pd_bound(ctx, db, U, U, 1)
    db.close()


def fine_parts(pd, mode, n, w):
    """Parts of the pass-0 cover a search uses: 32 where the fine flow applies, else 8."""
    return 32 if (pd == 2 and mode == "improved" and n >= 64 and R.effective_band(n, w) <= 52) else 8


@pytest.mark.parametrize("mode", ["keogh", "improved"])
@pytest.mark.parametrize("p,k", [(1, 1), (2, 3), (INF, 2), (1, 10)])
@pytest.mark.parametrize("n,w", [(128, 13), (200, 80), (37, 4), (256, 26), (64, 6), (100, 52)])
@pytest.mark.parametrize("pd", [1, 2])
def test_nn_search_pd_prefilter(L, ctx, mode, p, k, n, w, pd):
    """Pass 0 (piecewise sums, 8 parts ahead of LB_Keogh, or 32 parts with LB_Keogh computed
    inside LB_Improved): the same answers, bit for bit, as without it, matching the oracle; the
    pass prunes on random walks; counts stay within the invariants of the cover used."""
    _say(f"nn_search pd_prefilter={pd} mode={mode} p={p} k={k} n={n} w={w}")
    X = walks(3000, n, 34)
    Ys = walks(7, n, 35)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    ri, rd, _ = L.lbimp_nn_search(ctx, db, Yd, w, p, k, mode)
    L.lbimp_ctx_set_option(ctx, "pd_prefilter", pd)
    try:
        idx, dist, st = L.lbimp_nn_search(ctx, db, Yd, w, p, k, mode)
    finally:
        L.lbimp_ctx_set_option(ctx, "pd_prefilter", 0)
    assert torch.equal(idx, ri) and torch.equal(dist, rd)
    check_knn(X, Ys, w, p, k, idx.cpu().numpy(), dist.cpu().numpy(), f"pd {mode} p={p} k={k}")
    check_stats(X, Ys, w, p, st, mode, pd=True, pd_parts=fine_parts(pd, mode, n, w))
    assert st[:, 6].sum() > 0
    db.close()


@pytest.mark.parametrize("n,w", [(20, 3), (64, 6), (128, 13), (256, 26), (300, 45), (512, 51), (200, 63)])
@pytest.mark.parametrize("p,k", [(1, 1), (2, 3), (INF, 2)])
@pytest.mark.parametrize("slots,pd", [(1 << 18, 0), (64, 0), (1 << 18, 2)])
def test_nn_search_dtw_split(L, ctx, n, w, p, k, slots, pd):
    """The survivors' DTW in two row phases (pairs still running at half the series parked and
    repacked): the same answers, bit for bit, as one phase, matching the oracle; a pool of 64
    slots overflows, and the pairs without a slot finish in the first phase."""
    _say(f"nn_search dtw_split n={n} w={w} p={p} k={k} slots={slots} pd={pd}")
    X = walks(3000, n, 60)
    Ys = walks(9, n, 61)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    L.lbimp_ctx_set_option(ctx, "pd_prefilter", pd)
    try:
        ri, rd, _ = L.lbimp_nn_search(ctx, db, Yd, w, p, k, "improved")
        L.lbimp_ctx_set_option(ctx, "dtw_split", 1)
        L.lbimp_ctx_set_option(ctx, "dtw_pool_slots", slots)
        idx, dist, st = L.lbimp_nn_search(ctx, db, Yd, w, p, k, "improved")
    finally:
        L.lbimp_ctx_set_option(ctx, "dtw_split", 0)
        L.lbimp_ctx_set_option(ctx, "dtw_pool_slots", 1 << 18)
        L.lbimp_ctx_set_option(ctx, "pd_prefilter", 0)
    assert torch.equal(idx, ri) and torch.equal(dist, rd)
    check_knn(X, Ys[:4], w, p, k, idx.cpu().numpy()[:4], dist.cpu().numpy()[:4], f"split n={n} w={w} p={p}")
    check_stats(X, Ys, w, p, st, "improved", pd=bool(pd), pd_parts=fine_parts(pd, "improved", n, w))
    db.close()


def test_nn_search_dtw_split_chunked(L, ctx):
    """Row phases in every chunk of a bounded workspace (the pool capped by the bound)."""
    X = walks(9_000, 64, 62)
    Ys = walks(6, 64, 63)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    ri, rd, _ = L.lbimp_nn_search(ctx, db, Yd, 6, 1, 2, "improved")
    small = L.Ctx(0)
    try:
        L.lbimp_ctx_set_option(small, "dtw_split", 1)
        L.lbimp_ctx_set_option(small, "workspace_limit", 400_000)
        idx, dist, st = L.lbimp_nn_search(small, db, Yd, 6, 1, 2, "improved")
        torch.cuda.synchronize()
    finally:
        small.close()
    assert torch.equal(idx, ri) and torch.equal(dist, rd)
    check_knn(X, Ys, 6, 1, 2, idx.cpu().numpy(), dist.cpu().numpy(), "split chunked")
    db.close()


@pytest.mark.parametrize("n,w", [(128, 13), (256, 26), (300, 80), (512, 102), (2300, 600)])
@pytest.mark.parametrize("p,k", [(1, 1), (2, 3), (INF, 1)])
def test_nn_search_lbi_abandon(L, ctx, n, w, p, k):
    """Early abandoning inside LB_Improved (register, wave-per-pair and generic kernels) changes
    neither the answers nor any pruning count: a pair is abandoned only once its growing bound
    has reached the threshold it would have reached anyway."""
    _say(f"nn_search lbi_abandon n={n} w={w} p={p} k={k}")
    X = walks(3000 if n < 1000 else 300, n, 36)
    Ys = walks(9, n, 37)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    ri, rd, rst = L.lbimp_nn_search(ctx, db, Yd, w, p, k, "improved")
    L.lbimp_ctx_set_option(ctx, "lbi_abandon", 1)
    try:
        idx, dist, st = L.lbimp_nn_search(ctx, db, Yd, w, p, k, "improved")
    finally:
        L.lbimp_ctx_set_option(ctx, "lbi_abandon", 0)
    assert torch.equal(idx, ri) and torch.equal(dist, rd)
    assert np.array_equal(st[:, :5], rst[:, :5]) and np.array_equal(st[:, 6], rst[:, 6])
    check_knn(X, Ys[:3], w, p, k, idx.cpu().numpy()[:3], dist.cpu().numpy()[:3], f"lbi_abandon n={n} w={w}")
    db.close()


@pytest.mark.parametrize("n,w,N", [(128, 13, 9000), (256, 26, 9000), (64, 6, 20000), (300, 80, 9000), (512, 51, 9000),
                                   (2300, 600, 4200)])
@pytest.mark.parametrize("p,k", [(1, 1), (2, 3), (INF, 2)])
@pytest.mark.parametrize("pd", [0, 2])
def test_nn_search_lbi_buckets(L, ctx, n, w, N, p, k, pd):
    """LB_Improved over survivor lists bucketed by candidate range (walked bucket by bucket, one
    XCD per bucket), after the LB_Keogh sweep (pd 0) or fused with LB_Keogh after pass 0 on the
    32-part cover (pd 2, where the shape allows it): the same pairs are bounded, so answers and
    every pruning count equal those of the plain lists, bit for bit; the database spans several
    buckets of each shape."""
    _say(f"nn_search lbi_buckets n={n} w={w} N={N} p={p} k={k} pd={pd}")
    X = walks(N, n, 38)
    Ys = walks(11, n, 39)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    L.lbimp_ctx_set_option(ctx, "pd_prefilter", pd)
    try:
        ri, rd, rst = L.lbimp_nn_search(ctx, db, Yd, w, p, k, "improved")
        L.lbimp_ctx_set_option(ctx, "lbi_buckets", 1)
        idx, dist, st = L.lbimp_nn_search(ctx, db, Yd, w, p, k, "improved")
    finally:
        L.lbimp_ctx_set_option(ctx, "lbi_buckets", 0)
        L.lbimp_ctx_set_option(ctx, "pd_prefilter", 0)
    assert torch.equal(idx, ri) and torch.equal(dist, rd)
    assert np.array_equal(st[:, :5], rst[:, :5]) and np.array_equal(st[:, 6], rst[:, 6])
    m = 3 if n <= 512 else 0  # the wide case is checked against the plain lists only
    if m:
        check_knn(X, Ys[:m], w, p, k, idx.cpu().numpy()[:m], dist.cpu().numpy()[:m], f"lbi_buckets n={n} w={w}")
    db.close()


@pytest.mark.parametrize("depth", [0])
@pytest.mark.parametrize("n,w", [(128, 13), (256, 26), (200, 31), (300, 40)])
def test_nn_search_lbi_pipeline_depth(L, ctx, depth, n, w):
    """The register LB_Improved kernel with rows staged in batches instead of loaded a block
    ahead (the default): identical answers and counts."""
    _say(f"nn_search lbi_pipeline={depth} n={n} w={w}")
    X = walks(4000, n, 40)
    Ys = walks(9, n, 41)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    ri, rd, rst = L.lbimp_nn_search(ctx, db, Yd, w, 1, 2, "improved")
    L.lbimp_ctx_set_option(ctx, "lbi_pipeline", depth)
    try:
        idx, dist, st = L.lbimp_nn_search(ctx, db, Yd, w, 1, 2, "improved")
    finally:
        L.lbimp_ctx_set_option(ctx, "lbi_pipeline", 1)
    assert torch.equal(idx, ri) and torch.equal(dist, rd)
    assert np.array_equal(st[:, :5], rst[:, :5])
    check_knn(X, Ys[:2], w, 1, 2, idx.cpu().numpy()[:2], dist.cpu().numpy()[:2], f"lbi_pipeline={depth}")
    db.close()


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
@pytest.mark.parametrize("p,k", [(1, 1), (2, 5), (INF, 3)])
@pytest.mark.parametrize("pd", [0, 1, 2])
def test_nn_search_chunked(L, ctx, mode, p, k, pd):
    """A workspace bound splits the database into chunks of candidates searched one after another
    (the threshold carried across): the answers equal the unchunked search's, bit for bit, and the
    oracle's; the workspace stays under the bound; counts keep their invariants."""
    if pd and mode == "brute":
        pytest.skip("pass 0 does not apply to brute force")
    _say(f"nn_search chunked mode={mode} p={p} k={k} pd={pd}")
    X = walks(9_000, 64, 38)  # chunks of 2048 or 4096 candidates, the last one shorter
    Ys = walks(6, 64, 39)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    L.lbimp_ctx_set_option(ctx, "pd_prefilter", pd)
    try:
        ri, rd, _ = L.lbimp_nn_search(ctx, db, Yd, 6, p, k, mode)
        small = L.Ctx(0)
        L.lbimp_ctx_set_option(small, "pd_prefilter", pd)
        L.lbimp_ctx_set_option(small, "workspace_limit", 400_000)
        idx, dist, st = L.lbimp_nn_search(small, db, Yd, 6, p, k, mode)
        torch.cuda.synchronize()
        assert L.lbimp_ctx_workspace_bytes(small) <= 2 << 20  # reserve rounds up to whole MiB
        small.close()
    finally:
        L.lbimp_ctx_set_option(ctx, "pd_prefilter", 0)
    assert torch.equal(idx, ri) and torch.equal(dist, rd)
    check_knn(X, Ys, 6, p, k, idx.cpu().numpy(), dist.cpu().numpy(), f"chunked {mode} p={p} k={k}")
    check_stats(X, Ys, 6, p, st, mode, pd=bool(pd), pd_parts=fine_parts(pd, mode, 64, 6))
    if mode != "brute":
        assert np.all(st[:, 1] > 32)  # seeds drawn in every chunk: several chunks ran
    db.close()


# ------------------------------------------------------------------ nearest-neighbour search
def oracle_knn(X, Ys, w, p, k):
    idx, dist = native.nn_bruteforce(X, Ys, R.effective_band(X.shape[1], w), p, k)
    return idx, dist


def check_knn(X, Ys, w, p, k, gidx, gdist, what):
    n = X.shape[1]
    wb = R.effective_band(n, w)
    for q in range(Ys.shape[0]):
        D = native.dtw_pow_many(X, Ys[q], wb, p)
        order = R.key_order(D)
        want = order[:k]
        kk = min(k, X.shape[0])
        scale = lp_scale(X, Ys[q], p)
        assert np.all(gidx[q, kk:] == -1) and np.all(np.isinf(gdist[q, kk:]))
        for r in range(kk):
            c = int(gidx[q, r])
            dmin = float(rt(D[want[r]], p))
            if c != want[r]:
                assert 0 <= c < X.shape[0], (what, q, r, c)
                dc = float(rt(D[c], p))
                assert dc <= dmin + RTOL * max(dmin, 1e-3 * scale[c]), (what, q, r, c, int(want[r]), dc, dmin)
            assert abs(gdist[q, r] - dmin) <= RTOL * max(dmin, 1e-3 * scale[want[r]]) + 1e-30, (what, q, r)
        assert len(set(gidx[q, :kk].tolist())) == kk


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def check_golden(name, X, Ys, w, p, gidx, gdist):
    """Every query's 1-NN against the oracle's, stored by tests/golden/make_full_size.py (brute
    force over the whole database in fp64).  The index must equal the oracle's unless the
    device's pick is a tie within the tolerance (its oracle distance is recomputed); the
    distance must match the oracle's minimum.  Returns the relative errors of the distances."""
    path = os.path.join(GOLDEN, f"{name}_nn.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet: run tests/golden/make_full_size.py {name}")
    rows = np.loadtxt(path, comments="#", dtype=np.float64, ndmin=2)
    assert rows.shape[0] == Ys.shape[0] and np.array_equal(rows[:, 0], np.arange(Ys.shape[0]))
    oi, od = rows[:, 1].astype(np.int64), rows[:, 2]
    X64, Y64 = np.asarray(X, np.float64), np.asarray(Ys, np.float64)
    rel = np.empty(Ys.shape[0])
    ties = 0
    for q in range(Ys.shape[0]):
        dmin = float(rt(od[q], p))
        scale = float(lp_scale(X64[oi[q]][None, :], Y64[q], p)[0])
        c = int(gidx[q])
        if c != oi[q]:
            assert 0 <= c < X.shape[0], (name, q, c)
            dc = float(rt(native.dtw_pow(X64[c], Y64[q], w, p), p))
            sc = float(lp_scale(X64[c][None, :], Y64[q], p)[0])
            assert dc <= dmin + RTOL * max(dmin, 1e-3 * sc), (name, q, c, int(oi[q]), dc, dmin)
            ties += 1
        err = abs(float(gdist[q]) - dmin)
        assert err <= RTOL * max(dmin, 1e-3 * scale) + 1e-30, (name, q, float(gdist[q]), dmin)
        rel[q] = err / max(dmin, 1e-30)
    _say(f"  {name}: {Ys.shape[0]} queries against the oracle, {ties} ties, relative error "
         f"max {rel.max():.3g} median {np.median(rel):.3g}")
    return rel


def check_stats(X, Ys, w, p, st, mode, pd=False, pd_parts=8):
    """Counts relative to the exact final threshold b*: the device threshold is never below b*,
    so it prunes no candidate whose bound is below b* (up to float32 rounding).  The bounds are
    nested (P_d <= LB_Keogh <= LB_Improved), so each pass's cumulative count is checked against
    its own bound."""
    N, n = X.shape
    wb = R.effective_band(n, w)
    for q in range(Ys.shape[0]):
        cand, seeded, pk, pi, started, aband, ppd = st[q]
        assert cand == N
        assert seeded + ppd + pk + pi + (started - seeded) == N
        assert 0 <= aband <= started
        if mode == "brute":
            assert started == N and pk == pi == ppd == 0
            continue
        if not pd:
            assert ppd == 0
        D = native.dtw_pow_many(X, Ys[q], wb, p)
        s1, s2 = native.lb_many(X, Ys[q], wb, p)
        bstar = D.min()
        slack = 1 + 1e-4
        if pd:
            U, Lo = R.envelope_naive(Ys[q], wb)
            b0 = R.pd_bound_pow_many(X, U, Lo, p, d=pd_parts)
            assert ppd <= np.sum(b0 * slack >= bstar)
        assert ppd + pk <= np.sum(s1 * slack >= bstar)
        assert ppd + pk + pi <= np.sum(s2 * slack >= bstar)
        if mode == "keogh":
            assert pi == 0


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
@pytest.mark.parametrize("p", [1, 2, INF])
@pytest.mark.parametrize("k", [1, 5])
def test_nn_search_small_random_walk(L, ctx, mode, p, k):
    _say(f"nn_search rw128_small mode={mode} p={p} k={k}")
    db64, qs64 = gen.make_workload("rw128_small")
    X, Ys = f32(db64).astype(np.float64), f32(qs64).astype(np.float64)
    db = L.Db(ctx, to_dev(X))
    idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), 13, p, k, mode)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    check_knn(X, Ys, 13, p, k, idx, dist, f"{mode} p={p} k={k}")
    check_stats(X, Ys, 13, p, st, mode)
    if k == 1:
        # On the raw float64 data (before the float32 rounding the device sees) every query's
        # pick is the oracle's nearest neighbour, or within 1e-4 of its distance: rounding the
        # inputs moves each DTW by far less than that.
        for q in range(qs64.shape[0]):
            D = rt(native.dtw_pow_many(db64, qs64[q], 13, p), p)
            assert D[idx[q, 0]] <= D.min() * (1 + 1e-4), (q, int(idx[q, 0]), int(np.argmin(D)))
    db.close()


EDGE_CASES = {
    "N1": dict(N=1, n=16, w=2),
    "N65": dict(N=65, n=33, w=4),
    "n1": dict(N=50, n=1, w=0),
    "n2": dict(N=50, n=2, w=5),
    "w0": dict(N=300, n=40, w=0),
    "w_ge_n": dict(N=100, n=30, w=30),
    "wide_wave_path": dict(N=150, n=256, w=80),
    "ragged_n": dict(N=200, n=131, w=13),
    "long_wide": dict(N=80, n=2300, w=600),  # generic LB_Improved, strip DTW, LDS seeding DTW
}


@pytest.mark.parametrize("case", sorted(EDGE_CASES))
@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
def test_nn_search_edge_cases(L, ctx, case, mode):
    cfg = EDGE_CASES[case]
    _say(f"nn_search edge {case} mode={mode}")
    X = walks(cfg["N"], cfg["n"], 11)
    Ys = walks(5, cfg["n"], 12)
    db = L.Db(ctx, to_dev(X))
    for p, k in ((1, 1), (2, 3), (INF, 2)):
        idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), cfg["w"], p, k, mode)
        check_knn(X, Ys, cfg["w"], p, k, idx.cpu().numpy(), dist.cpu().numpy(), f"{case} {mode} p={p} k={k}")
        check_stats(X, Ys, cfg["w"], p, st, mode)
    db.close()


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
def test_nn_search_many_queries(L, ctx, mode):
    """2600 queries in one call: the work-item prefix over queries spans three 1024-query chunks."""
    _say(f"nn_search many queries Q=2600 mode={mode}")
    X = walks(500, 32, 44)
    Ys = walks(2600, 32, 45)
    db = L.Db(ctx, to_dev(X))
    for p, k in ((1, 1), (2, 3)):
        idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), 3, p, k, mode)
        check_knn(X, Ys, 3, p, k, idx.cpu().numpy(), dist.cpu().numpy(), f"Q2600 {mode} p={p} k={k}")
        check_stats(X, Ys, 3, p, st, mode)
    db.close()


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
def test_nn_search_ties_constant_and_negative(L, ctx, mode):
    _say(f"nn_search ties mode={mode}")
    g = np.random.default_rng(21)
    n = 48
    X = f32(np.cumsum(g.standard_normal((90, n)), axis=1) - 5.0).astype(np.float64)
    X[40] = X[7]          # exact duplicates: the smaller index must win
    X[77] = X[7]
    X[12] = -3.0          # constant series
    X[13] = -3.0
    Ys = np.stack([X[7], X[12], f32(X[30] + 0.25).astype(np.float64)])
    db = L.Db(ctx, to_dev(X))
    idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), 5, 1, 3, mode)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    assert list(idx[0]) == [7, 40, 77] and np.all(dist[0] == 0)
    assert list(idx[1][:2]) == [12, 13]
    check_knn(X, Ys, 5, 1, 3, idx, dist, f"ties {mode}")
    db.close()


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
@pytest.mark.parametrize("n,w", [(96, 9), (200, 80)])
@pytest.mark.parametrize("k", [10, 64])
def test_nn_search_large_k(L, ctx, mode, n, w, k):
    """k up to the maximum of 64 (the k-th best key as the threshold, sorted output), in the
    lane-per-pair and the strip DTW paths, against the oracle."""
    _say(f"nn_search large k={k} n={n} w={w} mode={mode}")
    X = walks(1500, n, 41)
    Ys = walks(6, n, 42)
    db = L.Db(ctx, to_dev(X))
    for p in (1, 2, INF):
        idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), w, p, k, mode)
        idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
        check_knn(X, Ys, w, p, k, idx, dist, f"large k={k} {mode} p={p}")
        assert np.all(np.diff(dist, axis=1) >= 0)
        check_stats(X, Ys, w, p, st, mode)
    db.close()


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
def test_nn_search_k64_ties_in_index_order(L, ctx, mode):
    """Seventy exact copies of one series: the 64 nearest neighbours of that series are the 64
    smallest indices among the copies, in index order, all at distance 0."""
    _say(f"nn_search k=64 ties mode={mode}")
    X = walks(400, 64, 43)
    copies = np.sort(np.random.default_rng(44).choice(400, 70, replace=False))
    X[copies] = X[copies[0]]
    db = L.Db(ctx, to_dev(X))
    idx, dist, _ = L.lbimp_nn_search(ctx, db, to_dev(X[copies[:1]]), 6, 1, 64, mode)
    assert list(idx.cpu().numpy()[0]) == list(copies[:64])
    assert np.all(dist.cpu().numpy()[0] == 0)
    db.close()


def test_nn_search_empty_database_and_k_above_n(L, ctx):
    _say("nn_search empty database, k > N")
    Ys = walks(3, 20, 13)
    db = L.Db(ctx, torch.empty((0, 20), dtype=torch.float32, device="cuda"))
    idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), 2, 1, 2, "improved")
    assert np.all(idx.cpu().numpy() == -1) and np.all(np.isinf(dist.cpu().numpy()))
    db.close()
    X = walks(3, 20, 14)
    db = L.Db(ctx, to_dev(X))
    for mode in ("brute", "keogh", "improved"):
        idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), 2, 1, 5, mode)
        check_knn(X, Ys, 2, 1, 5, idx.cpu().numpy(), dist.cpu().numpy(), f"k>N {mode}")
    db.close()


def test_invalid_arguments_return_status(L, ctx):
    _say("invalid arguments")
    X = to_dev(walks(10, 16, 15))
    y = to_dev(walks(1, 16, 16)[0])
    with pytest.raises(L.LbimpError) as e:
        L.lbimp_dtw_band(ctx, X, y, -1, 1)
    assert e.value.code == L.LBIMP_E_INVALID
    with pytest.raises(L.LbimpError) as e:
        L.lbimp_dtw_band(ctx, X, y, 2, 3)
    assert e.value.code == L.LBIMP_E_UNSUPPORTED
    db = L.Db(ctx, X)
    with pytest.raises(L.LbimpError) as e:
        L.lbimp_nn_search(ctx, db, to_dev(walks(2, 16, 17)), 2, 1, 65, "improved")
    assert e.value.code == L.LBIMP_E_INVALID
    db.close()


@pytest.mark.parametrize("p", [1, 2])
def test_nn_search_rw256_full_size(L, ctx, p):
    """The benchmarked workload (100,000 x 256 random walks, 256 queries, w = 26) in the launch
    configuration the benchmark times: every query of every mode against the oracle's brute force,
    and the three modes bit-equal."""
    _say(f"nn_search rw256 full size p={p}")
    db64, qs64 = gen.make_workload("rw256")
    X, Ys = f32(db64), f32(qs64)
    db = L.Db(ctx, to_dev(X))
    Yd = to_dev(Ys)
    res = {}
    for mode in ("improved", "keogh", "brute"):
        _say(f"  mode {mode}")
        res[mode] = L.lbimp_nn_search(ctx, db, Yd, 26, p, 1, mode)
    idx = {m: r[0].cpu().numpy()[:, 0] for m, r in res.items()}
    dist = {m: r[1].cpu().numpy()[:, 0] for m, r in res.items()}
    assert np.array_equal(idx["improved"], idx["keogh"])
    assert np.array_equal(idx["improved"], idx["brute"])
    assert np.allclose(dist["improved"], dist["brute"], rtol=0, atol=0)
    for mode in ("improved", "keogh", "brute"):
        check_golden(f"rw256_p{p}", X, Ys, 26, p, idx[mode], dist[mode])
    st = res["improved"][2]
    assert np.all(st[:, 0] == 100_000)
    # the second pass prunes something on this workload (the point of the method)
    assert st[:, 3].sum() > 0 and st[:, 4].mean() < 0.05 * 100_000
    db.close()


@pytest.fixture(scope="module")
def shape512(L, ctx):
    db64, qs64 = gen.make_workload("shape512")
    X, Ys = f32(db64), f32(qs64)
    db = L.Db(ctx, to_dev(X))
    yield X, Ys, db
    torch.cuda.synchronize()
    db.close()


@pytest.mark.parametrize("w", [26, 51])
def test_nn_search_shape512_full_size(L, ctx, shape512, w):
    """Shape-like signatures (50,000 x 512, 512 queries, w = 26 and 51, p = 1): the three modes
    agree on every query, bit for bit, and every query matches the oracle's brute force."""
    _say(f"nn_search shape512 full size w={w}")
    X, Ys, db = shape512
    Yd = to_dev(Ys)
    res = {m: L.lbimp_nn_search(ctx, db, Yd, w, 1, 1, m) for m in ("improved", "keogh", "brute")}
    idx = {m: r[0].cpu().numpy()[:, 0] for m, r in res.items()}
    dist = {m: r[1].cpu().numpy()[:, 0] for m, r in res.items()}
    assert np.array_equal(idx["improved"], idx["keogh"]) and np.array_equal(idx["improved"], idx["brute"])
    assert np.array_equal(dist["improved"].view(np.uint32), dist["brute"].view(np.uint32))
    for mode in ("improved", "keogh", "brute"):
        check_golden(f"shape512_w{w}", X, Ys, w, 1, idx[mode], dist[mode])
    st = res["improved"][2]
    assert np.all(st[:, 0] == 50_000)
    assert st[:, 3].sum() > 0  # LB_Improved prunes past LB_Keogh


@pytest.mark.parametrize("shape", [2, 3, 4, 5])
def test_nn_search_sweep_shapes(L, ctx, shape):
    _say(f"nn_search sweep shape {shape}")
    X = walks(20_000, 64, 22)
    Ys = walks(37, 64, 23)
    db = L.Db(ctx, to_dev(X))
    L.lbimp_ctx_set_option(ctx, "sweep_shape", shape)
    try:
        idx, dist, st = L.lbimp_nn_search(ctx, db, to_dev(Ys), 6, 1, 1, "improved")
    finally:
        L.lbimp_ctx_set_option(ctx, "sweep_shape", 0)
    check_knn(X, Ys[:8], 6, 1, 1, idx.cpu().numpy()[:8], dist.cpu().numpy()[:8], f"shape {shape}")
    db.close()


def test_nn_search_counts_are_deterministic(L, ctx):
    _say("determinism of results and pruning counts")
    X = walks(3000, 64, 18)
    Ys = walks(20, 64, 19)
    db = L.Db(ctx, to_dev(X))
    a = L.lbimp_nn_search(ctx, db, to_dev(Ys), 6, 1, 1, "improved")
    b = L.lbimp_nn_search(ctx, db, to_dev(Ys), 6, 1, 1, "improved")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert np.array_equal(a[2][:, :5], b[2][:, :5])
    db.close()
