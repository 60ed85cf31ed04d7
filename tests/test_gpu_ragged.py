"""GPU parity of the ragged batch (lbimp_nn_search_ragged): queries of mixed lengths, bands
and databases in one call, grouped and run concurrently, optionally as a replayed HIP graph.

Each query's answer is checked against the fp64 oracle (same tolerance as the homogeneous
search), and against lbimp_nn_search run alone on the same group of queries, which must
agree bit for bit: batching with other groups changes nothing.  Graph replays are checked
against the eager launches, with other device work between replays, with new query values
in the same buffer and with a regrouping that keeps the graph's shapes.
"""
import numpy as np
import pytest
import torch

from paper_0811_3301_amd import gen
from tests.test_gpu_parity import L, ctx, _say, check_knn, f32, to_dev  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu


def _walks(count, n, seed):
    return f32(gen.random_walk(count, n, gen.rng(600, 0, seed))).astype(np.float64)


def _mix(seed, Q, lengths, bands):
    """Q queries spread over the databases, with per-query bands drawn from bands[length]."""
    r = gen.rng(601, 0, seed)
    db_of = r.integers(0, len(lengths), Q).astype(np.int32)
    w = np.array([bands[lengths[b]][r.integers(0, len(bands[lengths[b]]))] for b in db_of], np.int32)
    Ys = [_walks(1, lengths[b], 1000 * seed + q)[0] for q, b in enumerate(db_of)]
    offsets = np.zeros(Q + 1, np.int64)
    offsets[1:] = np.cumsum([len(y) for y in Ys])
    packed = np.concatenate(Ys) if Q else np.zeros(0)
    return db_of, w, Ys, offsets, packed


LENGTHS = [64, 131, 256]
SIZES = [900, 700, 400]
BANDS = {64: [0, 6, 64], 131: [13, 3], 256: [26, 51]}


@pytest.fixture(scope="module")
def dbs(L, ctx):
    Xs = [_walks(N, n, 7 + i) for i, (N, n) in enumerate(zip(SIZES, LENGTHS))]
    handles = [L.Db(ctx, to_dev(X)) for X in Xs]
    yield Xs, handles
    torch.cuda.synchronize()
    for h in handles:
        h.close()


def _check_against_oracle(Xs, db_of, w, Ys, p, k, idx, dist, what):
    for q, b in enumerate(db_of):
        check_knn(Xs[b], Ys[q][None, :], int(w[q]), p, k, idx[q:q + 1], dist[q:q + 1], f"{what} q={q}")


def _alone(L, ctx, handles, db_of, w, Ys, p, k, mode, n_of):
    """lbimp_nn_search on each group (database, effective band) of the batch, in batch order."""
    Q = len(db_of)
    idx = np.zeros((Q, k), np.int64)
    dist = np.zeros((Q, k), np.float32)
    st = np.zeros((Q, 7), np.int64)
    keys = sorted({(int(b), min(int(wq), n_of[b] - 1)) for b, wq in zip(db_of, w)})
    for b, wb in keys:
        qs = [q for q in range(Q) if db_of[q] == b and min(int(w[q]), n_of[b] - 1) == wb]
        i, d, s = L.lbimp_nn_search(ctx, handles[b], to_dev(np.stack([Ys[q] for q in qs])), wb, p, k, mode)
        idx[qs], dist[qs], st[qs] = i.cpu().numpy(), d.cpu().numpy(), s
    return idx, dist, st


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
@pytest.mark.parametrize("p,k", [(1, 1), (2, 5), (float("inf"), 3)])
@pytest.mark.parametrize("graph,streams", [(0, 4), (1, 4), (0, 0), (1, 1)])
def test_ragged_matches_oracle_and_alone(L, ctx, dbs, mode, p, k, graph, streams):
    _say(f"ragged mix mode={mode} p={p} k={k} graph={graph} streams={streams}")
    Xs, handles = dbs
    db_of, w, Ys, offsets, packed = _mix(1 + min(p, 3) + 3 * k, 37, LENGTHS, BANDS)
    L.lbimp_ctx_set_option(ctx, "graph", graph)
    L.lbimp_ctx_set_option(ctx, "ragged_streams", streams)
    try:
        idx, dist, st = L.lbimp_nn_search_ragged(ctx, handles, to_dev(packed), offsets, db_of, w, p, k, mode)
    finally:
        L.lbimp_ctx_set_option(ctx, "graph", 1)
        L.lbimp_ctx_set_option(ctx, "ragged_streams", 4)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    _check_against_oracle(Xs, db_of, w, Ys, p, k, idx, dist, f"ragged {mode}")
    ai, ad, ast = _alone(L, ctx, handles, db_of, w, Ys, p, k, mode, LENGTHS)
    assert np.array_equal(idx, ai)
    assert np.array_equal(dist.view(np.uint32), ad.view(np.uint32))
    assert np.array_equal(st[:, :5], ast[:, :5])  # abandon counts depend on timing


def test_ragged_graph_replays(L, ctx, dbs):
    """Replays of one captured graph, with eager device work between them: each agrees with
    the eager launches, reads the query values present at launch time, and honours a new
    grouping of equal shapes (the grouping metadata is uploaded outside the graph)."""
    _say("ragged graph replays")
    Xs, handles = dbs
    db_of, w, Ys, offsets, packed = _mix(11, 24, LENGTHS, BANDS)
    buf = to_dev(packed)
    L.lbimp_ctx_set_option(ctx, "graph", 0)
    try:
        ref = L.lbimp_nn_search_ragged(ctx, handles, buf, offsets, db_of, w, 1, 3, "improved")
    finally:
        L.lbimp_ctx_set_option(ctx, "graph", 1)
    ref_i, ref_d = ref[0].cpu().numpy(), ref[1].cpu().numpy()
    out_i = torch.empty((24, 3), dtype=torch.int64, device="cuda")
    out_d = torch.empty((24, 3), dtype=torch.float32, device="cuda")
    for rep in range(4):
        out_i.fill_(-7)
        out_d.fill_(-7.0)
        L.lbimp_nn_search_ragged(ctx, handles, buf, offsets, db_of, w, 1, 3, "improved", idx=out_i, dist=out_d,
                                 stats=False)
        # eager work of the program between replays: another search and torch kernels
        L.lbimp_nn_search(ctx, handles[0], to_dev(_walks(5, 64, 90 + rep)), 6, 2, 1, "keogh", stats=False)
        junk = torch.randn(1 << 16, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        assert np.array_equal(out_i.cpu().numpy(), ref_i), rep
        assert np.array_equal(out_d.cpu().numpy().view(np.uint32), ref_d.view(np.uint32)), rep
        del junk
    # new values in the same query buffer: the replay reads them
    Ys2 = [_walks(1, len(Ys[q]), 5000 + q)[0] for q in range(24)]
    buf.copy_(to_dev(np.concatenate(Ys2)))
    L.lbimp_nn_search_ragged(ctx, handles, buf, offsets, db_of, w, 1, 3, "improved", idx=out_i, dist=out_d,
                             stats=False)
    torch.cuda.synchronize()
    _check_against_oracle(Xs, db_of, w, Ys2, 1, 3, out_i.cpu().numpy(), out_d.cpu().numpy(), "replay new values")
    # reversed query order: each group keeps its size, so the graph is replayed with new metadata
    perm = np.arange(23, -1, -1)
    Ys3 = [Ys2[q] for q in perm]
    off3 = np.zeros(25, np.int64)
    off3[1:] = np.cumsum([len(y) for y in Ys3])
    buf.copy_(to_dev(np.concatenate(Ys3)))
    L.lbimp_nn_search_ragged(ctx, handles, buf, off3, db_of[perm], w[perm], 1, 3, "improved", idx=out_i, dist=out_d,
                             stats=False)
    torch.cuda.synchronize()
    _check_against_oracle(Xs, db_of[perm], w[perm], Ys3, 1, 3, out_i.cpu().numpy(), out_d.cpu().numpy(),
                          "replay regrouped")


def test_ragged_edge_cases(L, ctx, dbs):
    _say("ragged edge cases: empty database, single-query groups, w >= n, k above N")
    Xs, handles = dbs
    empty = L.Db(ctx, torch.zeros((0, 40), dtype=torch.float32, device="cuda"))
    tiny = L.Db(ctx, to_dev(_walks(3, 17, 40)))
    X_tiny = _walks(3, 17, 40)
    all_h = handles + [empty, tiny]
    lengths = LENGTHS + [40, 17]
    Ys = [_walks(1, 64, 41)[0], _walks(1, 40, 42)[0], _walks(1, 17, 43)[0], _walks(1, 131, 44)[0],
          _walks(1, 17, 45)[0]]
    db_of = np.array([0, 3, 4, 1, 4], np.int32)
    w = np.array([100, 5, 16, 0, 2], np.int32)
    offsets = np.zeros(6, np.int64)
    offsets[1:] = np.cumsum([len(y) for y in Ys])
    k = 4
    idx, dist, st = L.lbimp_nn_search_ragged(ctx, all_h, to_dev(np.concatenate(Ys)), offsets, db_of, w, 1, k,
                                             "improved")
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    assert np.all(idx[1] == -1) and np.all(np.isinf(dist[1])) and st[1, 0] == 0
    Xall = Xs + [None, X_tiny]
    for q in (0, 2, 3, 4):
        check_knn(Xall[db_of[q]], Ys[q][None, :], int(w[q]), 1, k, idx[q:q + 1], dist[q:q + 1], f"edge q={q}")
    # zero queries is a no-op
    i0, d0, _ = L.lbimp_nn_search_ragged(ctx, all_h, torch.zeros(0, device="cuda"), np.zeros(1, np.int64),
                                         np.zeros(0, np.int32), 3, 1, 1, "improved")
    assert i0.shape == (0, 1)
    empty.close()
    tiny.close()


def test_ragged_invalid_arguments(L, ctx, dbs):
    _say("ragged invalid arguments")
    _, handles = dbs
    y = to_dev(_walks(1, 64, 50)[0])
    with pytest.raises(L.LbimpError):  # length differs from the database's
        L.lbimp_nn_search_ragged(ctx, handles, y, np.array([0, 64]), np.array([1]), 3, 1, 1, "improved")
    with pytest.raises(L.LbimpError):  # database index out of range
        L.lbimp_nn_search_ragged(ctx, handles, y, np.array([0, 64]), np.array([3]), 3, 1, 1, "improved")
    with pytest.raises(L.LbimpError):  # negative band
        L.lbimp_nn_search_ragged(ctx, handles, y, np.array([0, 64]), np.array([0]), -1, 1, 1, "improved")
    with pytest.raises(L.LbimpError):  # k out of range
        L.lbimp_nn_search_ragged(ctx, handles, y, np.array([0, 64]), np.array([0]), 3, 1, 65, "improved")


def test_ragged_uneven4096_full_size(L):
    """The uneven batch the benchmark times -- 4,096 random-walk queries, n uniform over
    {64, 128, 256, 512, 1024}, w = round(f n) with f in {0.05, 0.1, 0.2}, 20,000 series per
    length, p = 1, 1-NN -- in its launch configuration (every group autotuned on its own before
    the batch, graph replay on four streams): every query equals the search of its group alone, bit for bit, and the first query
    of every (length, band) group matches the oracle."""
    _say("ragged uneven batch, full size (4096 queries, 5 x 20000 series)")
    from paper_0811_3301_amd.serve import pretune_ragged
    ctx2 = L.Ctx(0)
    dbs64, qs, db_of, w = gen.make_ragged_workload()
    Xs = [f32(d) for d in dbs64]
    del dbs64
    handles = [L.Db(ctx2, to_dev(X)) for X in Xs]
    try:
        assert pretune_ragged(L, ctx2, handles, [f32(q) for q in qs], db_of, w, 1, 1, "improved") == 15
        offsets = np.zeros(len(qs) + 1, np.int64)
        offsets[1:] = np.cumsum([len(y) for y in qs])
        packed = to_dev(f32(np.concatenate(qs)))
        L.lbimp_nn_search_ragged(ctx2, handles, packed, offsets, db_of, w, 1, 1, "improved")  # captures
        idx, dist, st = L.lbimp_nn_search_ragged(ctx2, handles, packed, offsets, db_of, w, 1, 1, "improved")
        idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
        Ys = [f32(y) for y in qs]
        ai, ad, ast = _alone(L, ctx2, handles, db_of, w, Ys, 1, 1, "improved", list(gen.RAGGED_LENGTHS))
        assert np.array_equal(idx, ai)
        assert np.array_equal(dist.view(np.uint32), ad.view(np.uint32))
        assert np.array_equal(st[:, :5], ast[:, :5])
        assert np.all(st[:, 0] == 20_000)
        groups = sorted({(int(b), int(wq)) for b, wq in zip(db_of, w)})
        assert len(groups) == 15
        for b, wq in groups:
            q = next(q for q in range(len(qs)) if db_of[q] == b and w[q] == wq)
            _say(f"  oracle check n={gen.RAGGED_LENGTHS[b]} w={wq} q={q}")
            check_knn(Xs[b].astype(np.float64), Ys[q].astype(np.float64)[None, :], wq, 1, 1, idx[q:q + 1],
                      dist[q:q + 1], f"uneven4096 q={q}")
    finally:
        torch.cuda.synchronize()
        for h in handles:
            h.close()
        ctx2.close()


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
@pytest.mark.parametrize("p", [1, 2])
def test_ragged_per_query_k(L, ctx, dbs, mode, p):
    """k chosen per query (1, 3, 5 or 10) in one ragged call: row q holds query q's own k nearest
    neighbours, then -1 / +inf up to the largest k; each row equals lbimp_nn_search of that query
    alone with its own k, bit for bit, and matches the oracle.  One group has a single k, the
    others mix them."""
    _say(f"ragged per-query k mode={mode} p={p}")
    Xs, handles = dbs
    db_of, w, Ys, offsets, packed = _mix(50 + p, 41, LENGTHS, BANDS)
    kq = gen.rng(602, 0, p).choice(np.array([1, 3, 5, 10], np.int32), len(db_of))
    kq[db_of == 2] = 3  # the 256-length groups share one k
    idx, dist, st = L.lbimp_nn_search_ragged(ctx, handles, to_dev(packed), offsets, db_of, w, p, kq, mode)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    assert idx.shape == (len(db_of), int(kq.max()))
    for q, b in enumerate(db_of):
        k = int(kq[q])
        check_knn(Xs[b], Ys[q][None, :], int(w[q]), p, k, idx[q:q + 1], dist[q:q + 1], f"per-query k q={q} k={k}")
        ai, ad, _ = L.lbimp_nn_search(ctx, handles[b], to_dev(Ys[q][None, :]), int(w[q]), p, k, mode, stats=False)
        assert np.array_equal(idx[q, :k], ai.cpu().numpy()[0]), q
        assert np.array_equal(dist[q, :k].view(np.uint32), ad.cpu().numpy()[0].view(np.uint32)), q
        assert np.all(idx[q, k:] == -1) and np.all(np.isinf(dist[q, k:]))
