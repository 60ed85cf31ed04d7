"""GPU serving loop: continuous batching under a Poisson load.

The same request has the same answer alone and in the mix: every served result is compared,
bit for bit, with lbimp_nn_search on that one query, and spot-checked against the fp64
oracle.  A tight memory budget (smaller batches, fewer concurrent slots) must not change
any answer either.
"""
import numpy as np
import pytest
import torch

from paper_0811_3301_amd import gen
from paper_0811_3301_amd.serve import GpuExecutor, Request, serve
from tests.test_gpu_parity import L, ctx, _say, check_knn, f32, to_dev  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def workload(L, ctx):
    dbs64, req = gen.make_serving_workload(20_000, 600, N_main=8_000, N_side=2_000)
    Xs = [f32(d).astype(np.float64) for d in dbs64]
    handles = [L.Db(ctx, to_dev(X)) for X in Xs]
    reqs = [Request(rid=i, t_arrive=float(req["t"][i]), db=int(req["db"][i]), y=f32(req["y"][i]),
                    w=int(req["w"][i]), k=int(req["k"][i])) for i in range(len(req["t"]))]
    yield Xs, handles, reqs
    torch.cuda.synchronize()
    for h in handles:
        h.close()


def _alone(L, ctx, handles, r):
    i, d, _ = L.lbimp_nn_search(ctx, handles[r.db], to_dev(r.y[None, :]), r.w, 1, r.k, "improved", stats=False)
    return i.cpu().numpy()[0], d.cpu().numpy()[0]


def _run(L, handles, reqs, budget, slots, max_batch, bound=False):
    ex = GpuExecutor(handles, slots=slots, max_batch=max_batch, kmax=10,
                     workspace_limit=budget // slots if bound else 0)
    try:
        results, summary = serve(reqs, ex, budget_bytes=budget, max_batch=max_batch)
    finally:
        ex.close()
    return {r.rid: r for r in results}, summary


@pytest.mark.parametrize("budget,slots,max_batch,bound", [(8 << 30, 4, 256, False), (24 << 20, 3, 64, False),
                                                           (6 << 20, 3, 128, True)])
def test_serving_results_equal_alone(L, ctx, workload, budget, slots, max_batch, bound):
    """With bound, each slot's workspace is limited to its share of the budget, so batches larger
    than that search their databases in chunks of candidates."""
    _say(f"serving 600 requests at 20k q/s, budget {budget >> 20} MiB, {slots} slots, batch <= {max_batch}, "
         f"workspace bound {bound}")
    Xs, handles, reqs = workload
    got, summary = _run(L, handles, reqs, budget, slots, max_batch, bound)
    assert len(got) == len(reqs)
    assert summary["count"] == len(reqs) and summary["p99_ms"] >= summary["p50_ms"] > 0
    assert summary["workspace_bytes"] <= budget
    for r in reqs:
        res = got[r.rid]
        ai, ad = _alone(L, ctx, handles, r)
        assert res.idx.shape == (r.k,)
        assert np.array_equal(res.idx, ai), (r.rid, res.idx, ai)
        assert np.array_equal(res.dist.view(np.uint32), ad.view(np.uint32)), (r.rid, res.dist, ad)
        assert res.t_done >= res.t_admit >= res.t_arrive
    for r in reqs[::60]:  # spot checks against the oracle
        res = got[r.rid]
        check_knn(Xs[r.db], r.y.astype(np.float64)[None, :], r.w, 1, r.k, res.idx[None, :], res.dist[None, :],
                  f"served rid={r.rid}")


def test_serving_batches_overlap_under_load(L, ctx, workload):
    """At a rate well above one batch at a time, requests are admitted while others run:
    several batches share the device and most batches hold more than one request."""
    _say("serving overlap at 200k q/s offered")
    Xs, handles, reqs = workload
    fast = [Request(r.rid, r.t_arrive / 10.0, r.db, r.y, r.w, r.k) for r in reqs]
    got, summary = _run(L, handles, fast, 8 << 30, 4, 128)
    batches = sorted({(got[r.rid].t_admit, got[r.rid].t_done) for r in fast})
    assert len(batches) < len(fast) / 2          # requests were batched together
    admit = np.array([b[0] for b in batches])
    done = np.array([b[1] for b in batches])
    # some batch was admitted before an earlier-admitted batch had finished (overlap)
    assert np.any(admit[1:] < np.maximum.accumulate(done)[:-1])


def test_serving_full_size_sampled(L, ctx):
    """The serving workload the benchmark runs -- a resident 1,000,000 x 128 random-walk database
    (512 MB) and a 200,000 x 256 side database, w = round(0.1 n), k in {1, 5, 10} -- at 20k q/s
    offered, with the benchmark's four slots, batches of at most 512 and a 4 GiB budget (1 GiB of
    workspace per slot, larger batches searched in chunks of candidates), after pretuning: every
    result equals the same query searched alone, bit for bit, and the first request of each
    database matches the oracle."""
    _say("serving full size: 1M x 128 and 200k x 256 databases, 400 requests at 20k q/s")
    dbs64, req = gen.make_serving_workload(20_000, 400)
    Xs = [f32(d) for d in dbs64]
    del dbs64
    handles = [L.Db(ctx, to_dev(X)) for X in Xs]
    reqs = [Request(rid=i, t_arrive=float(req["t"][i]), db=int(req["db"][i]), y=f32(req["y"][i]),
                    w=int(req["w"][i]), k=int(req["k"][i])) for i in range(len(req["t"]))]
    ex = GpuExecutor(handles, slots=4, max_batch=512, kmax=10, workspace_limit=1 << 30)
    try:
        ex.pretune(reqs[:200])
        results, summary = serve(reqs, ex, budget_bytes=4 << 30, max_batch=512)
    finally:
        ex.close()
    try:
        got = {r.rid: r for r in results}
        assert len(got) == len(reqs) and summary["p99_ms"] >= summary["p50_ms"] > 0
        assert summary["workspace_bytes"] <= 4 << 30
        for r in reqs:
            ai, ad = _alone(L, ctx, handles, r)
            assert np.array_equal(got[r.rid].idx, ai), r.rid
            assert np.array_equal(got[r.rid].dist.view(np.uint32), ad.view(np.uint32)), r.rid
        for db in (0, 1):
            r = next(r for r in reqs if r.db == db)
            _say(f"  oracle check db={db} rid={r.rid} k={r.k}")
            res = got[r.rid]
            check_knn(Xs[db].astype(np.float64), r.y.astype(np.float64)[None, :], r.w, 1, r.k, res.idx[None, :],
                      res.dist[None, :], f"served full-size rid={r.rid}")
    finally:
        torch.cuda.synchronize()
        for h in handles:
            h.close()
