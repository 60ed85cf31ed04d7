"""Allocation-free search: lbimp_nn_search_noalloc against lbimp_nn_search.

The variant runs the same kernels on the library's fixed device scratch instead of the
context's workspace.  Its outputs must equal lbimp_nn_search's bit for bit (and hence the
oracle's, to the same tolerance); two calls in a row, the second smaller, check that the
shared scratch left by one call does not leak into the next; a search larger than the scratch
runs in chunks of candidates and one that cannot fit even so is refused before any work is
enqueued; the context's workspace is never touched.
"""
import numpy as np
import pytest
import torch

from paper_0811_3301_amd import gen
from tests.test_gpu_parity import L, _say, check_knn, f32, to_dev  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu


def _walks(count, n, seed):
    return f32(gen.random_walk(count, n, gen.rng(700, 0, seed))).astype(np.float64)


@pytest.mark.parametrize("mode", ["brute", "keogh", "improved"])
def test_noalloc_matches_search_on_two_calls(L, mode):
    _say(f"nn_search_noalloc mode={mode}")
    ctx = L.Ctx(0)
    ref = L.Ctx(0)  # lbimp_nn_search runs on its own context, whose workspace it grows
    X = _walks(20_000, 128, 1)
    db = L.Db(ctx, to_dev(X))
    try:
        # second call smaller than the first, with another p and k
        for step, (Q, w, p, k) in enumerate(((40, 13, 1, 1), (9, 6, 2, 5))):
            _say(f"  call {step}: Q={Q} w={w} p={p} k={k}")
            Y = _walks(Q, 128, 10 + step)
            Yd = to_dev(Y)
            i, d = L.lbimp_nn_search_noalloc(ctx, db, Yd, w, p, k, mode)
            torch.cuda.synchronize()
            assert L.lbimp_ctx_workspace_bytes(ctx) == 0  # the context's workspace was never allocated
            ri, rd, _ = L.lbimp_nn_search(ref, db, Yd, w, p, k, mode, stats=False)
            i, d, ri, rd = i.cpu().numpy(), d.cpu().numpy(), ri.cpu().numpy(), rd.cpu().numpy()
            assert np.array_equal(i, ri)
            assert np.array_equal(d.view(np.uint32), rd.view(np.uint32))
            check_knn(X, Y[:3], w, p, k, i[:3], d[:3], f"noalloc {mode} call {step}")
    finally:
        torch.cuda.synchronize()
        db.close()
        ref.close()
        ctx.close()


def test_noalloc_chunks_a_large_search_and_refuses_what_cannot_fit(L):
    _say("nn_search_noalloc: a search larger than the scratch, then one that cannot fit")
    ctx = L.Ctx(0)
    X = _walks(100_000, 16, 2)
    db = L.Db(ctx, to_dev(X))
    try:
        # about 12 Q N bytes = 120 MB unchunked: searched in chunks of candidates that fit 64 MiB
        Yd = to_dev(_walks(100, 16, 3))
        i, d = L.lbimp_nn_search_noalloc(ctx, db, Yd, 2, 1, 1, "improved")
        ri, rd, _ = L.lbimp_nn_search(ctx, db, Yd, 2, 1, 1, "improved", stats=False)
        assert torch.equal(i, ri) and torch.equal(d, rd)
        # 4,000 queries need 12 x 4000 x 2048 bytes even for the smallest chunk: refused, nothing run
        with pytest.raises(L.LbimpError) as e:
            L.lbimp_nn_search_noalloc(ctx, db, to_dev(_walks(4000, 16, 4)), 2, 1, 1, "improved")
        assert e.value.code == L.LBIMP_E_NOMEM
        # a search that fits still runs afterwards
        i, d = L.lbimp_nn_search_noalloc(ctx, db, Yd[:4], 2, 1, 1, "improved")
        assert torch.equal(i, ri[:4]) and torch.equal(d, rd[:4])
    finally:
        torch.cuda.synchronize()
        db.close()
        ctx.close()
