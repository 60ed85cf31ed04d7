"""Scheduling policy of the serving loop (no GPU): FIFO admission into free slots under a
device-memory budget, batch cutting, and the arrival stream of the serving workload."""
import numpy as np
import pytest

from paper_0811_3301_amd import gen
from paper_0811_3301_amd.serve import MemoryBudget, Request, Result, Scheduler, latency_summary


def _reqs(count, t=0.0):
    return [Request(rid=i, t_arrive=t + i * 1e-3, db=i % 2, y=np.zeros(4, np.float32), w=1, k=1) for i in range(count)]


def test_budget_counts_growth_only():
    b = MemoryBudget(100, 3)
    b.commit(0, 40)
    b.commit(1, 30)
    assert b.fits(2, 30) and not b.fits(2, 31)
    assert b.fits(0, 70) and not b.fits(0, 71)  # slot 0 reuses its own 40
    b.commit(0, 10)                             # workspaces never shrink
    assert b.held[0] == 40


def test_fifo_prefix_and_max_batch():
    b = MemoryBudget(10**9, 2)
    s = Scheduler(b, max_batch=3, need=lambda reqs: 10 * len(reqs))
    for r in _reqs(5):
        s.arrive(r)
    slot, reqs, need = s.take([0, 1])
    assert [r.rid for r in reqs] == [0, 1, 2] and need == 30
    slot, reqs, _ = s.take([1])
    assert slot == 1 and [r.rid for r in reqs] == [3, 4]
    assert s.take([0, 1]) is None


def test_batch_is_cut_to_fit_memory():
    b = MemoryBudget(100, 2)
    b.commit(1, 60)
    s = Scheduler(b, max_batch=8, need=lambda reqs: 15 * len(reqs))
    for r in _reqs(8):
        s.arrive(r)
    # slot 1 (holding 60) is tried first: 0 + max(60, 15c) <= 100 -> c = 4 (halving 8 -> 4)
    slot, reqs, need = s.take([0, 1])
    assert slot == 1 and len(reqs) == 4 and need == 60
    # slot 0 next to slot 1's 60: 60 + 15c <= 100 -> c = 2
    slot, reqs, need = s.take([0])
    assert slot == 0 and [r.rid for r in reqs] == [4, 5]


def test_request_that_fits_nowhere_waits():
    b = MemoryBudget(100, 2)
    b.commit(0, 90)
    s = Scheduler(b, max_batch=4, need=lambda reqs: 50)
    s.arrive(_reqs(1)[0])
    assert s.take([1]) is None          # slot 1: 90 + 50 > 100
    assert s.take([0, 1])[0] == 0       # slot 0 reuses its 90
    assert not s.pending


def test_latency_summary():
    res = [Result(i, np.zeros(1), np.zeros(1), 0.0, 0.0, (i + 1) * 1e-3) for i in range(100)]
    s = latency_summary(res)
    assert s["count"] == 100
    assert s["p50_ms"] == pytest.approx(50.5)
    assert s["p99_ms"] == pytest.approx(99.01)


def test_serving_workload_stream():
    dbs, req = gen.make_serving_workload(10_000, 5000, N_main=10, N_side=10)
    assert dbs[0].shape == (10, 128) and dbs[1].shape == (10, 256)
    t = req["t"]
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 10_000) < 10_000 * 0.05          # Poisson rate
    assert abs(req["db"].mean() - 0.2) < 0.03                     # 80/20 mix
    assert set(np.unique(req["k"])) == {1, 5, 10}
    assert set(np.unique(req["w"])) == {13, 26}                   # w = 0.1 n
    assert all(len(y) == (128, 256)[b] for y, b in zip(req["y"], req["db"]))


class _InstantExecutor:
    """Stand-in for the GPU executor: a launched batch is done at the next poll.  Records
    whether the cyclic garbage collector was on at each launch."""

    def __init__(self, slots=2, fail_at=None):
        self.slots = [None] * slots
        self.busy = {}
        self.gc_at_launch = []
        self.fail_at = fail_at

    def held(self, slot):
        return 0

    def need(self, slot, reqs):
        return len(reqs)

    def free_slots(self):
        return [i for i in range(len(self.slots)) if i not in self.busy]

    def launch(self, slot, reqs, now):
        import gc
        self.gc_at_launch.append(gc.isenabled())
        if self.fail_at is not None and len(self.gc_at_launch) > self.fail_at:
            raise RuntimeError("launch failed")
        self.busy[slot] = (list(reqs), now)

    def poll(self, now_fn):
        out = []
        for slot, (reqs, t_admit) in list(self.busy.items()):
            t = now_fn()
            out += [Result(r.rid, np.zeros(r.k, np.int64), np.zeros(r.k, np.float32), r.t_arrive, t_admit, t)
                    for r in reqs]
            del self.busy[slot]
        return out


@pytest.mark.parametrize("enabled_before", [True, False])
def test_serve_runs_with_cyclic_gc_off_and_restores_it(enabled_before):
    import gc
    from paper_0811_3301_amd.serve import serve
    ex = _InstantExecutor()
    reqs = _reqs(40)
    was = gc.isenabled()
    try:
        (gc.enable if enabled_before else gc.disable)()
        results, summary = serve(reqs, ex, budget_bytes=10**6, max_batch=8, idle_sleep=0)
        assert sorted(r.rid for r in results) == list(range(40)) and summary["requests"] == 40
        assert ex.gc_at_launch and not any(ex.gc_at_launch)
        assert gc.isenabled() == enabled_before
        # an error inside the loop restores the collector too
        with pytest.raises(RuntimeError):
            serve(_reqs(40), _InstantExecutor(fail_at=1), budget_bytes=10**6, max_batch=8, idle_sleep=0)
        assert gc.isenabled() == enabled_before
    finally:
        (gc.enable if was else gc.disable)()
