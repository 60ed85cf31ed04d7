"""Serving loop: continuous batching of k-NN DTW queries over device-resident databases.

Requests (a query series, its database, band w and k) arrive over time.  The loop keeps a
few batches in flight at once, each on its own library context and HIP stream.  Whenever a
slot is free it admits the requests that have arrived, oldest first, as one ragged batch
(mixed lengths and bands), so work that arrives while the GPU is busy joins the next free
slot instead of waiting for a fixed batch to fill.  A batch is admitted only if the device
workspace it needs fits the memory budget next to what the other slots hold; otherwise it is
cut down, and a request that fits nowhere waits for a slot with enough memory.

Each request's answer is the one ``lbimp_nn_search`` gives for it alone: batching only
changes which kernels run side by side (the distance of every pair is computed by the same
arithmetic, and the k nearest keys are a property of the set).  A batch is one ragged search
whatever the mix of lengths, bands and k of its requests.

The scheduling policy (``Scheduler``, ``MemoryBudget``) is plain Python and runs without a
GPU; ``GpuExecutor`` drives the HIP library through its C-ABI binding.
"""
from __future__ import annotations

import gc
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    t_arrive: float          # seconds from the start of the run
    db: int                  # database index
    y: np.ndarray            # float32 [n] query series (n = length of the database)
    w: int
    k: int


@dataclass
class Result:
    rid: int
    idx: np.ndarray          # int64 [k]
    dist: np.ndarray         # float32 [k]
    t_arrive: float
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class MemoryBudget:
    """Device-memory admission: each slot holds a workspace that only grows; a batch may start
    on a slot if the total held after it grows stays within the budget."""

    def __init__(self, budget_bytes: int, slots: int):
        self.budget = int(budget_bytes)
        self.held = [0] * slots

    def fits(self, slot: int, need: int) -> bool:
        others = sum(self.held) - self.held[slot]
        return others + max(self.held[slot], need) <= self.budget

    def commit(self, slot: int, held_after: int):
        self.held[slot] = max(self.held[slot], int(held_after))


class Scheduler:
    """FIFO admission of arrived requests into free slots, at most ``max_batch`` per batch.

    ``need(requests)`` estimates the device workspace of a batch; ``take`` returns the longest
    FIFO prefix of the arrived requests whose need fits the budget on the slot (halving the
    prefix until it fits).  A prefix of one request that fits nowhere stays queued."""

    def __init__(self, budget: MemoryBudget, max_batch: int, need):
        self.budget = budget
        self.max_batch = int(max_batch)
        self.need = need
        self.pending: deque[Request] = deque()

    def arrive(self, req: Request):
        self.pending.append(req)

    def take(self, free_slots):
        """Pick a slot among ``free_slots`` and the requests to run on it: (slot, reqs, need)
        or None.  Slots holding the most memory are tried first (they need no new memory)."""
        if not self.pending:
            return None
        order = sorted(free_slots, key=lambda s: -self.budget.held[s])
        count = min(self.max_batch, len(self.pending))
        while count >= 1:
            reqs = [self.pending[i] for i in range(count)]
            need = self.need(reqs)
            for slot in order:
                if self.budget.fits(slot, need):
                    for _ in range(count):
                        self.pending.popleft()
                    return slot, reqs, need
            count //= 2
        return None


def pretune_ragged(L, ctx, dbs, queries, db_of, w, p: int = 1, k=1, mode: str = "improved"):
    """Autotune every group of a ragged batch on its own before the batch runs.

    The library runs a ragged batch as one search per (database, effective band) group, each
    with the tuned choices recorded for its shape.  This tunes each group as a homogeneous
    batch (``lbimp_autotune`` on the group's queries, with the group's largest k), so the ragged
    call then uses the tuned choices without tuning inside it.  ``queries`` is a list of host
    float32 series."""
    import torch
    kq = np.broadcast_to(np.asarray(k, dtype=np.int64), (len(queries),))
    wq = np.broadcast_to(np.asarray(w, dtype=np.int64), (len(queries),))
    groups = {}
    for q, (b, wv) in enumerate(zip(db_of, wq)):
        n = len(queries[q])
        groups.setdefault((int(b), min(int(wv), n - 1)), []).append(q)
    for (b, wb), ids in sorted(groups.items()):
        Y = torch.from_numpy(np.stack([np.asarray(queries[q], np.float32) for q in ids])).cuda()
        L.lbimp_autotune(ctx, dbs[b], Y, wb, p, int(kq[ids].max()), mode)
    torch.cuda.synchronize()
    return len(groups)


def latency_summary(results) -> dict:
    lat = np.array([r.latency for r in results], dtype=np.float64) * 1e3
    if lat.size == 0:
        return dict(count=0)
    return dict(count=int(lat.size), p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()))


@dataclass
class _Slot:
    ctx: object
    stream: object
    qbuf: object                # device float32 [max_elems]
    qhost: object               # pinned float32 [max_elems]
    idx: object                 # device int64 [max_batch, kmax]
    dist: object                # device float32 [max_batch, kmax]
    idx_h: object               # pinned copies
    dist_h: object
    event: object = None
    batch: list = field(default_factory=list)
    kb: int = 1                 # output row stride of the batch in flight (its largest k)
    t_admit: float = 0.0
    busy: bool = False


class GpuExecutor:
    """In-flight batches on ``slots`` library contexts, one HIP stream each."""

    def __init__(self, dbs, slots: int = 4, max_batch: int = 512, kmax: int = 10, p: int = 1, mode: str = "improved",
                 workspace_limit: int = 0):
        import torch

        from . import lbimp as L
        self.torch, self.L = torch, L
        self.dbs, self.p, self.mode, self.kmax = dbs, p, mode, kmax
        self.max_batch = max_batch
        max_len = max(d.n for d in dbs)
        self.slots = []
        for _ in range(slots):
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                ctx = L.Ctx(0)
            # batches change shape from one launch to the next: launch directly, no graph capture,
            # and keep each batch on its slot's stream (the slots already overlap each other)
            L.lbimp_ctx_set_option(ctx, "graph", 0)
            L.lbimp_ctx_set_option(ctx, "ragged_streams", 0)
            # a bound on each slot's workspace: larger batches search the database in chunks
            L.lbimp_ctx_set_option(ctx, "workspace_limit", int(workspace_limit))
            elems = max_batch * max_len
            self.slots.append(_Slot(
                ctx=ctx, stream=stream,
                qbuf=torch.empty(elems, dtype=torch.float32, device="cuda"),
                qhost=torch.empty(elems, dtype=torch.float32, pin_memory=True),
                idx=torch.empty((max_batch, kmax), dtype=torch.int64, device="cuda"),
                dist=torch.empty((max_batch, kmax), dtype=torch.float32, device="cuda"),
                idx_h=torch.empty((max_batch, kmax), dtype=torch.int64, pin_memory=True),
                dist_h=torch.empty((max_batch, kmax), dtype=torch.float32, pin_memory=True),
                event=torch.cuda.Event()))

    def pretune(self, sample, sizes=(8, 16, 32, 64, 128, 256, 512)):
        """Autotune the batch shapes the loop will meet -- each (database, band, k) of `sample`
        at each batch size in `sizes` -- on slot 0, then share the choices with every slot."""
        torch, L = self.torch, self.L
        s0 = self.slots[0]
        shapes = {}
        for r in sample:
            shapes.setdefault((r.db, r.w, r.k), []).append(r.y)
        with torch.cuda.stream(s0.stream):
            for (db, w, k), ys in sorted(shapes.items()):
                for q in sizes:
                    Y = torch.from_numpy(np.stack([ys[i % len(ys)] for i in range(q)]).astype(np.float32)).cuda()
                    L.lbimp_autotune(s0.ctx, self.dbs[db], Y, w, self.p, k, self.mode)
        for s in self.slots[1:]:
            L.lbimp_ctx_copy_tuning(s.ctx, s0.ctx)
        torch.cuda.synchronize()

    def need(self, slot: int, reqs) -> int:
        """Workspace of the batch's ragged search on this slot."""
        return self.L.lbimp_nn_search_ragged_workspace(self.slots[slot].ctx, self.dbs, [r.db for r in reqs],
                                                       [r.w for r in reqs], self.p, [r.k for r in reqs], self.mode)

    def held(self, slot: int) -> int:
        return self.L.lbimp_ctx_workspace_bytes(self.slots[slot].ctx)

    def free_slots(self):
        return [i for i, s in enumerate(self.slots) if not s.busy]

    def launch(self, slot: int, reqs, now: float):
        torch, L = self.torch, self.L
        s = self.slots[slot]
        if len(reqs) > self.max_batch or any(r.k > self.kmax for r in reqs):
            raise ValueError("batch exceeds the executor's preallocated sizes")
        offsets = np.zeros(len(reqs) + 1, dtype=np.int64)
        np.cumsum([len(r.y) for r in reqs], out=offsets[1:])
        host = s.qhost.numpy()
        for r, o in zip(reqs, offsets[:-1]):
            host[o:o + len(r.y)] = r.y
        total = int(offsets[-1])
        ks = [r.k for r in reqs]
        kb = max(ks)  # output rows of the batch: each request's k nearest, then -1 / +inf up to kb
        used = len(reqs) * kb
        with torch.cuda.stream(s.stream):
            s.qbuf[:total].copy_(s.qhost[:total], non_blocking=True)
            out_i = s.idx.view(-1)[:used].view(len(reqs), kb)
            out_d = s.dist.view(-1)[:used].view(len(reqs), kb)
            L.lbimp_nn_search_ragged(s.ctx, self.dbs, s.qbuf, offsets, [r.db for r in reqs], [r.w for r in reqs],
                                     self.p, ks, self.mode, idx=out_i, dist=out_d, stats=False)
            s.idx_h.view(-1)[:used].copy_(s.idx.view(-1)[:used], non_blocking=True)
            s.dist_h.view(-1)[:used].copy_(s.dist.view(-1)[:used], non_blocking=True)
            s.event.record(s.stream)
        s.batch, s.kb, s.t_admit, s.busy = reqs, kb, now, True

    def poll(self, now_fn):
        """Results of the batches that have finished (non-blocking)."""
        out = []
        for s in self.slots:
            if not s.busy or not s.event.query():
                continue
            t_done = now_fn()
            ih, dh = s.idx_h.view(-1).numpy(), s.dist_h.view(-1).numpy()
            for j, r in enumerate(s.batch):
                a = j * s.kb
                out.append(Result(r.rid, ih[a:a + r.k].copy(), dh[a:a + r.k].copy(), r.t_arrive, s.t_admit, t_done))
            s.busy, s.batch = False, []
        return out

    def close(self):
        self.torch.cuda.synchronize()
        for s in self.slots:
            s.ctx.close()


def serve(requests, executor, budget_bytes: int, max_batch: int = 512, clock=time.perf_counter, idle_sleep=2e-5):
    """Run the request stream (sorted by arrival time) in real time; return (results, summary).

    Requests are released at their arrival times (seconds from the start); each free slot
    takes the arrived requests that fit the memory budget; finished batches are harvested
    as soon as their stream has run.  Latency counts from arrival to the harvest."""
    slots = len(executor.slots)
    budget = MemoryBudget(budget_bytes, slots)
    for i in range(slots):
        budget.commit(i, executor.held(i))
    # the workspace of a batch does not depend on the slot (all contexts share one device)
    sched = Scheduler(budget, max_batch, lambda reqs: executor.need(0, reqs))
    results = []
    n = len(requests)
    # The cyclic garbage collector stays off while the loop runs: a full collection over the
    # request and result objects pauses the loop for tens of milliseconds (measured p99 at
    # 20k requests/s: 70 ms with it, 10 ms without).  Requests and results hold no reference
    # cycles, so reference counting frees them; the collector's state is restored afterwards.
    gc_was_enabled = gc.isenabled()
    gc.disable()
    try:
        t_end = _serve_loop(requests, executor, budget, sched, results, clock, idle_sleep)
    finally:
        if gc_was_enabled:
            gc.enable()
    first = requests[0].t_arrive if n else 0.0
    summary = latency_summary(results)
    summary.update(requests=n, seconds=t_end - first, qps=n / max(t_end - first, 1e-9),
                   offered_qps=(n / max(requests[-1].t_arrive - first, 1e-9)) if n > 1 else None,
                   workspace_bytes=int(sum(budget.held)))
    return results, summary


def _serve_loop(requests, executor, budget, sched, results, clock, idle_sleep) -> float:
    """The real-time loop of ``serve``: appends to ``results``; returns its length in seconds."""
    slots = len(executor.slots)
    nxt = 0
    n = len(requests)
    t0 = clock()
    now = 0.0
    while len(results) < n:
        now = clock() - t0
        while nxt < n and requests[nxt].t_arrive <= now:
            sched.arrive(requests[nxt])
            nxt += 1
        done = executor.poll(lambda: clock() - t0)
        results.extend(done)
        progressed = bool(done)
        while True:
            free = executor.free_slots()
            if not free:
                break
            pick = sched.take(free)
            if pick is None:
                break
            slot, reqs, _ = pick
            executor.launch(slot, reqs, clock() - t0)
            budget.commit(slot, executor.held(slot))
            progressed = True
        if not progressed:
            if sched.pending and len(executor.free_slots()) == slots:
                raise RuntimeError("a request needs more device memory than the budget allows")
            if idle_sleep:
                time.sleep(idle_sleep)
    return clock() - t0
