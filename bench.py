"""Benchmark: 1-NN search under band-constrained DTW_1 on one MI355X.

Workload (the paper's 256-sample random-walk experiment, Sec. 10.1, at a 100,000-series
database): N = 100,000 random walks of length n = 256, Q = 256 fresh random-walk queries,
w = 26 (10% of n), p = 1, 1-NN.  A step is one nn_search call over the whole query batch in
the two-pass mode (LB_Keogh -> LB_Improved -> DTW); the database and queries are resident in
HBM before timing.  The same batch is also timed in LB_Keogh-only and brute-force mode, and at
p = 2.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1-NN DTW queries/sec (LB_Improved vs LB_Keogh vs brute); LB GB/s; p50/p99"
# fp32 vector peak 157.3 TFLOP/s counts an FMA as 2 flops: 78.65e12 VALU lane-instructions per
# second (256 CUs x 4 SIMDs x 64 lanes / 2 cycles x 2.4 GHz).  Algorithmic instruction counts:
# an LB_Keogh element is a clamp to the envelope (one med3), a subtract and an accumulate (add of
# |d|, or fma for p = 2): 3 instructions; a DTW cell is a subtract, a 3-way min (min3) and an
# accumulate: 3 instructions; an LB_Improved element about 9 (clamp, the running and block
# max/min of the projection's envelope, the distance of y to it, the accumulate).  A model of
# the issue cost, kept beside the count: a 3-operand med3/min3 issues in two slots, so an
# LB_Keogh element or a DTW cell costs 4 slots.  Pass 0 on the 32-part cover costs per (query,
# candidate) 3 instructions per part (clamp, subtract, accumulate), and reads 128 bytes of sums
# per candidate; with it, LB_Improved computes LB_Keogh too: 3 + 9 per element.
VALU_PEAK = 157.3e12 / 2
HBM_PEAK_GBPS = 8000.0
LBK_INSTR_PER_ELEM = 3
LBK_SLOTS_PER_ELEM_MODEL = 4
DTW_INSTR_PER_CELL = 3
LBI_INSTR_PER_ELEM = 9
PD_FINE_PARTS = 32
PDF_INSTR_PER_PART = 3


def sweep_traffic(profile="lbk_sweep_rw256_traffic.md", source="kernels_lb.hip"):
    """HBM bytes per launch of a kernel from its committed PMC summary under profiles/, if it was
    taken on the current source of that kernel (else None)."""
    import hashlib
    src = os.path.join(ROOT, "paper_0811_3301_amd", "csrc", source)
    prof = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(prof):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    fields = {}
    for line in open(prof):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != sha:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_mode(L, ctx, db, Yd, w, p, mode, steps, warmup):
    """A step is one search over the batch plus the copy of its results (idx, dist) to pinned
    host memory; each step ends when the results are on the host."""
    import torch
    Q = Yd.shape[0]
    idx = torch.empty((Q, 1), dtype=torch.int64, device="cuda")
    dist = torch.empty((Q, 1), dtype=torch.float32, device="cuda")
    idx_h = torch.empty((Q, 1), dtype=torch.int64, pin_memory=True)
    dist_h = torch.empty((Q, 1), dtype=torch.float32, pin_memory=True)

    def step():
        L.lbimp_nn_search(ctx, db, Yd, w, p, 1, mode, idx=idx, dist=dist, stats=False)
        idx_h.copy_(idx, non_blocking=True)
        dist_h.copy_(dist, non_blocking=True)
        torch.cuda.current_stream().synchronize()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per = []
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        a = time.perf_counter()
        step()
        per.append((time.perf_counter() - a) * 1e3)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    return dict(ms_per_step=ev_ms / steps, wall_ms_per_step=wall * 1e3 / steps, step_ms=per,
                idx=idx_h.numpy()[:, 0].copy(), dist=dist_h.numpy()[:, 0].copy())


def stage_work(mode, Q, N, n, w, st, pd=0):
    """Algorithmic work of the stages of one step from the measured counts: (instructions, HBM
    bytes) of the first pass, instructions of LB_Improved, and the DTW instructions bracketed
    low/high.  First pass: 3 instructions per LB_Keogh element of every pair and the database
    read once, or with pass 0 on the 32-part cover (pd = 2) 3 per part of every pair and its
    128-byte sums per candidate.  LB_Improved: 9 per element of every pass-1 survivor, or with
    pd = 2 (3 + 9) per element of every pass-0 survivor (LB_Keogh computed there).  DTW: 3 per
    cell of the DTWs that ran to the end, plus those that were abandoned counted at 0 cells (low)
    or in full (high); the two bracket the cells actually computed."""
    cells = n * (2 * w + 1) - w * (w + 1)
    started, abandoned = float(st[:, 4].sum()), float(st[:, 5].sum())
    dtw = (DTW_INSTR_PER_CELL * cells * (started - abandoned), DTW_INSTR_PER_CELL * cells * started)
    if mode == "brute":
        return dict(first=(0.0, 0.0), lbi=0.0, dtw=dtw)
    if pd == 2 and mode == "improved":
        first = (PDF_INSTR_PER_PART * PD_FINE_PARTS * Q * N, N * PD_FINE_PARTS * 4)
        survivors0 = float((st[:, 0] - st[:, 1] - st[:, 6]).sum())  # pass-0 survivors (seeds excluded)
        lbi = (LBK_INSTR_PER_ELEM + LBI_INSTR_PER_ELEM) * n * survivors0
    else:
        first = (LBK_INSTR_PER_ELEM * Q * N * n, N * n * 4)
        survivors1 = float((st[:, 3] + st[:, 4] - st[:, 1]).sum())  # pass-1 survivors (seeds excluded)
        lbi = LBI_INSTR_PER_ELEM * n * survivors1 if mode == "improved" else 0.0
    return dict(first=first, lbi=lbi, dtw=dtw)


def t_roof(mode, Q, N, n, w, st, pd=0):
    """Roofline time of one step from the measured counts (stage_work): max(first-pass HBM
    bytes / HBM peak, first-pass instructions / VALU peak) + (LB_Improved + DTW instructions) /
    VALU peak, with the DTW bracketed low/high."""
    wk = stage_work(mode, Q, N, n, w, st, pd)
    base = max(wk["first"][1] / (HBM_PEAK_GBPS * 1e9), wk["first"][0] / VALU_PEAK)
    lo = base + (wk["lbi"] + wk["dtw"][0]) / VALU_PEAK
    hi = base + (wk["lbi"] + wk["dtw"][1]) / VALU_PEAK
    return lo * 1e3, hi * 1e3


def golden_errors(name, idx, dist, p):
    """Index agreement and relative distance errors of the device's 1-NN against the oracle's
    brute force, stored in tests/golden by tests/golden/make_full_size.py."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_nn.txt")
    if not os.path.exists(path):
        return None
    rows = np.loadtxt(path, comments="#", dtype=np.float64, ndmin=2)
    oi, od = rows[:, 1].astype(np.int64), rows[:, 2]
    want = od if p == 1 else np.sqrt(od)
    rel = np.abs(np.asarray(dist, np.float64) - want) / np.maximum(want, 1e-30)
    return dict(queries=int(rows.shape[0]), index_agreement=float(np.mean(oi == np.asarray(idx))),
                rel_err_max=float(rel.max()), rel_err_median=float(np.median(rel)),
                rel_err_p99=float(np.percentile(rel, 99)))


def stage_profile(L, ctx, db, Yd, w, p, mode, steps, k=1):
    import torch
    L.lbimp_ctx_set_timing(ctx, True)
    acc = {}
    for _ in range(steps):
        L.lbimp_nn_search(ctx, db, Yd, w, p, k, mode, stats=False)
        for name, v in L.lbimp_ctx_stage_times(ctx).items():
            acc[name] = acc.get(name, 0.0) + v
    L.lbimp_ctx_set_timing(ctx, False)
    torch.cuda.synchronize()
    return {name: v / steps for name, v in acc.items()}


def big_database(L, ctx):
    """The 1,000,000 x 128 random-walk database of the serving workload (512 MB, twice the
    256 MB Infinity Cache), resident on the device."""
    import torch
    from paper_0811_3301_amd import gen
    X = torch.from_numpy(gen.random_walk(1_000_000, 128, gen.rng(5, gen.ROLE_DB)).astype(np.float32)).cuda()
    db = L.Db(ctx, X)
    del X
    torch.cuda.synchronize()
    return db


def single_query_lb_gbps(L, ctx, steps=20, db=None):
    """LB_Keogh of one query over a 1,000,000 x 128 random-walk database (512 MB, larger than
    the 256 MB Infinity Cache): the HBM-bound form of the first pass."""
    import torch
    from paper_0811_3301_amd import gen
    N, n, w = 1_000_000, 128, 13
    own = db is None
    if own:
        db = big_database(L, ctx)
    y = torch.from_numpy(gen.random_walk(1, n, gen.rng(5, gen.ROLE_QUERY)).astype(np.float32)).cuda()
    U, Lo = L.lbimp_envelope(ctx, y, w)
    out = torch.empty((1, N), dtype=torch.float32, device="cuda")
    for _ in range(3):
        L.lbimp_db_lb_keogh(ctx, db, U, Lo, 1, out=out)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        L.lbimp_db_lb_keogh(ctx, db, U, Lo, 1, out=out)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if own:
        db.close()
    nbytes = N * n * 4
    return dict(db_bytes=nbytes, ms=ms, gbps=nbytes / ms / 1e6, frac_hbm=nbytes / ms / 1e6 / HBM_PEAK_GBPS)


def pd_bench(L, ctx, db, steps=20, qs=(1, 4, 16)):
    """Pass 0 (piecewise sums, Sec. 9) ahead of LB_Keogh on the 512 MB database, w = 13, p = 1,
    1-NN, two-pass search of Q queries per call: the time per call and the database bytes the
    first passes read with and without it, at identical results."""
    import torch
    from paper_0811_3301_amd import gen
    N, n, w = 1_000_000, 128, 13
    ctx = L.Ctx(0)  # untuned: both forms run with the default choices
    Y = torch.from_numpy(gen.random_walk(max(qs), n, gen.rng(5, gen.ROLE_QUERY, 7)).astype(np.float32)).cuda()
    out = dict(workload="1,000,000 x 128 random walks (512 MB), w=13, p=1, 1-NN, two-pass search",
               pass0_bytes_per_candidate=64)
    for Q in qs:
        Yq = Y[:Q].contiguous()
        r = {}
        for pd in (0, 1):
            L.lbimp_ctx_set_option(ctx, "pd_prefilter", pd)
            t = time_mode(L, ctx, db, Yq, w, 1, "improved", steps, 2)
            _, _, st = L.lbimp_nn_search(ctx, db, Yq, w, 1, 1, "improved")
            st_ms = stage_profile(L, ctx, db, Yq, w, 1, "improved", 5)
            c0 = float((N - st[:, 1] - st[:, 6]).sum())  # pass-0 survivors (all candidates without pass 0)
            # bytes of the database read by the passes before LB_Improved: the sweep reads every
            # row once per query group of 16; pass 0 reads the sums, then the rows of its survivors
            first = (N * 8 * 8 * -(-Q // 16) + c0 * n * 4) if pd else N * n * 4 * -(-Q // 16)
            r["pd" if pd else "sweep"] = dict(ms_per_call=t["ms_per_step"], qps=Q / t["ms_per_step"] * 1e3,
                                              first_pass_db_bytes=first, stage_ms=st_ms,
                                              pass0_survivor_fraction=c0 / (N * Q) if pd else None,
                                              idx=t["idx"].tolist())
        L.lbimp_ctx_set_option(ctx, "pd_prefilter", 0)
        r["same_results"] = r["pd"].pop("idx") == r["sweep"].pop("idx")
        r["speedup"] = r["sweep"]["ms_per_call"] / r["pd"]["ms_per_call"]
        out[f"Q{Q}"] = r
    torch.cuda.synchronize()
    ctx.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(X, Ys, w, p, gpu_idx, budget_s=8.0):
    """The fp64 oracle on the host: brute-force DTW over the whole database (the definition) on
    all cores and on one core, and the paper's own sequential Algorithms 3 and 2 (one query per
    thread, database order), each on a bounded sample of the headline's queries."""
    from oracle import native
    native.load()
    X64 = X.astype(np.float64)
    Y64 = Ys.astype(np.float64)
    cores = len(os.sched_getaffinity(0))
    native.set_num_threads(cores)
    threads = native.num_threads()

    def timed(fn, *a):
        t = time.perf_counter()
        r = fn(*a)
        return r, time.perf_counter() - t

    (idx, _), first = timed(native.nn_bruteforce, X64, Y64[:1], w, p, 1)
    more = int(max(0, min(Ys.shape[0] - 1, budget_s / max(first, 1e-3) - 1)))
    (idx2, _), rest = timed(native.nn_bruteforce, X64, Y64[1:1 + more], w, p, 1)
    nq = 1 + more
    allidx = np.concatenate([idx[:, 0], idx2[:, 0]]) if more else idx[:, 0]
    out = dict(value=nq / (first + rest), unit="queries/s", cores=threads, kind="oracle",
               sample=f"{nq} of {Ys.shape[0]} queries, brute-force fp64 DTW against all {X.shape[0]} candidates, "
                      f"{threads} threads", seconds=first + rest,
               index_agreement_sample=float(np.mean(allidx == gpu_idx[:nq])), cpu_model=cpu_model(),
               host_cores=cores)
    native.set_num_threads(1)
    _, t1 = timed(native.nn_bruteforce, X64, Y64[:1], w, p, 1)
    out["brute_force_1_core"] = dict(value=1.0 / t1, unit="queries/s", sample="1 query")
    # the paper's method on the host: one query per thread, sequential scan in database order
    for name, improved in (("algorithm3_lb_improved", True), ("algorithm2_lb_keogh", False)):
        r = {}
        native.set_num_threads(1)
        q1 = 4
        (i1, _, c1), t = timed(native.nn_sequential, X64, Y64[:q1], w, p, improved)
        r["1_core"] = dict(value=q1 / t, unit="queries/s", sample=f"{q1} queries")
        native.set_num_threads(threads)
        qa = min(Ys.shape[0], 2 * threads)
        (ia, _, ca), t = timed(native.nn_sequential, X64, Y64[:qa], w, p, improved)
        r["all_cores"] = dict(value=qa / t, unit="queries/s", sample=f"{qa} queries, {threads} threads")
        r["same_index_as_device"] = float(np.mean(ia == gpu_idx[:qa]))
        r["dtw_fraction"] = float(ca[:, 2].sum() / (qa * X.shape[0]))
        out[name] = r
    native.set_num_threads(threads)
    return out


def ragged_bench(L, steps, warmup):
    """Uneven batch: 4,096 random-walk queries, lengths uniform over {64,...,1024}, w = round(f n)
    with f uniform over {0.05, 0.1, 0.2}, one 20,000-series database per length, p = 1, 1-NN,
    one lbimp_nn_search_ragged call per step (captured once as a HIP graph, then replayed).  Every
    group is autotuned on its own first (lbimp_autotune on the group's queries); the ragged call
    then runs with the tuned choices and tunes nothing itself."""
    import torch
    from paper_0811_3301_amd import gen
    from paper_0811_3301_amd.serve import pretune_ragged
    ctx = L.Ctx(0)
    dbs, qs, db_of, w = gen.make_ragged_workload()
    handles = [L.Db(ctx, torch.from_numpy(d.astype(np.float32)).cuda()) for d in dbs]
    pretune_ragged(L, ctx, handles, [q.astype(np.float32) for q in qs], db_of, w, 1, 1, "improved")
    off = np.zeros(len(qs) + 1, np.int64)
    off[1:] = np.cumsum([len(y) for y in qs])
    packed = torch.from_numpy(np.concatenate(qs).astype(np.float32)).cuda()
    Q = len(qs)
    idx = torch.empty((Q, 1), dtype=torch.int64, device="cuda")
    dist = torch.empty((Q, 1), dtype=torch.float32, device="cuda")
    out = {}
    for graph in (1, 0):
        L.lbimp_ctx_set_option(ctx, "graph", graph)
        call = lambda: L.lbimp_nn_search_ragged(ctx, handles, packed, off, db_of, w, 1, 1, "improved", idx=idx,
                                                dist=dist, stats=False)
        for _ in range(warmup):
            call()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / steps * 1e3
        out["graph" if graph else "eager"] = dict(ms_per_step=ms, qps=Q / ms * 1e3)
    L.lbimp_ctx_set_option(ctx, "graph", 1)
    _, _, st = L.lbimp_nn_search_ragged(ctx, handles, packed, off, db_of, w, 1, 1, "improved")
    torch.cuda.synchronize()
    for h in handles:
        h.close()
    ctx.close()
    return dict(workload="uneven batch: 4096 random-walk queries, n in {64,128,256,512,1024}, w = round(f n), "
                         "f in {0.05,0.1,0.2}, 20000-series database per length, p=1, 1-NN",
                queries=Q, groups=len(set(zip(db_of.tolist(), w.tolist()))), autotuned="per group, before the batch", **out,
                dtw_fraction=float(st[:, 4].sum() / st[:, 0].sum()))


def shape_bench(L, steps):
    """Shape-like signatures: 50,000 x 512 database, 512 queries, w = 26 and 51, p = 1, 1-NN;
    two-pass, LB_Keogh-only and brute-force search, autotuned on an untimed first call."""
    import torch
    from paper_0811_3301_amd import gen
    db64, qs64 = gen.make_workload("shape512")
    N, n = db64.shape
    Q = qs64.shape[0]
    ctx = L.Ctx(0)
    L.lbimp_ctx_set_option(ctx, "autotune", 1)
    db = L.Db(ctx, torch.from_numpy(db64.astype(np.float32)).cuda())
    Yd = torch.from_numpy(qs64.astype(np.float32)).cuda()
    del db64
    out = dict(workload="shape-like centroid-distance signatures, n=512, database 50000, 512 queries, p=1, 1-NN",
               N=N, n=n, Q=Q)
    for w in (26, 51):
        r = {}
        for mode, k in (("improved", steps), ("keogh", steps), ("brute", 2)):
            t = time_mode(L, ctx, db, Yd, w, 1, mode, k, 1)
            r[mode] = dict(qps=Q / (t["ms_per_step"] / 1e3), ms_per_step=t["ms_per_step"],
                           oracle=golden_errors(f"shape512_w{w}", t["idx"], t["dist"], 1))
        _, _, st = L.lbimp_nn_search(ctx, db, Yd, w, 1, 1, "improved")
        r["pruned_keogh"] = float(st[:, 2].sum() / (N * Q))
        r["pruned_improved"] = float(st[:, 3].sum() / (N * Q))
        r["dtw_fraction"] = float(st[:, 4].sum() / (N * Q))
        out[f"w{w}"] = r
    torch.cuda.synchronize()
    db.close()
    ctx.close()
    return out


def lbi_abandon_bench(L, steps=10):
    """Early abandoning inside LB_Improved (the paper's Sec. 10 experiment on the CPU measured
    under 1%): the two-pass search with it off and on, untuned, on the headline workload (the
    register kernel, w = 26) and on wide bands (the wave-per-pair kernel: 20,000 x 1024 random
    walks, 64 queries, w = 102 and 205)."""
    import torch
    from paper_0811_3301_amd import gen
    out = {}
    cases = (("rw256_w26", "rw256", 26), ("rw1024_w102", None, 102), ("rw1024_w205", None, 205))
    ctx = L.Ctx(0)
    cache = {}
    for name, wl, w in cases:
        if wl not in cache:
            if wl:
                db64, qs64 = gen.make_workload(wl)
            else:
                db64 = gen.random_walk(20_000, 1024, gen.rng(4, gen.ROLE_DB, 4))
                qs64 = gen.random_walk(64, 1024, gen.rng(4, gen.ROLE_QUERY, 9))
            cache[wl] = (L.Db(ctx, torch.from_numpy(db64.astype(np.float32)).cuda()),
                         torch.from_numpy(qs64.astype(np.float32)).cuda())
        db, Yd = cache[wl]
        r = {}
        for ab in (0, 1):
            L.lbimp_ctx_set_option(ctx, "lbi_abandon", ab)
            t = time_mode(L, ctx, db, Yd, w, 1, "improved", steps, 1)
            st_ms = stage_profile(L, ctx, db, Yd, w, 1, "improved", 3)
            r["on" if ab else "off"] = dict(ms_per_call=t["ms_per_step"], lb_improved_ms=st_ms["lb_improved"],
                                            idx=t["idx"].tolist())
        L.lbimp_ctx_set_option(ctx, "lbi_abandon", 0)
        r["same_results"] = r["on"].pop("idx") == r["off"].pop("idx")
        r["lb_improved_speedup"] = r["off"]["lb_improved_ms"] / r["on"]["lb_improved_ms"]
        out[name] = r
    torch.cuda.synchronize()
    for db, _ in cache.values():
        db.close()
    ctx.close()
    return out


def strip_bench(L, steps=3, N=5_000, Q=16):
    """The wide-band DTW kernels on their own: brute-force search (every pair's full DTW) of Q
    random-walk queries over N x 1024 random walks at w = 102 and 205, p = 1, untuned (lane per
    pair in strips of rows).  Reports DTW cells per second: n (2w + 1) - w (w + 1) per pair."""
    import torch
    from paper_0811_3301_amd import gen
    n = 1024
    ctx = L.Ctx(0)
    db = L.Db(ctx, torch.from_numpy(gen.random_walk(N, n, gen.rng(4, gen.ROLE_DB, 5)).astype(np.float32)).cuda())
    Yd = torch.from_numpy(gen.random_walk(Q, n, gen.rng(4, gen.ROLE_QUERY, 10)).astype(np.float32)).cuda()
    out = {}
    for w in (102, 205):
        t = time_mode(L, ctx, db, Yd, w, 1, "brute", steps, 1)
        cells = Q * N * (n * (2 * w + 1) - w * (w + 1))
        out[f"w{w}"] = dict(ms_per_call=t["ms_per_step"], cells_per_s=cells / (t["ms_per_step"] / 1e3),
                            frac_of_alu_peak=DTW_INSTR_PER_CELL * cells / (t["ms_per_step"] / 1e3) / VALU_PEAK)
    db.close()
    ctx.close()
    return dict(workload=f"brute-force DTW_1, {Q} queries over {N} x {n} random walks", **out)


def triangle_bench(L, ctx, count=100_000, n=100, steps=5):
    """App. B: 100,000 triples (x, y, z) of 100-sample random walks (and white noise),
    unconstrained DTW_1 and DTW_2 (w = n), C = DTW(x,z) / (DTW(x,y) + DTW(y,z)); one
    lbimp_dtw_pairs call computes the 300,000 distances of a p."""
    import torch
    from paper_0811_3301_amd import gen
    cells = n * n
    out = dict(workload=f"{count} triples of {n}-sample series, unconstrained DTW (w = n)", pairs_per_call=3 * count,
               paper_violation_share={"random_walk": {"p1": 0.20, "p2": 0.15}, "white_noise": {"p1": 0.0, "p2": 0.0}})
    for kind in ("random_walk", "white_noise"):
        X, Y, Z = (torch.from_numpy(a.astype(np.float32)).cuda() for a in gen.triangle_triples(count, n, kind))
        A = torch.cat([X, Y, X]).contiguous()
        B = torch.cat([Y, Z, Z]).contiguous()
        dist = torch.empty(3 * count, dtype=torch.float32, device="cuda")
        r = {}
        for p in (1, 2):
            L.lbimp_dtw_pairs(ctx, A, B, n, p, out=dist)
            torch.cuda.synchronize()
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(steps):
                L.lbimp_dtw_pairs(ctx, A, B, n, p, out=dist)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            d = dist.cpu().numpy().astype(np.float64).reshape(3, count)
            C = d[2] / (d[0] + d[1])
            r[f"p{p}"] = dict(violation_share=float(np.mean(C > 1)), C_max=float(C.max()), ms=ms,
                              pairs_per_s=3 * count / ms * 1e3, cells_per_s=3 * count * cells / ms * 1e3,
                              dtw_frac_of_alu_peak=DTW_INSTR_PER_CELL * 3 * count * cells / (ms / 1e3) / VALU_PEAK)
        out[kind] = r
        del X, Y, Z, A, B, dist
    return out


def serving_bench(L, rates, measured=20_000, warmup_s=2.0, max_batch=512, slots=4, budget=4 << 30):
    """Serving: Poisson arrivals over a resident 1,000,000 x 128 random-walk database (512 MB)
    and a 200,000 x 256 side database (20% of requests), w = round(0.1 n), k uniform over
    {1, 5, 10}; continuous batching on `slots` in-flight batches under a device-memory budget.
    Each arrival rate runs one stream: warmup_s seconds of arrivals, then `measured` requests;
    latencies (arrival to results on the host) and throughput come from the measured ones."""
    from paper_0811_3301_amd.serve import latency_summary
    import torch
    from paper_0811_3301_amd import gen
    from paper_0811_3301_amd.serve import GpuExecutor, Request, serve
    dbs64, _ = gen.make_serving_workload(1.0, 1, with_databases=True)
    ctx = L.Ctx(0)
    handles = [L.Db(ctx, torch.from_numpy(d.astype(np.float32)).cuda()) for d in dbs64]
    del dbs64
    torch.cuda.synchronize()
    # each slot's workspace is bounded by its share of the budget: a batch larger than that
    # searches the database in chunks of candidates
    ex = GpuExecutor(handles, slots=slots, max_batch=max_batch, kmax=10, workspace_limit=budget // slots)
    runs = []
    try:
        _, sample = gen.make_serving_workload(rates[-1], 300, with_databases=False)
        ex.pretune([Request(rid=j, t_arrive=0.0, db=int(sample["db"][j]), y=sample["y"][j].astype(np.float32),
                            w=int(sample["w"][j]), k=int(sample["k"][j])) for j in range(300)])
        for rate in rates:
            warm = max(200, int(rate * warmup_s))
            count = warm + measured
            _, req = gen.make_serving_workload(rate, count, with_databases=False)
            reqs = [Request(rid=j, t_arrive=float(req["t"][j]), db=int(req["db"][j]),
                            y=req["y"][j].astype(np.float32), w=int(req["w"][j]), k=int(req["k"][j]))
                    for j in range(count)]
            del req
            results, whole = serve(reqs, ex, budget_bytes=budget, max_batch=max_batch)
            meas = [r for r in results if r.rid >= warm]
            summ = latency_summary(meas)
            t0 = min(r.t_arrive for r in meas)
            t1 = max(r.t_done for r in meas)
            summ.update(offered_rate=rate, warmup_requests=warm, qps=len(meas) / max(t1 - t0, 1e-9),
                        offered_qps=len(meas) / max(reqs[-1].t_arrive - reqs[warm].t_arrive, 1e-9),
                        workspace_bytes=whole["workspace_bytes"])
            runs.append(summ)
            log(f"serving at {rate} q/s: p50 {summ['p50_ms']:.3f} ms, p99 {summ['p99_ms']:.3f} ms, "
                f"{summ['qps']:.0f} q/s over {len(meas)} requests")
            del reqs, results, meas
    finally:
        ex.close()
        for h in handles:
            h.close()
        ctx.close()
    return dict(workload="serving: Poisson arrivals, 80% n=128 over a resident 1,000,000-series database "
                         "(512 MB), 20% n=256 over a 200,000-series database, w=round(0.1 n), k in {1,5,10}, "
                         "two-pass search", slots=slots, max_batch=max_batch, memory_budget_bytes=budget,
                workspace_limit_per_slot=budget // slots,
                protocol=f"{warmup_s:g} s of arrivals as warm-up, then {measured} measured requests per rate",
                runs=runs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--quick", action="store_true", help="two-pass mode only (for profiling runs)")
    ap.add_argument("--no-ragged", action="store_true", help="skip the uneven-batch measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-shapes", action="store_true", help="skip the shape-signature measurement")
    ap.add_argument("--no-triangle", action="store_true", help="skip the App. B triangle-inequality workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the headline with the context's default choices (with --set: profiling A/B)")
    ap.add_argument("--set", action="append", default=[], metavar="NAME=VALUE",
                    help="context option for the headline searches (repeatable), e.g. lbi_buckets=1")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device-to-device copy (calibrates the PMC byte counters)")
    ap.add_argument("--only", choices=("ragged", "serving", "shapes", "triangle", "lbsingle", "pd", "abandon",
                                       "batch1m", "strip"),
                    help="run only the uneven-batch or the serving measurement and print its JSON (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0811_3301_amd import gen, lbimp as L

    if args.copy_probe:
        a = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4}), flush=True)
        return

    L.load()
    if args.only == "ragged":
        print(json.dumps(ragged_bench(L, args.steps, args.warmup)), flush=True)
        return
    if args.only == "shapes":
        print(json.dumps(shape_bench(L, args.steps)), flush=True)
        return
    if args.only == "batch1m":
        # one serving-sized batch: 410 random-walk queries over the 1,000,000 x 128 database,
        # w = 13, p = 1, k = 10, two-pass search (the shape profiled for the LB_Improved and DTW
        # counters of a serving batch)
        ctx = L.Ctx(0)
        big = big_database(L, ctx)
        Yq = torch.from_numpy(gen.random_walk(410, 128, gen.rng(5, gen.ROLE_QUERY, 8)).astype(np.float32)).cuda()
        for _ in range(args.warmup + args.steps):
            L.lbimp_nn_search(ctx, big, Yq, 13, 1, 10, "improved", stats=False)
        torch.cuda.synchronize()
        st = stage_profile(L, ctx, big, Yq, 13, 1, "improved", 3, k=10)
        print(json.dumps({"batch1m_stage_ms": st}), flush=True)
        big.close()
        ctx.close()
        return
    if args.only == "strip":
        print(json.dumps(strip_bench(L, args.steps)), flush=True)
        return
    if args.only == "abandon":
        print(json.dumps(lbi_abandon_bench(L, args.steps)), flush=True)
        return
    if args.only in ("triangle", "lbsingle", "pd"):
        ctx = L.Ctx(0)
        if args.only == "triangle":
            out = triangle_bench(L, ctx)
        elif args.only == "lbsingle":
            out = single_query_lb_gbps(L, ctx, args.steps)
        else:
            big = big_database(L, ctx)
            out = pd_bench(L, ctx, big, args.steps)
            big.close()
        print(json.dumps(out), flush=True)
        ctx.close()
        return
    if args.only == "serving":
        print(json.dumps(serving_bench(L, rates=(10_000,), measured=3000, warmup_s=0.3)), flush=True)
        return
    N, n, Q, w = 100_000, 256, 256, 26
    log("generating workload")
    db64, qs64 = gen.make_workload("rw256")
    X, Ys = db64.astype(np.float32), qs64.astype(np.float32)
    ctx = L.Ctx(0)
    db = L.Db(ctx, torch.from_numpy(X).cuda())
    Yd = torch.from_numpy(Ys).cuda()
    torch.cuda.synchronize()
    # the autotuner picks seeds, tiling and kernels for each mode/p on its first (warm-up) call
    L.lbimp_ctx_set_option(ctx, "autotune", 0 if args.no_autotune else 1)
    for kv in args.set:
        name, value = kv.split("=", 1)
        L.lbimp_ctx_set_option(ctx, name, int(value))

    # the headline's tuned choices, recorded (the searches below find them and tune nothing)
    set_opts = {k: int(v) for k, v in (kv.split("=", 1) for kv in args.set)}
    knobs = {}
    for mode in ("improved", "keogh"):
        knobs[mode] = None if args.no_autotune else L.lbimp_autotune(ctx, db, Yd, w, 1, 1, mode)
    pd_of = {m: (kn["pd"] if kn else set_opts.get("pd_prefilter", 0)) for m, kn in knobs.items()}
    pd_of["brute"] = 0

    log("timing two-pass p=1")
    imp = time_mode(L, ctx, db, Yd, w, 1, "improved", args.steps, args.warmup)
    gpu_idx = imp["idx"]
    _, _, st = L.lbimp_nn_search(ctx, db, Yd, w, 1, 1, "improved")
    stages = stage_profile(L, ctx, db, Yd, w, 1, "improved", max(3, args.steps // 2))

    def mode_entry(r, stats, mode):
        lo, hi = t_roof(mode, Q, N, n, w, stats, pd_of[mode])
        return dict(qps=Q / (r["ms_per_step"] / 1e3), ms_per_step=r["ms_per_step"],
                    t_roof_ms=[lo, hi], roof_frac=[lo / r["ms_per_step"], hi / r["ms_per_step"]])

    modes = {"improved": mode_entry(imp, st, "improved")}
    accuracy = {"rw256_p1": golden_errors("rw256_p1", imp["idx"], imp["dist"], 1)}
    if not args.quick:
        for mode, steps in (("keogh", args.steps), ("brute", max(2, args.steps // 10))):
            log(f"timing {mode} p=1")
            r = time_mode(L, ctx, db, Yd, w, 1, mode, steps, 1)
            _, _, st_m = L.lbimp_nn_search(ctx, db, Yd, w, 1, 1, mode)
            modes[mode] = mode_entry(r, st_m, mode)
            modes[mode]["same_result_as_two_pass"] = bool(np.array_equal(r["idx"], gpu_idx))
            modes[mode]["oracle"] = golden_errors("rw256_p1", r["idx"], r["dist"], 1)
        log("timing two-pass p=2")
        r2 = time_mode(L, ctx, db, Yd, w, 2, "improved", args.steps, 1)
        rk2 = time_mode(L, ctx, db, Yd, w, 2, "keogh", args.steps, 1)
        _, _, st2 = L.lbimp_nn_search(ctx, db, Yd, w, 2, 1, "improved")
        p2 = dict(improved_qps=Q / (r2["ms_per_step"] / 1e3), keogh_qps=Q / (rk2["ms_per_step"] / 1e3),
                  pruned_keogh=float(st2[:, 2].sum() / (N * Q)), pruned_improved=float(st2[:, 3].sum() / (N * Q)),
                  dtw_fraction=float(st2[:, 4].sum() / (N * Q)))
        accuracy["rw256_p2"] = golden_errors("rw256_p2", r2["idx"], r2["dist"], 2)
    else:
        p2 = None

    # rooflines of the stages of the tuned two-pass step; the bench line reports the longest
    wk = stage_work("improved", Q, N, n, w, st, pd_of["improved"])
    fine = pd_of["improved"] == 2

    def roof(kernel, ms, instr, **extra):
        achieved = instr / (ms / 1e3)
        return dict(kernel=kernel, bound="alu", kernel_ms=ms, instructions=instr, achieved=achieved / 1e12,
                    peak=VALU_PEAK / 1e12, unit="T VALU lane-instructions/s", frac=achieved / VALU_PEAK, **extra)

    elems = Q * N * n
    if fine:
        first = roof("k_pdf_scan (pass 0: 32-part piecewise-sum bound of every query x candidate)",
                     stages["lb_keogh"], wk["first"][0], instructions_per_pair=PDF_INSTR_PER_PART * PD_FINE_PARTS,
                     pairs=Q * N, algorithmic_hbm_bytes=wk["first"][1] + Q * ((N + 63) // 64 * 64) * 4)
    else:
        first = roof("k_lbk_sweep (LB_Keogh of every query x candidate)", stages["lb_keogh"], wk["first"][0],
                     instructions_per_element=LBK_INSTR_PER_ELEM, elements=elems,
                     frac_issue_model=LBK_SLOTS_PER_ELEM_MODEL * elems / (stages["lb_keogh"] / 1e3) / VALU_PEAK,
                     issue_model="med3 issues in two slots: 4 slots per element",
                     algorithmic_hbm_bytes=N * n * 4 + Q * ((N + 63) // 64 * 64) * 4)
    lbi_pairs = float((st[:, 0] - st[:, 1] - st[:, 6]).sum()) if fine else float((st[:, 3] + st[:, 4] - st[:, 1]).sum())
    second = roof("k_lbi_reg (LB_Improved" + (" with LB_Keogh, of every pass-0 survivor)" if fine else
                                              " of every pass-1 survivor)"),
                  stages["lb_improved"], wk["lbi"],
                  instructions_per_element=(LBK_INSTR_PER_ELEM if fine else 0) + LBI_INSTR_PER_ELEM,
                  pairs=lbi_pairs, row_bytes=lbi_pairs * n * 4)
    dtw = roof("k_dtw_lane (DTW of the survivors, abandoned DTWs counted in full)", stages["dtw"], wk["dtw"][1],
               frac_low=wk["dtw"][0] / (stages["dtw"] / 1e3) / VALU_PEAK)
    stage_roofs = {"first_pass": first, "lb_improved": second, "dtw": dtw}
    dom = max(stage_roofs, key=lambda k_: stage_roofs[k_]["kernel_ms"])
    traffic = None
    if dom == "first_pass" and not fine:
        traffic = sweep_traffic()
    elif dom == "lb_improved" and fine:
        traffic = sweep_traffic("lbi_fused_rw256_traffic.md", "lbi_reg.h")
    roofline = dict(stage_roofs[dom], traffic=traffic, stage=dom)
    if "brute" in modes:
        cells = Q * N * (n * (2 * w + 1) - w * (w + 1))
        t = modes["brute"]["ms_per_step"] / 1e3
        modes["brute"]["dtw_cells_per_s"] = cells / t
        modes["brute"]["dtw_frac_of_alu_peak"] = DTW_INSTR_PER_CELL * cells / t / VALU_PEAK

    lbg = pdb = None
    if not args.quick:
        log("single-query LB_Keogh sweep over a 512 MB database")
        big = big_database(L, ctx)
        lbg = single_query_lb_gbps(L, ctx, db=big)
        log("pass 0 (piecewise sums) against the sweep on the 512 MB database")
        pdb = pd_bench(L, ctx, big)
        big.close()

    ragged = None
    if not (args.quick or args.no_ragged):
        log("uneven batch (4096 queries of mixed lengths and bands)")
        ragged = ragged_bench(L, max(3, args.steps // 4), 2)

    shapes = None
    if not (args.quick or args.no_shapes):
        log("shape signatures (n=512, w=26 and 51)")
        shapes = shape_bench(L, max(3, args.steps // 4))

    serving = None
    if not (args.quick or args.no_serving):
        log("serving loop")
        serving = serving_bench(L, rates=(1_000, 2_000, 5_000, 10_000, 20_000, 35_000, 50_000))

    lbi_ab = wide = None
    if not args.quick:
        log("early abandoning inside LB_Improved, off and on")
        lbi_ab = lbi_abandon_bench(L)
        log("wide-band DTW (brute force, n=1024, w=102 and 205)")
        wide = strip_bench(L)

    triangle = None
    if not (args.quick or args.no_triangle):
        log("App. B triangle-inequality workload (100000 triples, n=100, unconstrained DTW)")
        triangle = triangle_bench(L, ctx)

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline")
        cpu = cpu_baseline(X, Ys, w, 1, gpu_idx)
        if accuracy.get("rw256_p1"):
            cpu["index_agreement"] = accuracy["rw256_p1"]["index_agreement"]
            cpu["index_agreement_over"] = "all 256 queries against the oracle's brute force (tests/golden)"

    step_ms = np.array(imp["step_ms"])
    out = {
        "metric": METRIC,
        "value": modes["improved"]["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": imp["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "random-walk 1-NN, DTW_1, n=256, database 100000, 256 queries per step, w=26, "
                               "two-pass LB_Keogh->LB_Improved->DTW", "N": N, "n": n, "Q": Q, "w": w, "p": 1, "k": 1},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes_p1": modes,
        "p2": p2,
        "pruning_p1": dict(pruned_keogh=float(st[:, 2].sum() / (N * Q)),
                           pruned_improved=float(st[:, 3].sum() / (N * Q)),
                           dtw_fraction=float(st[:, 4].sum() / (N * Q)),
                           abandoned_fraction_of_dtw=float(st[:, 5].sum() / max(1, st[:, 4].sum()))),
        "stage_ms_p1": stages,
        "headline_options": {"autotune": not args.no_autotune, "set": args.set, "tuned": knobs},
        "stage_rooflines_p1": stage_roofs,
        "accuracy_vs_oracle": accuracy,
        "lb_single_query_hbm": lbg,
        "pd_prefilter": pdb,
        "batch_latency_ms": dict(p50=float(np.percentile(step_ms, 50)), p99=float(np.percentile(step_ms, 99))),
        "ragged": ragged,
        "shapes": shapes,
        "serving": serving,
        "triangle": triangle,
        "lbi_abandon": lbi_ab,
        "wide_band_dtw": wide,
    }
    print(json.dumps(out), flush=True)
    db.close()
    ctx.close()


if __name__ == "__main__":
    main()
