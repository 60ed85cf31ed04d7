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
# fp32 vector peak 157.3 TFLOP/s counts an FMA as 2 flops: 78.6e12 VALU lane-slots per second
# (256 CUs x 128 lane-ops per clock x 2.4 GHz).  One LB_Keogh element is 2 comparisons (one
# 3-operand med3, which issues in two slots), a subtract and an accumulate: 4 slots.  A DTW cell
# is a subtract, a 3-way min (two slots) and an accumulate: 4 slots.
VALU_PEAK_OPS = 157.3e12 / 2
HBM_PEAK_GBPS = 8000.0
LBK_OPS_PER_ELEM = 4
DTW_OPS_PER_CELL = 4


def sweep_traffic():
    """HBM bytes per sweep launch from the committed PMC summary, if it was taken on the
    current sweep kernel source (else None)."""
    import hashlib
    src = os.path.join(ROOT, "paper_0811_3301_amd", "csrc", "kernels_lb.hip")
    prof = os.path.join(ROOT, "profiles", "lbk_sweep_rw256_traffic.md")
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
    import torch
    for _ in range(warmup):
        L.lbimp_nn_search(ctx, db, Yd, w, p, 1, mode, stats=False)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per = []
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        a = time.perf_counter()
        L.lbimp_nn_search(ctx, db, Yd, w, p, 1, mode, stats=False)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - a) * 1e3)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    return dict(ms_per_step=ev_ms / steps, wall_ms_per_step=wall * 1e3 / steps, step_ms=per)


def stage_profile(L, ctx, db, Yd, w, p, mode, steps):
    import torch
    L.lbimp_ctx_set_timing(ctx, True)
    acc = {}
    for _ in range(steps):
        L.lbimp_nn_search(ctx, db, Yd, w, p, 1, mode, stats=False)
        for k, v in L.lbimp_ctx_stage_times(ctx).items():
            acc[k] = acc.get(k, 0.0) + v
    L.lbimp_ctx_set_timing(ctx, False)
    torch.cuda.synchronize()
    return {k: v / steps for k, v in acc.items()}


def single_query_lb_gbps(L, ctx, steps=20):
    """LB_Keogh of one query over a 1,000,000 x 128 random-walk database (512 MB, larger than
    the 256 MB Infinity Cache): the HBM-bound form of the first pass."""
    import torch
    from paper_0811_3301_amd import gen
    N, n, w = 1_000_000, 128, 13
    g = gen.rng(5, gen.ROLE_DB)
    X = torch.from_numpy(gen.random_walk(N, n, g).astype(np.float32)).cuda()
    db = L.Db(ctx, X)
    del X
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
    db.close()
    nbytes = N * n * 4
    return dict(db_bytes=nbytes, ms=ms, gbps=nbytes / ms / 1e6, frac_hbm=nbytes / ms / 1e6 / HBM_PEAK_GBPS)


def cpu_baseline(X, Ys, w, p, gpu_idx, budget_s=12.0):
    """The fp64 oracle (brute-force DTW over the whole database) on a bounded sample of queries."""
    from oracle import native
    native.load()
    X64 = X.astype(np.float64)
    t = time.perf_counter()
    idx, _ = native.nn_bruteforce(X64, Ys[:1].astype(np.float64), w, p, 1)
    first = time.perf_counter() - t
    more = int(max(0, min(Ys.shape[0] - 1, budget_s / max(first, 1e-3) - 1)))
    t = time.perf_counter()
    idx2, _ = native.nn_bruteforce(X64, Ys[1:1 + more].astype(np.float64), w, p, 1)
    rest = time.perf_counter() - t
    nq = 1 + more
    total = first + rest
    allidx = np.concatenate([idx[:, 0], idx2[:, 0]]) if more else idx[:, 0]
    agree = float(np.mean(allidx == gpu_idx[:nq]))
    return dict(value=nq / total, unit="queries/s", cores=native.num_threads(), kind="oracle",
                sample=f"{nq} of {Ys.shape[0]} queries, brute-force fp64 DTW against all {X.shape[0]} candidates",
                seconds=total, index_agreement=agree)


def ragged_bench(L, steps, warmup):
    """Uneven batch: 4,096 random-walk queries, lengths uniform over {64,...,1024}, w = round(f n)
    with f uniform over {0.05, 0.1, 0.2}, one 20,000-series database per length, p = 1, 1-NN,
    one lbimp_nn_search_ragged call per step (captured once as a HIP graph, then replayed).  The
    context autotunes every group on the first (untimed) call."""
    import torch
    from paper_0811_3301_amd import gen
    ctx = L.Ctx(0)
    L.lbimp_ctx_set_option(ctx, "autotune", 1)
    dbs, qs, db_of, w = gen.make_ragged_workload()
    handles = [L.Db(ctx, torch.from_numpy(d.astype(np.float32)).cuda()) for d in dbs]
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
                queries=Q, groups=len(set(zip(db_of.tolist(), w.tolist()))), autotuned=True, **out,
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
            r[mode] = dict(qps=Q / (t["ms_per_step"] / 1e3), ms_per_step=t["ms_per_step"])
        _, _, st = L.lbimp_nn_search(ctx, db, Yd, w, 1, 1, "improved")
        r["pruned_keogh"] = float(st[:, 2].sum() / (N * Q))
        r["pruned_improved"] = float(st[:, 3].sum() / (N * Q))
        r["dtw_fraction"] = float(st[:, 4].sum() / (N * Q))
        out[f"w{w}"] = r
    torch.cuda.synchronize()
    db.close()
    ctx.close()
    return out


def serving_bench(L, rates, seconds, max_batch=512, slots=4, budget=16 << 30):
    """Serving: Poisson arrivals over a resident 1,000,000 x 128 random-walk database (512 MB)
    and a 200,000 x 256 side database (20% of requests), w = round(0.1 n), k uniform over
    {1, 5, 10}; continuous batching on `slots` in-flight batches under a device-memory budget."""
    import torch
    from paper_0811_3301_amd import gen
    from paper_0811_3301_amd.serve import GpuExecutor, Request, serve
    dbs64, _ = gen.make_serving_workload(1.0, 1, with_databases=True)
    ctx = L.Ctx(0)
    handles = [L.Db(ctx, torch.from_numpy(d.astype(np.float32)).cuda()) for d in dbs64]
    del dbs64
    torch.cuda.synchronize()
    ex = GpuExecutor(handles, slots=slots, max_batch=max_batch, kmax=10)
    runs = []
    try:
        _, sample = gen.make_serving_workload(rates[-1], 300, with_databases=False)
        ex.pretune([Request(rid=j, t_arrive=0.0, db=int(sample["db"][j]), y=sample["y"][j].astype(np.float32),
                            w=int(sample["w"][j]), k=int(sample["k"][j])) for j in range(300)])
        for i, rate in enumerate([rates[-1]] + list(rates)):  # the first run warms the workspaces up
            count = max(200, min(int(rate * seconds), 40_000))
            _, req = gen.make_serving_workload(rate, count, with_databases=False)
            reqs = [Request(rid=j, t_arrive=float(req["t"][j]), db=int(req["db"][j]),
                            y=req["y"][j].astype(np.float32), w=int(req["w"][j]), k=int(req["k"][j]))
                    for j in range(count)]
            _, summ = serve(reqs, ex, budget_bytes=budget, max_batch=max_batch)
            if i > 0:
                summ["offered_rate"] = rate
                runs.append(summ)
                log(f"serving at {rate} q/s: p50 {summ['p50_ms']:.3f} ms, p99 {summ['p99_ms']:.3f} ms, "
                    f"{summ['qps']:.0f} q/s")
    finally:
        ex.close()
        for h in handles:
            h.close()
        ctx.close()
    return dict(workload="serving: Poisson arrivals, 80% n=128 over a resident 1,000,000-series database "
                         "(512 MB), 20% n=256 over a 200,000-series database, w=round(0.1 n), k in {1,5,10}, "
                         "two-pass search", slots=slots, max_batch=max_batch, memory_budget_bytes=budget,
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
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device-to-device copy (calibrates the PMC byte counters)")
    ap.add_argument("--only", choices=("ragged", "serving", "shapes"),
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
    if args.only == "serving":
        print(json.dumps(serving_bench(L, rates=(10_000,), seconds=0.3)), flush=True)
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
    L.lbimp_ctx_set_option(ctx, "autotune", 1)

    log("timing two-pass p=1")
    imp = time_mode(L, ctx, db, Yd, w, 1, "improved", args.steps, args.warmup)
    idx, dist, st = L.lbimp_nn_search(ctx, db, Yd, w, 1, 1, "improved")
    gpu_idx = idx.cpu().numpy()[:, 0]
    stages = stage_profile(L, ctx, db, Yd, w, 1, "improved", max(3, args.steps // 2))

    modes = {"improved": dict(qps=Q / (imp["ms_per_step"] / 1e3), ms_per_step=imp["ms_per_step"])}
    if not args.quick:
        for mode, steps in (("keogh", args.steps), ("brute", max(2, args.steps // 10))):
            log(f"timing {mode} p=1")
            r = time_mode(L, ctx, db, Yd, w, 1, mode, steps, 1)
            modes[mode] = dict(qps=Q / (r["ms_per_step"] / 1e3), ms_per_step=r["ms_per_step"])
            idx_m = L.lbimp_nn_search(ctx, db, Yd, w, 1, 1, mode, stats=False)[0].cpu().numpy()[:, 0]
            modes[mode]["same_result_as_two_pass"] = bool(np.array_equal(idx_m, gpu_idx))
        log("timing two-pass p=2")
        r2 = time_mode(L, ctx, db, Yd, w, 2, "improved", args.steps, 1)
        rk2 = time_mode(L, ctx, db, Yd, w, 2, "keogh", args.steps, 1)
        _, _, st2 = L.lbimp_nn_search(ctx, db, Yd, w, 2, 1, "improved")
        p2 = dict(improved_qps=Q / (r2["ms_per_step"] / 1e3), keogh_qps=Q / (rk2["ms_per_step"] / 1e3),
                  pruned_keogh=float(st2[:, 2].sum() / (N * Q)), pruned_improved=float(st2[:, 3].sum() / (N * Q)),
                  dtw_fraction=float(st2[:, 4].sum() / (N * Q)))
    else:
        p2 = None

    sweep_ms = stages["lb_keogh"]
    elems = Q * N * n
    achieved = LBK_OPS_PER_ELEM * elems / (sweep_ms / 1e3) / 1e12
    roofline = dict(bound="alu", kernel="k_lbk_sweep (LB_Keogh of every query x candidate)",
                    achieved=achieved, peak=VALU_PEAK_OPS / 1e12, unit="TOP/s", frac=achieved * 1e12 / VALU_PEAK_OPS,
                    traffic=sweep_traffic(), kernel_ms=sweep_ms, ops_per_element=LBK_OPS_PER_ELEM, elements=elems,
                    algorithmic_hbm_bytes=N * n * 4 * (Q // 16) + Q * ((N + 63) // 64 * 64) * 4)
    if "brute" in modes:
        cells = Q * N * (n * (2 * w + 1) - w * (w + 1))
        t = modes["brute"]["ms_per_step"] / 1e3
        modes["brute"]["dtw_cells_per_s"] = cells / t
        modes["brute"]["dtw_frac_of_alu_peak"] = DTW_OPS_PER_CELL * cells / t / VALU_PEAK_OPS

    lbg = None
    if not args.quick:
        log("single-query LB_Keogh sweep over a 512 MB database")
        lbg = single_query_lb_gbps(L, ctx)

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
        serving = serving_bench(L, rates=(1_000, 2_000, 5_000, 10_000, 20_000, 35_000, 50_000), seconds=0.5)

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline")
        cpu = cpu_baseline(X, Ys, w, 1, gpu_idx)

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
        "lb_single_query_hbm": lbg,
        "batch_latency_ms": dict(p50=float(np.percentile(step_ms, 50)), p99=float(np.percentile(step_ms, 99))),
        "ragged": ragged,
        "shapes": shapes,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    db.close()
    ctx.close()


if __name__ == "__main__":
    main()
