"""Benchmark: exact k-NN queries/s on one MI355X.

Workload (default): 1M synthetic trajectory points (5000 x 200, 3000 km box,
12 h), segment length 32, 100k queries sampled from the points, k = 32,
scales (1, 1, 10, 0.05), mask t' < t.  A step is one pass of the query path
over the whole query batch with the index and the inputs resident in HBM.
Prints one JSON line.
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

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CU x 64 lanes x 2.4 GHz x 2 (FMA)
FP32_VECTOR_PEAK_TFLOPS = 157.3  # twice the binary64 rate
HBM_PEAK_GBS = 8000.0

# Algorithmic work per unit of the TNN query kernel (the scope table's
# per-unit counts): a block bound is 20 float32 operations (4 gaps of 2 max
# each, 4 squares, 4 scaled terms summed), a cylinder bound 28 (differences,
# the scaled dot product and projection, the residual's scaled norm, square
# root, radius and time terms), a point 12 binary64 operations (4
# differences, 4 squares, 4 scaled terms summed) plus 2 float32 (the time
# mask and the admission compare).
FLOPS_BLOCK_BOUND = 20     # float32
FLOPS_SEG_BOUND = 28       # float32
FLOPS_POINT_F64 = 12       # binary64
FLOPS_POINT_F32 = 2        # float32

# The linear search on matrix cores: 16 algorithmic flop per (query, point)
# pair (the distance as an augmented 4-term dot product: 8 multiply-adds),
# against the dense BF16 MFMA peak (2.5 PFLOP/s).
FLOPS_PAIR_BF16 = 16
BF16_MFMA_PEAK_TFLOPS = 2500.0


# HBM traffic of one learned-radius search launch on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each
# scaled by what the counter reads for a 256 MiB device-to-device copy
# (FETCH_SIZE x 2.00, WRITE_SIZE x 1.00): 100,210 KiB fetched (x 2 = 205.2 MB)
# and 40,451 KiB written (41.4 MB).  It describes the kernel built from the
# sources with this SHA-256 (the search kernel's sources, the index build's
# ordering of segments and points, and the C header) only; after any change
# to them the figure is reported as null.
KERNEL_SOURCES = ("query.hip", "query.h", "bounds.h", "wave.h", "gka.h", "tnn_internal.h",
                  "build.hip", "host.cpp")
MEASURED_TRAFFIC = {
    "sha256": "37ee3f3e9fcf9e648d0f1adb2699adf1a87eae0df436fd356a4e1cede0a5248d",
    "bytes_per_launch": 246.6e6,
}


# Safety factor of the learned radius: the predicted k-th distance is scaled so
# that this fraction of the training queries' true k-th distances falls inside.
# With best-first expansion a generous radius costs little and a fallback
# (second round) costs more, so high quantiles win (a sweep on the training
# queries of the 1M-point workload picks 0.99; --radius-quantile 0 repeats it).
RADIUS_QUANTILES = (0.9, 0.95, 0.98, 0.99, 0.995)
# A learned setting must beat plain TNN on the training queries by this much
# to be kept (about the spread of repeated timings of a 0.2-0.3 ms call).
LEARNED_MARGIN = 0.02
BATCH_QUANTILE = 0.99


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2112_10408_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "tnn.h"), "rb") as fh:
        h.update(fh.read())
    return MEASURED_TRAFFIC["bytes_per_launch"] if h.hexdigest() == MEASURED_TRAFFIC["sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def scratch_for(T, capi, ix, n, scale, tw, k, model=None):
    """Scratch for plain TNN and for the learned search with the radius
    predicted inside the call (the larger of the two workspaces)."""
    import torch
    need = T.tnn_query_workspace(ix, n, T.make_params(scale, tw, k))
    if model is not None:
        need = max(need, T.tnn_query_workspace(
            ix, n, T.make_params(scale, tw, k, capi.TNN_LEARNED, radius_model=model)))
    return torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")


def strategy_name(capi, flags):
    if not flags & capi.TNN_LEARNED:
        return "plain (the learned radius did not pay on the training queries)"
    return "learned radius + plain seed" if flags & capi.TNN_LEARNED_SEED else "learned radius"


STRATEGY = "auto"  # --radius-strategy


def choose_radius(T, capi, radius, model, ptr, pdist, ix, scale, tw, k, quantiles, stream,
                  steps=3, warmup=1, query_scale=None):
    """Calibration of the learned radius on the training queries (setup, not
    timed): for each quantile of the safety factor, and with and without the
    plain seed (TNN_LEARNED_SEED), time radius inference + learned search on
    the training queries; plain TNN (no inference) is timed as well, and the
    fastest learned setting replaces it only when it is faster by more than
    LEARNED_MARGIN (the timing noise of these short calls), so the learned
    path is not chosen where it does not pay.  Returns (ms, quantile, alpha,
    flags); flags 0 means plain TNN was kept."""
    import torch
    n = ptr[0].shape[0]
    out = (torch.empty((n, k), dtype=torch.int32, device="cuda"),
           torch.empty((n, k), dtype=torch.float64, device="cuda"))
    scr = scratch_for(T, capi, ix, n, scale, tw, k, model)

    def run_plain():
        T.tnn_query(ix, *ptr, scale, tw, k, out=out, scratch=scr, query_scale=query_scale)

    best = None
    if STRATEGY in ("auto", "plain"):
        ms = timed(run_plain, steps, warmup, stream)
        log(f"  plain TNN: {ms:.3f} ms on the training queries")
        best = (ms, None, 1.0, 0)
    best_learned = None
    flag_sets = {"auto": (capi.TNN_LEARNED, capi.TNN_LEARNED | capi.TNN_LEARNED_SEED),
                 "plain": (), "learned": (capi.TNN_LEARNED,),
                 "seeded": (capi.TNN_LEARNED | capi.TNN_LEARNED_SEED,)}[STRATEGY]
    for qnt in (quantiles if flag_sets else ()):
        a = radius.calibrate(model, *ptr, pdist, k, quantile=qnt)
        for fl in flag_sets:
            def run():  # radius predicted inside the call
                T.tnn_query(ix, *ptr, scale, tw, k, flags=fl, radius_model=model, radius_alpha=a,
                            out=out, scratch=scr, query_scale=query_scale)
            ms = timed(run, steps, warmup, stream)
            log(f"  quantile {qnt}, {'seeded' if fl & capi.TNN_LEARNED_SEED else 'unseeded'}: "
                f"alpha {a:.3f}, {ms:.3f} ms on the training queries")
            if best_learned is None or ms < best_learned[0]:
                best_learned = (ms, qnt, a, fl)
    if best is None:
        return best_learned
    if best_learned is not None and best_learned[0] < best[0] * (1.0 - LEARNED_MARGIN):
        return best_learned
    return best


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per step


def cpu_baseline(ps, qs, k, scale, budget_s=15.0):
    """The oracle (C, OpenMP, binary64 brute force) on a bounded sample of the
    same queries, timed on the host cores."""
    import oracle
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    omp = int(os.environ.get("OMP_NUM_THREADS", cores))
    threads = min(cores, omp)
    n_try = 256
    t0 = time.perf_counter()
    oracle.knn(ps.soa(), qs.take(np.arange(n_try)).soa(), scale, 0.0, k)
    dt = time.perf_counter() - t0
    n = int(min(qs.n, max(n_try, n_try * budget_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    oracle.knn(ps.soa(), qs.take(np.arange(n)).soa(), scale, 0.0, k)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of the {qs.n} queries against all {ps.n} points, "
                      f"{dt:.1f} s wall"}


def run_batched(args, T, capi, radius, synth, torch, stream):
    """64 independent airspaces (log-uniform sizes, k in {8, 32, 64}), each
    with its own index and learned radius; the step (per-airspace radius
    inference + one persistent batched search) is captured in a HIP graph."""
    scale = synth.SCALE
    t0 = time.perf_counter()
    airs = synth.airspaces(args.airspaces)
    entries, models = [], []
    total_q = total_p = 0
    fallback_guess = []
    for a in airs:
        ps, qs = a["points"], a["queries"]
        x, y, z, t = T.to_device(ps.x, ps.y, ps.z, ps.t)
        ix = T.tnn_build_segments(x, y, z, t, ps.offsets, a["seg_len"], scale)
        ix._keep = (x, y, z, t)
        n_tr = min(20000, ps.n // 2)
        excl = a["qidx"] if ps.n - qs.n >= n_tr else None  # small airspace: queries cover it
        tq, _ = synth.sample_queries(ps, n_tr, 77, exclude=excl)
        tx = T.to_device(tq.x, tq.y, tq.z, tq.t)
        model, _, pdist, ptr = radius.train(ix, *tx, scale, 0.0, a["k"], epochs=4, batch=2048)
        alpha = radius.calibrate(model, *ptr, pdist, a["k"], quantile=BATCH_QUANTILE)
        q = T.to_device(qs.x, qs.y, qs.z, qs.t)
        r2 = torch.empty(qs.n, dtype=torch.float32, device="cuda")
        entries.append(dict(index=ix, q=q, scale=scale, k=a["k"], flags=capi.TNN_LEARNED, radius2=r2))
        models.append((model, alpha, q, r2))
        total_q += qs.n
        total_p += ps.n
    setup_s = time.perf_counter() - t0
    best = T.tnn_autotune_batched(entries, None)
    b = T.tnn_batch_prepare(entries, best)

    # the per-airspace radius inferences are independent: spread them over a
    # few streams forked from the launch stream (parallel graph branches)
    infer_streams = [torch.cuda.Stream() for _ in range(4)]

    def step():
        main = torch.cuda.current_stream()
        for s in infer_streams:
            s.wait_stream(main)
        for i, (model, alpha, q, r2) in enumerate(models):
            with torch.cuda.stream(infer_streams[i % len(infer_streams)]):
                T.tnn_radius_infer(model, *q, alpha, out=r2)
        for s in infer_streams:
            main.wait_stream(s)
        T.tnn_query_batched(b)

    step()
    torch.cuda.synchronize()
    # exactness: every airspace against its own plain TNN search
    exact = True
    for e, out in zip(entries, b.outs):
        pi, pd = T.tnn_query(e["index"], *e["q"], scale, 0.0, e["k"])
        exact &= bool(torch.equal(pi, out[0])) and bool(torch.equal(pd, out[1]))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    ms = timed(g.replay, args.steps, args.warmup, stream)
    g.replay()
    torch.cuda.synchronize()
    ticks = T.tnn_batch_ticks(b).cpu().numpy().astype(np.float64)
    khz = T.tnn_wall_clock_rate_khz()
    lat_ms = [(ticks[i + 1] - ticks[0]) / khz for i in range(len(entries)) if entries[i]["q"][0].shape[0]]
    lat_ms = np.array(lat_ms)
    out = {"workload": f"{len(entries)} airspaces, {total_p} points, {total_q} queries, "
                       "k in {8,32,64}, learned radius, one persistent graph-captured launch",
           "queries_per_s": total_q / ms * 1e3, "ms_per_step": ms,
           "airspace_latency_ms_p50": float(np.percentile(lat_ms, 50)),
           "airspace_latency_ms_p99": float(np.percentile(lat_ms, 99)),
           "autotuned_chunk_waves_blocks": list(best), "exact_vs_plain": exact,
           "setup_s": setup_s}
    log("batched:", out)
    return out


def run_config(name, args, T, capi, radius, synth, torch, stream):
    """One of the other synthetic workloads: plain TNN, learned-radius TNN
    (trained on queries disjoint from the test queries where the data allow),
    BF16 MFMA brute force with binary64 rescoring and, where it finishes in
    seconds, binary64 brute force.  Every path is checked against plain TNN."""
    scale = synth.SCALE
    ps, qs, qidx, cfg = synth.make_config(name)
    k, K, tw = cfg["k"], cfg["seg_len"], cfg["t_window"]
    x, y, z, t = T.to_device(ps.x, ps.y, ps.z, ps.t)
    q = T.to_device(qs.x, qs.y, qs.z, qs.t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = T.tnn_build_segments(x, y, z, t, ps.offsets, K, scale)
    build_s = time.perf_counter() - t0
    n = qs.n
    out = (torch.empty((n, k), dtype=torch.int32, device="cuda"),
           torch.empty((n, k), dtype=torch.float64, device="cuda"))
    scratch = scratch_for(T, capi, ix, n, scale, tw, k)
    steps = max(1, min(args.steps, 5))
    res = {"points": ps.n, "queries": n, "k": k, "seg_len": K, "t_window": tw,
           "index_build_s": build_s}

    def plain():
        T.tnn_query(ix, *q, scale, tw, k, out=out, scratch=scratch)

    ms = timed(plain, steps, 1, stream)
    # small workloads take well under a millisecond per call: time enough calls
    # that each measurement spans about 20 ms
    steps = int(min(200, max(steps, 20.0 / max(ms, 1e-3))))
    ms = timed(plain, steps, 1, stream)
    ref = (out[0].clone(), out[1].clone())
    res["plain_qps"] = n / ms * 1e3
    # learned radius
    if "train_idx" in cfg:
        tq = ps.take(cfg["train_idx"])
    else:
        n_tr = min(100_000, ps.n // 2)
        tq, _ = synth.sample_queries(ps, n_tr, cfg["seed"] + 2000,
                                     exclude=qidx if ps.n - n >= n_tr else None)
    tx = T.to_device(tq.x, tq.y, tq.z, tq.t)
    t0 = time.perf_counter()
    model, loss, pdist, ptr = radius.train(ix, *tx, scale, tw, k, epochs=args.train_epochs,
                                           batch=4096, lr=3e-3)
    torch.cuda.synchronize()
    res["radius_train_s"] = time.perf_counter() - t0
    res["radius_train_queries"] = tq.n
    best = choose_radius(T, capi, radius, model, ptr, pdist, ix, scale, tw, k,
                         RADIUS_QUANTILES if not args.radius_quantile else (args.radius_quantile,),
                         stream, steps=2)
    alpha, lflags = best[2], best[3]
    scratch = scratch_for(T, capi, ix, n, scale, tw, k, model)

    def learned(**kw):  # the radius predicted inside the call
        T.tnn_query(ix, *q, scale, tw, k, flags=lflags, radius_model=model if lflags else None,
                    radius_alpha=alpha, out=out, scratch=scratch, **kw)

    ms_l = timed(learned, steps, 1, stream)
    st = T.new_stats()
    learned(stats=st)
    torch.cuda.synchronize()
    st = T.stats_dict(st)
    res.update(learned_qps=n / ms_l * 1e3, learned_speedup_vs_plain=ms / ms_l,
               learned_matches_plain=bool(torch.equal(out[0], ref[0])) and bool(torch.equal(out[1], ref[1])),
               fallback_rate=st["fallbacks"] / max(n, 1), radius_quantile=best[1], radius_alpha=alpha,
               radius_strategy=strategy_name(capi, lflags),
               work_per_query_learned={kk: st[kk] / max(n, 1) for kk in ("blocks", "segments", "points", "merges")})
    if not args.no_brute:
        mf = capi.TNN_BRUTE | capi.TNN_MIXED_BF16
        mscr = torch.empty(T.tnn_query_workspace(ix, n, T.make_params(scale, tw, k, mf)),
                           dtype=torch.uint8, device="cuda")

        def mixed():
            T.tnn_query(ix, *q, scale, tw, k, flags=mf, out=out, scratch=mscr)

        ms_m = timed(mixed, 1, 1, stream)
        mst = T.new_stats()
        T.tnn_query(ix, *q, scale, tw, k, flags=mf, out=out, scratch=mscr, stats=mst)
        torch.cuda.synchronize()
        mst = T.stats_dict(mst)
        res.update(mixed_brute_qps=n / ms_m * 1e3,
                   mixed_brute_exact=bool(torch.equal(out[0], ref[0])) and bool(torch.equal(out[1], ref[1])),
                   mixed_brute_rescored_per_query=mst["rescored"] / max(n, 1),
                   mixed_max_abs_dist_err=mst["max_err"],
                   mixed_pairs_scanned_frac=mst["points"] / max(float(ps.n) * n, 1.0))
        del mscr
        if float(ps.n) * n <= 2e12:
            def brute():
                T.tnn_query(ix, *q, scale, tw, k, flags=capi.TNN_BRUTE, out=out, scratch=scratch)

            ms_b = timed(brute, 1, 1, stream)
            res.update(brute_qps=n / ms_b * 1e3,
                       brute_matches_tnn=bool(torch.equal(out[0], ref[0])))
            res["learned_speedup_vs_brute"] = ms_b / ms_l
        res["learned_speedup_vs_mixed_brute"] = ms_m / ms_l
    log(f"{name}:", res)
    return res


def run_query_scales(args, T, capi, radius, synth, torch, stream):
    """The 1M-point, 100k-query workload with scales that vary over space
    (one row per query, within exp(+-0.7) of the shared scales): plain TNN,
    learned-radius TNN (radius trained under the shared scales, so only a
    rough guess here: exact either way) and binary64 brute force under the
    same per-query metric."""
    scale = synth.SCALE
    ps, qs, qidx, cfg = synth.make_config("c2")
    k, K, tw = cfg["k"], cfg["seg_len"], cfg["t_window"]
    x, y, z, t = T.to_device(ps.x, ps.y, ps.z, ps.t)
    q = T.to_device(qs.x, qs.y, qs.z, qs.t)
    rows = synth.scale_field(qs.x, qs.y, qs.z, 3000.0, seed=cfg["seed"] + 77)
    qscale = torch.from_numpy(rows).cuda()
    ix = T.tnn_build_segments(x, y, z, t, ps.offsets, K, scale)
    n = qs.n
    out = (torch.empty((n, k), dtype=torch.int32, device="cuda"),
           torch.empty((n, k), dtype=torch.float64, device="cuda"))
    scratch = torch.empty(max(T.tnn_query_workspace(ix, n, T.make_params(scale, tw, k)), 256),
                          dtype=torch.uint8, device="cuda")
    steps = max(1, min(args.steps, 5))
    res = {"points": ps.n, "queries": n, "k": k, "seg_len": K,
           "scales": "per query, exp(+-0.7) smooth field around (1, 1, 10, 0.05)"}

    def plain():
        T.tnn_query(ix, *q, scale, tw, k, out=out, scratch=scratch, query_scale=qscale)

    ms = timed(plain, steps, 1, stream)
    ref = (out[0].clone(), out[1].clone())
    res["plain_qps"] = n / ms * 1e3
    n_tr = min(100_000, ps.n // 2)
    tq, _ = synth.sample_queries(ps, n_tr, cfg["seed"] + 2000, exclude=qidx)
    tx = T.to_device(tq.x, tq.y, tq.z, tq.t)
    model, loss, pdist, ptr = radius.train(ix, *tx, scale, tw, k, epochs=args.train_epochs,
                                           batch=4096, lr=3e-3)
    # (the training queries' scales: the same field at their own positions)
    tr_rows = torch.from_numpy(synth.scale_field(tq.x, tq.y, tq.z, 3000.0, seed=cfg["seed"] + 77)).cuda()
    best = choose_radius(T, capi, radius, model, ptr, pdist, ix, scale, tw, k, (BATCH_QUANTILE,),
                         stream, steps=2, query_scale=tr_rows)
    alpha, lflags = best[2], best[3]
    scratch = scratch_for(T, capi, ix, n, scale, tw, k, model)

    def learned(**kw):  # the radius predicted inside the call
        T.tnn_query(ix, *q, scale, tw, k, flags=lflags, radius_model=model if lflags else None,
                    radius_alpha=alpha, out=out, scratch=scratch, query_scale=qscale, **kw)

    ms_l = timed(learned, steps, 1, stream)
    st = T.new_stats()
    learned(stats=st)
    torch.cuda.synchronize()
    st = T.stats_dict(st)
    res.update(learned_qps=n / ms_l * 1e3, learned_speedup_vs_plain=ms / ms_l,
               learned_matches_plain=bool(torch.equal(out[0], ref[0])) and bool(torch.equal(out[1], ref[1])),
               fallback_rate=st["fallbacks"] / max(n, 1), radius_strategy=strategy_name(capi, lflags))
    if not args.no_brute:
        def brute():
            T.tnn_query(ix, *q, scale, tw, k, flags=capi.TNN_BRUTE, out=out, scratch=scratch,
                        query_scale=qscale)

        ms_b = timed(brute, 1, 1, stream)
        res.update(brute_qps=n / ms_b * 1e3,
                   brute_matches_tnn=bool(torch.equal(out[0], ref[0])) and bool(torch.equal(out[1], ref[1])),
                   learned_speedup_vs_brute=ms_b / ms_l)
    log("scales:", res)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-brute", action="store_true")
    ap.add_argument("--train-queries", type=int, default=100_000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--airspaces", type=int, default=64)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (10k points, 1M queries, 8M points, "
                         "30-min window, airways, random points, per-query scales)")
    ap.add_argument("--train-epochs", type=int, default=8)
    ap.add_argument("--radius-quantile", type=float, default=0.99,
                    help="calibration quantile of the radius safety factor (default 0.99); "
                         "0 sweeps 0.9-0.995 and keeps the fastest on the training queries")
    ap.add_argument("--radius-strategy", default="auto",
                    choices=("auto", "plain", "learned", "seeded"),
                    help="auto (default): the fastest of plain TNN, learned radius and learned "
                         "radius + plain seed on the training queries; the others force one "
                         "(profilers distort the timing the automatic choice relies on)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    global STRATEGY
    STRATEGY = args.radius_strategy
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(queries shard across GPUs with a replicated index; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_10408_amd import capi, radius, synth
    from paper_2112_10408_amd import tnn as T

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ps, qs, qidx, cfg = synth.make_config("c2")
    k, K, scale = cfg["k"], cfg["seg_len"], synth.SCALE
    log(f"workload: {ps.n} points, {qs.n} queries, k={k}, K={K}")
    x, y, z, t = T.to_device(ps.x, ps.y, ps.z, ps.t)
    qx, qy, qz, qt = T.to_device(qs.x, qs.y, qs.z, qs.t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = T.tnn_build_segments(x, y, z, t, ps.offsets, K, scale)
    build_s = time.perf_counter() - t0
    log(f"index: {ix.n_segments} segments, {ix.n_blocks} blocks, build {build_s:.3f} s")

    out = (torch.empty((qs.n, k), dtype=torch.int32, device="cuda"),
           torch.empty((qs.n, k), dtype=torch.float64, device="cuda"))
    p_plain = T.make_params(scale, 0.0, k)
    scratch = torch.empty(max(T.tnn_query_workspace(ix, qs.n, p_plain), 256), dtype=torch.uint8,
                          device="cuda")

    # ---- plain TNN ----------------------------------------------------------
    def plain():
        T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, out=out, scratch=scratch)

    ms_plain = timed(plain, args.steps, args.warmup, stream)
    log(f"plain TNN: {ms_plain:.3f} ms/step, {qs.n / ms_plain * 1e3:.0f} q/s")
    stats = T.new_stats()
    T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, stats=stats, out=out, scratch=scratch)
    torch.cuda.synchronize()
    st_plain = T.stats_dict(stats)
    log("plain stats:", st_plain)
    ref_idx = out[0].clone()
    ref_dist = out[1].clone()

    # ---- learned radius: train on the method's own output (setup, untimed) --
    tq, _ = synth.sample_queries(ps, args.train_queries, cfg["seed"] + 2000, exclude=qidx)
    tx, ty, tz, tt = T.to_device(tq.x, tq.y, tq.z, tq.t)
    t0 = time.perf_counter()
    model, loss, pdist, ptr = radius.train(ix, tx, ty, tz, tt, scale, 0.0, k,
                                           epochs=args.train_epochs, batch=4096, lr=3e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"radius model: {args.train_queries} labelled queries, loss {loss:.4f}, {train_s:.2f} s")
    r2 = torch.empty(qs.n, dtype=torch.float32, device="cuda")
    # safety factor (and whether to also take the plain seed): the choice whose
    # learned search is fastest on the training queries
    sweep = RADIUS_QUANTILES if not args.radius_quantile else (args.radius_quantile,)
    best = choose_radius(T, capi, radius, model, ptr, pdist, ix, scale, 0.0, k, sweep, stream,
                         steps=5, warmup=2)
    alpha, lflags = best[2], best[3]

    # ---- learned TNN: the headline step (radius inference + search) ---------
    # one call: the library predicts the radius in the launch of its per-call
    # preparation, then searches
    scratch = scratch_for(T, capi, ix, qs.n, scale, 0.0, k, model)

    def learned(**kw):
        T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, flags=lflags,
                    radius_model=model if lflags else None, radius_alpha=alpha, out=out,
                    scratch=scratch, **kw)

    ms_learned = timed(learned, args.steps, args.warmup, stream)

    # the search alone (radius predicted beforehand, not timed): the time the
    # roofline of the search kernel is taken over
    if lflags:
        T.tnn_radius_infer(model, qx, qy, qz, qt, alpha, out=r2)

    def learned_search_only(**kw):
        T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, flags=lflags, radius2=r2 if lflags else None,
                    out=out, scratch=scratch, **kw)

    ms_search = timed(learned_search_only, args.steps, 1, stream)
    exact = bool(torch.equal(out[0], ref_idx)) and bool(torch.equal(out[1], ref_dist))
    stats = T.new_stats()
    learned(stats=stats)
    torch.cuda.synchronize()
    st = T.stats_dict(stats)
    exact = exact and bool(torch.equal(out[0], ref_idx)) and bool(torch.equal(out[1], ref_dist))
    log(f"learned TNN: {ms_learned:.3f} ms/step ({ms_search:.3f} ms search), "
        f"{qs.n / ms_learned * 1e3:.0f} q/s, same as plain {exact}, fallbacks {st['fallbacks']}")
    log("learned stats:", st)

    # ---- Gaussian kernel averaging over the context (Sec. 3.2, Eq. gka) ----
    # synthetic 2-component wind measurements, one per point
    wind = torch.from_numpy(np.random.default_rng(cfg["seed"] + 3000)
                            .normal(0.0, 15.0, (ps.n, 2)).astype(np.float32)).cuda()
    gka_out = torch.empty((qs.n, 2), dtype=torch.float64, device="cuda")
    learned()
    ms_gka = timed(lambda: T.tnn_gka_average(out[0], out[1], wind, out=gka_out), args.steps, 1,
                   stream)
    gka_sep = gka_out.clone()

    # the averaging asked of the same call: the library runs the averaging
    # kernel on the call's stream right after the search; the learned step is
    # timed again beside it, so that the difference is not a drift of clocks
    # over the run
    def learned_gka():
        learned(gka_values=wind, gka_out=gka_out)

    ms_learned_ref = timed(learned, args.steps, 1, stream)
    ms_learned_gka = timed(learned_gka, args.steps, 1, stream)
    # byte comparison: queries without a past have NaN rows on both sides
    gka_in_call_same = gka_out.cpu().numpy().tobytes() == gka_sep.cpu().numpy().tobytes()
    log(f"GKA average kernel: {ms_gka:.3f} ms; learned TNN with the averaging in the call "
        f"{ms_learned_gka:.3f} ms/step against {ms_learned_ref:.3f} without "
        f"(same as the kernel: {gka_in_call_same})")

    if args.calib_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    result_extra = {}
    if not args.no_brute:
        bsteps = max(1, min(args.steps, 3))

        def brute():
            T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, flags=capi.TNN_BRUTE, out=out, scratch=scratch)

        ms_brute = timed(brute, bsteps, 1, stream)
        same = bool(torch.equal(out[0], ref_idx))
        log(f"brute: {ms_brute:.3f} ms/step, {qs.n / ms_brute * 1e3:.0f} q/s, same idx {same}")
        result_extra["brute_qps"] = qs.n / ms_brute * 1e3
        result_extra["brute_matches_tnn"] = same

        def mixed():
            T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, flags=capi.TNN_BRUTE | capi.TNN_MIXED_BF16,
                        out=out, scratch=mscratch)

        mp = T.make_params(scale, 0.0, k, capi.TNN_BRUTE | capi.TNN_MIXED_BF16)
        mscratch = torch.empty(T.tnn_query_workspace(ix, qs.n, mp), dtype=torch.uint8, device="cuda")
        ms_mixed = timed(mixed, bsteps, 1, stream)
        same_m = bool(torch.equal(out[0], ref_idx)) and bool(torch.equal(out[1], ref_dist))
        mstats = T.new_stats()
        T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, flags=capi.TNN_BRUTE | capi.TNN_MIXED_BF16,
                    out=out, scratch=mscratch, stats=mstats)
        torch.cuda.synchronize()
        mst = T.stats_dict(mstats)
        log(f"mixed brute (BF16 MFMA + binary64 rescoring): {ms_mixed:.3f} ms/step, "
            f"{qs.n / ms_mixed * 1e3:.0f} q/s, exact {same_m}, rescored {mst['rescored']}, "
            f"max |approx - exact| {mst['max_err']:.3g}")
        result_extra["mixed_brute_qps"] = qs.n / ms_mixed * 1e3
        result_extra["mixed_brute_exact"] = same_m
        result_extra["mixed_brute_rescored_per_query"] = mst["rescored"] / qs.n
        result_extra["mixed_max_abs_dist_err"] = mst["max_err"]
        # Roofline of the BF16 linear search at 16 algorithmic flop per (query,
        # point) pair: the pairs of the stages it scans (the pilot pass's
        # included; stages a query tile's time mask rejects entirely are
        # skipped), over the whole call (home blocks, pilot, MFMA scan, merge).
        pairs = mst["points"]
        result_extra["mixed_brute_roofline"] = {
            "bound": "mfma", "unit": "TFLOP/s", "peak": BF16_MFMA_PEAK_TFLOPS,
            "flop_per_pair": FLOPS_PAIR_BF16, "pairs": pairs, "pairs_all": qs.n * ps.n,
            "achieved": FLOPS_PAIR_BF16 * pairs / (ms_mixed * 1e-3) / 1e12,
            "frac": FLOPS_PAIR_BF16 * pairs / (ms_mixed * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS,
            "achieved_all_pairs": FLOPS_PAIR_BF16 * qs.n * ps.n / (ms_mixed * 1e-3) / 1e12,
            "call_ms": ms_mixed}

    f32 = (FLOPS_BLOCK_BOUND * st["blocks"] + FLOPS_SEG_BOUND * st["segments"]
           + FLOPS_POINT_F32 * st["points"])
    f64 = FLOPS_POINT_F64 * st["points"]
    flops = f32 + f64
    achieved = flops / (ms_search * 1e-3) / 1e12
    # ALU roof of this float32/binary64 mix: the time the flops take at the
    # two vector peaks, expressed as one rate
    peak = flops / (f32 / FP32_VECTOR_PEAK_TFLOPS + f64 / FP64_VECTOR_PEAK_TFLOPS)
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic(),
                "kernel": "tnn_query_lds_kernel (learned radius; the timed call also runs the per-call prep_kernel)",
                "kernel_ms": ms_search}
    value = qs.n / ms_learned * 1e3
    res = {
        "metric": "exact k-NN queries/sec at 1M pts, k=32: learned+mixed TNN vs plain TNN vs brute",
        "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_learned, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1M trajectory points (5000x200), K=32, 100k sampled queries, k=32, "
                               "scales (1,1,10,0.05), mask t'<t",
                   "path": ("TNN, " + strategy_name(capi, lflags)
                            + (" (radius inference + search)" if lflags else "")
                            + "; binary64 point scan (the BF16 MFMA tiles serve the linear "
                              "search baseline)"),
                   "global_batch": qs.n, "seed": cfg["seed"]},
        "roofline": roofline,
        "plain_qps": qs.n / ms_plain * 1e3, "learned_qps": value,
        "learned_speedup_vs_plain": ms_plain / ms_learned,
        "learned_matches_plain": exact, "fallback_rate": st["fallbacks"] / qs.n,
        "gka_average_ms": ms_gka, "learned_plus_gka_qps": qs.n / ms_learned_gka * 1e3,
        "learned_plus_gka_ms_per_step": ms_learned_gka,
        "gka_added_ms": ms_learned_gka - ms_learned_ref,
        "gka_in_call_matches_kernel": gka_in_call_same,
        "radius_alpha": alpha, "radius_quantile": best[1],
        "radius_strategy": strategy_name(capi, lflags), "radius_train_s": train_s,
        "radius_train_queries": args.train_queries,
        "index_build_s": build_s, "stats_learned": st, "stats_plain": st_plain,
    }
    res.update(result_extra)
    if not args.no_configs:
        res["configs"] = {}
        for name, label in (("c1", "10k_points_k8"), ("c3", "1M_points_1M_queries_k32"),
                            ("c4", "8M_points_1M_queries_k64"),
                            ("c2w", "1M_points_100k_queries_k32_window_30min"),
                            ("routes", "1M_points_40_airways_100k_queries_k32"),
                            ("rand", "1M_random_points_100k_queries_k32")):
            res["configs"][label] = run_config(name, args, T, capi, radius, synth, torch, stream)
            torch.cuda.empty_cache()
        res["configs"]["1M_points_100k_queries_k32_per_query_scales"] = run_query_scales(
            args, T, capi, radius, synth, torch, stream)
        torch.cuda.empty_cache()
    if not args.no_batched:
        res["batched"] = run_batched(args, T, capi, radius, synth, torch, stream)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(ps, qs, k, scale)
        log("cpu baseline:", res["cpu_baseline"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
