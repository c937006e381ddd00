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
HBM_PEAK_GBS = 8000.0

# Algorithmic floating-point work per unit of the TNN query kernel (counted
# from the source; FMA = 2): see the design notes.
FLOPS_BLOCK_BOUND = 20     # float32 box distance
FLOPS_SEG_BOUND = 39       # binary64 cylinder bound
FLOPS_POINT = 15           # binary64 exact distance


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-brute", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(queries shard across GPUs with a replicated index; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_10408_amd import capi, synth
    from paper_2112_10408_amd import tnn as T

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ps, qs, _, cfg = synth.make_config("c2")
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

    def plain():
        T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, out=out, scratch=scratch)

    ms_plain = timed(plain, args.steps, args.warmup, stream)
    log(f"plain TNN: {ms_plain:.3f} ms/step, {qs.n / ms_plain * 1e3:.0f} q/s")
    stats = T.new_stats()
    T.tnn_query(ix, qx, qy, qz, qt, scale, 0.0, k, stats=stats, out=out, scratch=scratch)
    torch.cuda.synchronize()
    st = T.stats_dict(stats)
    log("plain stats:", st)
    ref_idx = out[0].clone()

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

    flops = (FLOPS_BLOCK_BOUND * st["blocks"] + FLOPS_SEG_BOUND * st["segments"]
             + FLOPS_POINT * st["points"])
    achieved = flops / (ms_plain * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                "kernel": "tnn_query_kernel"}
    value = qs.n / ms_plain * 1e3
    res = {
        "metric": "exact k-NN queries/sec at 1M pts, k=32: learned+mixed TNN vs plain TNN vs brute",
        "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_plain, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1M trajectory points (5000x200), K=32, 100k sampled queries, k=32, "
                               "scales (1,1,10,0.05), mask t'<t",
                   "path": "plain TNN", "global_batch": qs.n, "seed": cfg["seed"]},
        "roofline": roofline,
        "plain_qps": value, "index_build_s": build_s, "stats": st,
    }
    res.update(result_extra)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(ps, qs, k, scale)
        log("cpu baseline:", res["cpu_baseline"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
