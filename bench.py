"""Benchmark: escape-time Mandelbrot on one MI355X.

Workload (the 8192 x 8192 full view): re in [-2, 1], im in [-1.2, 1.2], pixel
centres, R = 2, max_iter 10000, FP64, int32 counts.  One step = one
mandel_render of the whole view (the persistent FCFS tile kernel) with the
output already resident in HBM.  Reported value = pixel-iterations per second
(sum of the counts / step time).  FP64 FLOP/s counts 7 operations per
iteration (x*x, y*y, x*y, x2, -, +cx, +cy).

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz
FLOPS_PER_ITER = 7


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(view, rows_step: int, threads: int) -> dict:
    """The oracle (single-threaded loop per worker) on every rows_step-th row of the
    view, spread over `threads` host threads."""
    import numpy as np

    import oracle
    rows = np.arange(0, view.m, rows_step)
    idx = (rows[:, None] * view.n + np.arange(view.n)[None, :]).ravel()
    t0 = time.perf_counter()
    counts = oracle.render_pixels(view.window, view.m, view.n, view.max_iter, view.R, idx,
                                  threads=threads)
    dt = time.perf_counter() - t0
    return {"value": float(counts.sum(dtype=np.int64)) / dt, "unit": "pixel-iterations/s",
            "cores": threads, "kind": "oracle",
            "sample": f"rows i = 0 mod {rows_step} of the {view.m}x{view.n} view "
                      f"({len(rows)} rows, {idx.size} px, {int(counts.sum(dtype=np.int64))} "
                      f"iterations, {dt:.2f} s wall)",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=8192)
    ap.add_argument("--max-iter", type=int, default=10000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows-step", type=int, default=4)
    ap.add_argument("--block-iters", type=int, default=0)
    ap.add_argument("--young-iters", type=int, default=0)
    ap.add_argument("--waves-per-group", type=int, default=0)
    ap.add_argument("--check-every", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on a single GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2007_00745_amd import native, workloads

    native.lib()  # fails loudly when the library is missing
    view = workloads.c2(args.side, args.max_iter)
    torch.cuda.set_device(0)
    out = torch.empty((view.m, view.n), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    sched = dict(block_iters=args.block_iters, young_iters=args.young_iters,
                 waves_per_group=args.waves_per_group, check_every=args.check_every)

    def step():
        native.render_sched(view.window, view.m, view.n, view.max_iter, view.R, out=out,
                            stream=stream, **sched)

    log(f"bench: {view.m}x{view.n} max_iter {view.max_iter}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sum_counts = int(out.sum(dtype=torch.int64).item())
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    native.render_sched(view.window, view.m, view.n, view.max_iter, view.R, out=out,
                        stream=stream, stats=stats, **sched)
    torch.cuda.synchronize()
    st = [int(v) for v in stats.cpu().tolist()]
    lane_occ = st[1] / (64.0 * st[0]) if st[0] else None

    log(f"bench: timing {args.steps} steps")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in evs]
    ms_mean = sum(ms) / len(ms)
    sec = ms_mean / 1e3
    value = sum_counts / sec
    tflops = FLOPS_PER_ITER * sum_counts / sec / 1e12

    res = {
        "metric": "pixel-iterations/s (FP64)",
        "value": value,
        "unit": "pixel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mean,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"full view {view.m}x{view.n}, re[-2,1] x im[-1.2,1.2], "
                               f"R=2, max_iter {view.max_iter}",
                   "policy": "persistent FCFS tile queue, 64x8 tiles",
                   "parallelism": "single GPU"},
        "sum_counts": sum_counts,
        "fp64_tflops": tflops,
        "pct_fp64_peak": 100.0 * tflops / FP64_PEAK_TFLOPS,
        "lane_occupancy": lane_occ,
        "ms_min": min(ms),
        "wall_s": wall,
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / FP64_PEAK_TFLOPS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"bench: cpu baseline on {threads} threads")
        res["cpu_baseline"] = cpu_baseline(view, args.cpu_rows_step, threads)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
