"""Benchmark: escape-time Mandelbrot on one MI355X.

Headline workload (the 8192 x 8192 full view): re in [-2, 1], im in
[-1.2, 1.2], pixel centres, R = 2, max_iter 10000, FP64, int32 counts.  One
step = one mandel_render of the whole view (persistent FCFS queue of 64 x 8
tiles) with the output resident in HBM.  value = pixel-iterations per second
(sum of the counts / mean step time).  FP64 FLOP/s counts 7 operations per
iteration (x*x, y*y, x*y, 2*, -, +cx, +cy).

Also reported (not the value):
  * makespans on the uneven 64-view batch (seed 745): per-view static rows
    (paper Sec. III-A) and alternating rows (Sec. III-C) at their best worker
    count, per-view FCFS, and one batched persistent launch (hipGraph) in FCFS,
    probe-heuristic, learned-model and true-cost orders;
  * the oracle's rate on the host cores for a bounded sample.

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz
FLOPS_PER_ITER = 7
KERNEL_SRC = os.path.join(ROOT, "paper_2007_00745_amd", "csrc", "render_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_fcfs_8192_traffic.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the render kernel from the committed counter
    summary, or None if the kernel source changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_sha():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(view, rows_step: int, threads: int) -> dict:
    """The oracle (one single-threaded loop per worker) on every rows_step-th row."""
    import numpy as np

    import oracle
    rows = np.arange(0, view.m, rows_step)
    idx = (rows[:, None] * view.n + np.arange(view.n)[None, :]).ravel()
    t0 = time.perf_counter()
    counts = oracle.render_pixels(view.window, view.m, view.n, view.max_iter, view.R, idx,
                                  threads=threads)
    dt = time.perf_counter() - t0
    total = int(counts.sum(dtype=np.int64))
    return {"value": total / dt, "unit": "pixel-iterations/s", "cores": threads,
            "kind": "oracle",
            "sample": f"rows i = 0 mod {rows_step} of the {view.m}x{view.n} view "
                      f"({len(rows)} rows, {idx.size} px, {total} iterations, {dt:.2f} s wall)"}


def timed_ms(torch, fn, reps: int, name: str) -> float:
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for r in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
        log(f"  {name} rep {r}: {a.elapsed_time(b):.2f} ms")
    return best


def tail_fraction(st, clock_khz):
    """From the launch timestamps: time between the first claim that found the
    queue empty and the last wavefront exit, and its share of the launch."""
    if st[6] == 0 or st[4] < 0 or st[5] < 0 or st[6] <= st[4] or st[5] < st[4]:
        return None
    return {"tail_ms": (st[6] - st[5]) / clock_khz, "span_ms": (st[6] - st[4]) / clock_khz,
            "tail_fraction": (st[6] - st[5]) / (st[6] - st[4])}


def makespans(torch, native, workloads, costmodel, reps: int, clock_khz: float) -> dict:
    """Uneven 64-view batch: per-view row partitions and FCFS vs one batched launch."""
    res = {}
    views = workloads.c3()
    log(f"makespan: {len(views)} views, {sum(v.pixels for v in views)} px")
    t0 = time.perf_counter()
    tun, trials = native.autotune(views)
    res["autotune"] = {"tuning": tun, "trials": trials, "seconds": time.perf_counter() - t0}
    plan = native.Plan(views, tun)
    out = torch.empty(plan.out_size(), dtype=torch.int32, device="cuda")
    cost = torch.empty(plan.ntiles, dtype=torch.int64, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    plan.launch(out, tile_cost=cost)
    torch.cuda.synchronize()
    sum_counts = int(cost.sum().item())
    ref = out.clone()
    res["sum_counts"] = sum_counts
    res["tiles"] = plan.ntiles

    def per_view(policy, wsel):
        for v, o in zip(views, plan.out_offsets):
            kw = {"policy": policy}
            if policy in ("static", "alternating"):
                kw["workers"] = wsel(v)
            native.render_sched(v.window, v.m, v.n, v.max_iter, v.R,
                                out=out[o:o + v.pixels].view(v.m, v.n), **kw)

    ms = {}
    for pol in ("static", "alternating"):
        best = None
        for label, wsel in (("W=m", lambda v: v.m), ("W=m/2", lambda v: max(1, v.m // 2)),
                            ("W=m/4", lambda v: max(1, v.m // 4))):
            t = timed_ms(torch, lambda: per_view(pol, wsel), 1, f"{pol} {label}")
            if best is None or t < best[0]:
                best = (t, label)
        ms[f"{pol}_rows_per_view"] = {"ms": best[0], "workers": best[1]}
    assert torch.equal(out, ref), "row partitions changed the counts"
    ms["fcfs_per_view"] = {"ms": timed_ms(torch, lambda: per_view("fcfs", None), 1, "fcfs/view")}

    log("makespan: training the cost model")
    t0 = time.perf_counter()
    tv = workloads.training_views(range(1000, 1016), per_seed=4)
    feat, target, _, tplan = costmodel.collect(tv, tun)
    params, losses = costmodel.train(feat, target, epochs=30, batch=512, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    res["cost_model"] = {"train_tiles_logged": int(tplan.ntiles),
                         "train_samples": min(int(tplan.ntiles), 200000), "epochs": 30,
                         "final_train_loss": losses[-1], "seconds": time.perf_counter() - t0}
    res["cost_model"].update(costmodel.evaluate(params, plan.features(), native.cost_targets(cost)))
    tplan.close()
    true_perm = torch.argsort(cost, descending=True).to(torch.int32)
    names = {"fcfs": "fcfs", "probe": "probe_lpt", "learned": "learned_lpt",
             "ordered": "true_cost_lpt"}
    for mode, kw in (("fcfs", {}), ("probe", {}), ("learned", {"mlp": params}),
                     ("ordered", {"order": true_perm})):
        out.fill_(-1)
        t = timed_ms(torch, lambda: plan.launch(out, mode=mode, use_graph=True, **kw), reps,
                     f"batched {mode}")
        assert torch.equal(out, ref), f"batched {mode} changed the counts"
        stats.zero_()
        plan.launch(out, mode=mode, stats=stats, **kw)
        torch.cuda.synchronize()
        st = [int(v) for v in stats.cpu().tolist()]
        ms[f"batched_{names[mode]}"] = {"ms": t, "tail": tail_fraction(st, clock_khz)}
    res["makespan_ms"] = ms
    static = min(ms["static_rows_per_view"]["ms"], ms["alternating_rows_per_view"]["ms"])
    res["speedup_batched_learned_vs_static_rows"] = static / ms["batched_learned_lpt"]["ms"]
    res["speedup_batched_fcfs_vs_static_rows"] = static / ms["batched_fcfs"]["ms"]
    res["batched_fcfs_pixel_iterations_per_s"] = sum_counts / (ms["batched_fcfs"]["ms"] / 1e3)
    plan.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=8192)
    ap.add_argument("--max-iter", type=int, default=10000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-makespan", action="store_true")
    ap.add_argument("--makespan-reps", type=int, default=3)
    ap.add_argument("--cpu-rows-step", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on a single GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2007_00745_amd import costmodel, native, workloads

    native.lib()  # fails loudly when the library is missing
    view = workloads.c2(args.side, args.max_iter)
    torch.cuda.set_device(0)
    dinfo = native.device_info()
    clock_khz = float(dinfo["wall_clock_khz"]) or 100000.0
    out = torch.empty((view.m, view.n), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        native.render(view.window, view.m, view.n, view.max_iter, view.R, out=out, stream=stream)

    log(f"bench: {view.m}x{view.n} max_iter {view.max_iter}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    native.render_sched(view.window, view.m, view.n, view.max_iter, view.R, out=out,
                        stream=stream, stats=stats)
    torch.cuda.synchronize()
    sum_counts = int(out.sum(dtype=torch.int64).item())
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
    log(f"bench: {ms_mean:.3f} ms/step, {tflops:.2f} TFLOP/s")

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("bench: copy calibration done (1 GiB read, 1 GiB written)")

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
                               f"pixel centres, R=2, max_iter {view.max_iter}",
                   "policy": "persistent FCFS tile queue, 64x8 tiles",
                   "parallelism": "single GPU"},
        "sum_counts": sum_counts,
        "fp64_tflops": tflops,
        "pct_fp64_peak": 100.0 * tflops / FP64_PEAK_TFLOPS,
        "lane_occupancy": lane_occ,
        "tail": tail_fraction(st, clock_khz),
        "ms_min": min(ms),
        "wall_s": wall,
        "device": dinfo,
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic()},
        "kernel_source_sha256_16": kernel_sha(),
    }
    if not args.no_makespan:
        res["makespan"] = makespans(torch, native, workloads, costmodel, args.makespan_reps,
                                    clock_khz)
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"bench: cpu baseline on {threads} threads")
        res["cpu_baseline"] = cpu_baseline(view, args.cpu_rows_step, threads)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
