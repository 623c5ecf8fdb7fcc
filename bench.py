"""Benchmark: escape-time Mandelbrot on one MI355X.

Headline workload (the 8192 x 8192 full view): re in [-2, 1], im in
[-1.2, 1.2], pixel centres, R = 2, max_iter 10000, FP64, int32 counts.
One step = one pass of the whole hot path over the view, with the output
resident in HBM: one replay of the plan's hipGraph = probe features (64 probe
pixels per 64 x 8 tile) -> cost-model MLP -> descending tile order ->
persistent render over the ordered device queue.  The cost model is trained
once before timing (on views disjoint from every timed workload).
Consecutive steps alternate over two streams, each with its own plan and
output buffer, so one step's features and render start while the previous
render drains; every step computes its whole image.
value = pixel-iterations per second (K x sum of the counts / time of the K
steps, events on both streams); the one-stream step time is reported beside it.
FP64 FLOP/s counts 7 operations per iteration (x*x, y*y, x*y, 2*, -, +cx, +cy).

Also reported (not the value): the plain mandel_render (FCFS queue in tile
order) and the order by true tile costs on the same view; the paper's contiguous
and alternating row partitions of the same view over 256..2048 workers, the FCFS
queue's claim grain and the grid launch; the time to the same
image with exact periodicity detection (updates skipped reported apart, never
counted as executed); the paper's image shape (8000 x 8000, max_iter 2000,
R 400, window assumed) next to the paper's 32-task computation time; makespans
on the uneven 64-view batch (seed 745) for per-view static rows (paper
Sec. III-A), alternating rows (Sec. III-C), per-view FCFS, the two row
partitions as one launch over all rows of the batch, and one batched launch in
FCFS, probe-heuristic, learned and true-cost orders; the stress batch (a
16384 x 16384 deep zoom of width 1e-12 plus 4096 views of 512 x 512) in one plan
against the paper's row partitions over all its rows; the oracle's rate on the
host cores for a bounded sample and on one core for the 640 x 480 view.

Prints one JSON line.  --gpus N > 1 is refused: the benchmark runs on one GPU.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_ordered_8192_traffic.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_code(text: str) -> str:
    """The render kernel source without comments and whitespace, so that counters
    taken for some code stay attached to it across edits of comments only."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":                      # string or char literal, kept
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return "".join("".join(out).split())


def kernel_sha() -> str:
    return hashlib.sha256(kernel_code(open(KERNEL_SRC).read()).encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the render kernel from the committed counter
    summary, or None if the kernel code changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_code_sha256_16") != kernel_sha():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_rows(tasks, threads: int) -> tuple[int, float]:
    """Runs the oracle on (view, rows) tasks: each task renders the given rows of one
    view on one thread; `threads` workers take tasks first come first served (the
    paper's dynamic scheme, Sec. III-B, on the host).  Returns (sum of counts, wall
    seconds)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    def one(task):
        v, rows = task
        idx = (np.asarray(rows, dtype=np.int64)[:, None] * v.n +
               np.arange(v.n, dtype=np.int64)[None, :]).ravel()
        c = oracle.render_pixels(v.window, v.m, v.n, v.max_iter, v.R, idx, threads=1)
        return int(c.sum(dtype=np.int64))

    t0 = time.perf_counter()
    if threads <= 1:
        total = sum(one(t) for t in tasks)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            total = sum(ex.map(one, tasks))
    return total, time.perf_counter() - t0


def cpu_baseline(view, rows_step: int, threads: int) -> dict:
    """The oracle (plain single-threaded C loops, one per worker) timed on the host:
    all cores on every rows_step-th row of the headline view (the reported value);
    one core on a band of that view's rows and on the whole 640 x 480 view; all cores
    on row samples of the uneven 64-view batch and of the stress batch's 512 x 512
    views.  Samples are spread over each image so their cost mix is the image's."""
    import numpy as np

    import oracle
    from paper_2007_00745_amd import workloads

    def band(v, step, offset=0):
        return [(v, [int(r)]) for r in range(offset, v.m, step)]

    total, dt = _oracle_rows(band(view, rows_step), threads)
    nrows = len(range(0, view.m, rows_step))
    # one core: every 24th row of the headline view (about 12 s on one core)
    s_band, d_band = _oracle_rows(band(view, 24, 12), 1)
    # one core on the small 640 x 480 view, whole image
    c1 = workloads.c1()
    t1 = time.perf_counter()
    img = oracle.render(c1.window, c1.m, c1.n, c1.max_iter, c1.R)
    d1 = time.perf_counter() - t1
    s1 = int(img.sum(dtype=np.int64))
    # all cores: every 32nd row of every view of the uneven batch, every 128th row of
    # every small view of the stress batch (rows offset so that both halves are hit)
    c3 = workloads.c3()
    s3, d3 = _oracle_rows([t for v in c3 for t in band(v, 32, 7)], threads)
    c5s = workloads.c5()[1:]
    s5, d5 = _oracle_rows([t for v in c5s for t in band(v, 128, 61)], threads)
    import platform
    import subprocess
    try:
        gcc = subprocess.run(["gcc", "--version"], capture_output=True, text=True,
                             timeout=10).stdout.splitlines()[0]
    except (OSError, subprocess.SubprocessError, IndexError):
        gcc = None
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    host = {"cpu_model": model or platform.processor() or None,
            "nproc": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else None,
            "compiler": gcc, "cflags": " ".join(oracle.CFLAGS)}
    unit = "pixel-iterations/s"
    return {"value": total / dt, "unit": unit, "cores": threads,
            "kind": "oracle", "host": host,
            "sample": f"rows i = 0 mod {rows_step} of the {view.m}x{view.n} view "
                      f"({nrows} rows, {nrows * view.n} px, {total} iterations, {dt:.2f} s "
                      f"wall), one row per task, {threads} worker threads",
            "single_core": {"value": s_band / d_band, "unit": unit, "seconds": d_band,
                            "iterations": s_band,
                            "workload": f"rows i = 12 mod 24 of the {view.m}x{view.n} view, "
                                        "one thread"},
            "single_core_small_view": {"value": s1 / d1, "unit": unit, "seconds": d1,
                                       "iterations": s1,
                                       "workload": f"{c1.m}x{c1.n} full view, max_iter "
                                                   f"{c1.max_iter}, whole image, one thread"},
            "all_core_uneven_batch": {"value": s3 / d3, "unit": unit, "cores": threads,
                                      "seconds": d3, "iterations": s3,
                                      "workload": "rows i = 7 mod 32 of every view of the "
                                                  "uneven 64-view batch"},
            "all_core_stress_small_views": {"value": s5 / d5, "unit": unit, "cores": threads,
                                            "seconds": d5, "iterations": s5,
                                            "workload": "rows i = 61 mod 128 of each of the "
                                                        "stress batch's 4096 views of 512^2"}}


# Computation times of the paper's alternating-row run with 32 MPI tasks on two Xeon
# Gold 6150 nodes, 8000 x 8000 image, iterationMax 2000, escape radius 400 (the five
# runs of its appendix listing; the window is not stated).
PAPER_ALT32_COMPUTE_S = (2.855784, 2.857663, 2.858120, 2.855122, 2.855696)


def tail_analysis(torch, native, plan, out, params, cost, clock_khz, stream, last=64) -> dict:
    """One learned launch with per-tile timestamps: which tiles finish last, how
    their true cost and predicted cost rank among all tiles (percentiles, 100 = most
    expensive), and how long before the queue ran dry they were claimed."""
    import numpy as np
    nt = plan.ntiles
    tt = torch.zeros(2 * nt, dtype=torch.int64, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    plan.launch(out, mode="learned", mlp=params, tile_time=tt, stats=stats, stream=stream)
    keys = native.mlp_forward(params, plan.features(stream=stream), stream=stream)
    torch.cuda.synchronize()
    t = tt.cpu().numpy().view(np.uint64).reshape(nt, 2).astype(np.float64)
    st = stats.cpu().numpy().view(np.uint64).astype(np.float64)
    c = cost.cpu().numpy()
    k = keys.cpu().numpy()
    pct = lambda a: 100.0 * np.argsort(np.argsort(a)) / max(nt - 1, 1)
    cp, kp = pct(c), pct(k)
    idx = np.argsort(t[:, 1])[-last:]
    return {"last_tiles": last,
            "true_cost_percentile_mean": float(cp[idx].mean()),
            "predicted_percentile_mean": float(kp[idx].mean()),
            "claimed_ms_before_queue_dry_mean": float(((st[5] - t[idx, 0]) / clock_khz).mean()),
            "finished_ms_after_queue_dry_max": float(((t[idx, 1] - st[5]) / clock_khz).max())}


# Deferred-block length for the launches with periodicity detection (64-256 measure
# alike on the 8192 x 8192 view; 1024, the default, finds cycles later).
PERIOD_BLOCK_ITERS = 128


def periodicity(torch, native, view, plan, out, sum_counts, headline_ms, clock_khz,
                stream) -> dict:
    """Time to the same image with exact periodicity detection: lanes whose FP64
    state recurs bit for bit stop early with count max_iter.  Skipped updates are
    reported, not counted as executed.  Timed on the headline plan (FCFS queue,
    blocks of up to 1024 updates), and on a plan whose blocks stop at 128 updates
    (a cycle is found at the end of the first block that starts on it, so shorter
    blocks find it sooner), with and without row stealing (the tiles whose orbits
    never settle are the tail; stealing spreads their rows over idle wavefronts)."""
    ref = out.clone()
    short = native.Plan([view], {"block_iters": PERIOD_BLOCK_ITERS})

    def run(p, steal, stats=None, graph=True):
        p.launch(out, periodicity=1, use_graph=graph, steal=steal, stats=stats, stream=stream)

    res = {}
    for name, p, steal in (("blocks_1024_fcfs", plan, 0),
                           (f"blocks_{PERIOD_BLOCK_ITERS}_fcfs", short, 0),
                           (f"blocks_{PERIOD_BLOCK_ITERS}_fcfs_row_stealing", short, 1)):
        ms = timed_ms(torch, lambda: run(p, steal), 3, f"periodicity detection {name}")
        assert torch.equal(out, ref), f"periodicity detection changed the counts ({name})"
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        out.fill_(-1)
        run(p, steal, stats, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"periodicity detection changed the counts ({name})"
        st = [int(v) for v in stats.cpu().tolist()]
        executed = sum_counts - st[7]
        res[name] = {"ms": ms, "updates_skipped": st[7], "updates_executed": executed,
                     "executed_pixel_iterations_per_s": executed / (ms / 1e3),
                     "time_to_image_speedup_vs_step": headline_ms / ms,
                     "tail": tail_fraction(st, clock_khz)}
    short.close()
    best = res[f"blocks_{PERIOD_BLOCK_ITERS}_fcfs_row_stealing"]
    return dict(best, sum_counts=sum_counts,
                configuration=f"plan block_iters {PERIOD_BLOCK_ITERS}, FCFS queue, row stealing",
                variants=res)


def output_path(torch, native, out, view, step, stream) -> dict:
    """The paper's total-time analog: the headline step, then Boolean colouring,
    the copy to pinned host memory and the PPM write (to a temporary directory),
    each timed; plus an 8-frame zoom sequence written sequentially and with the
    writes overlapped with the next frame's render."""
    import shutil
    import tempfile

    from paper_2007_00745_amd import output, workloads
    npx = view.pixels
    rgb = torch.empty(3 * npx, dtype=torch.uint8, device="cuda")
    host = torch.empty(3 * npx, dtype=torch.uint8, pin_memory=True)
    colour_ms = timed_ms(torch, lambda: native.colour_boolean(out, view.max_iter, rgb,
                                                              stream=stream), 3, "colour")
    copy_ms = timed_ms(torch, lambda: host.copy_(rgb, non_blocking=True), 3, "copy to host")
    tmp = tempfile.mkdtemp(prefix="mandel_ppm_")
    try:
        t0 = time.perf_counter()
        native.write_ppm(os.path.join(tmp, "c2.ppm"), host, view.m, view.n)
        write_s = time.perf_counter() - t0
        # total, end to end: step -> colour -> copy -> write
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        native.colour_boolean(out, view.max_iter, rgb, stream=stream)
        host.copy_(rgb, non_blocking=True)
        torch.cuda.synchronize()
        native.write_ppm(os.path.join(tmp, "c2.ppm"), host, view.m, view.n)
        total_s = time.perf_counter() - t0
        frames = [workloads.View((SEAHORSE[0], SEAHORSE[1], 4e-3 / 4096 / 2 ** k,
                                  4e-3 / 4096 / 2 ** k), 4096, 4096, 5000) for k in range(8)]
        seq = {}
        for pipelined in (False, True):
            paths = [os.path.join(tmp, f"f{k}.ppm") for k in range(len(frames))]
            seq["pipelined" if pipelined else "sequential"] = output.render_to_ppm(
                frames, paths, pipelined=pipelined)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    gbs = 7.0 * npx / (colour_ms / 1e3) / 1e9
    return {"image": f"{view.m}x{view.n}", "colour_ms": colour_ms,
            "colour_kernel": {"bound": "hbm", "bytes_per_pixel": 7, "achieved_gbs": gbs,
                              "frac": gbs / HBM_PEAK_GBS},
            "copy_to_host_ms": copy_ms, "copy_gbs": 3.0 * npx / (copy_ms / 1e3) / 1e9,
            "ppm_write_s": write_s, "total_time_s": total_s,
            "zoom_sequence_8x4096sq": seq}


# FP64 instructions of one double-double update + test as the kernel issues them: 66
# add/sub, 3 mul, 13 fma (the two doublings of mul(X, Y) ride on fma's); the flops of
# the arithmetic as defined: 72 add/sub, 5 mul, 7 fma
DD_INSTR_PER_ITER = 82
DD_FLOPS_PER_ITER = 72 + 5 + 2 * 7


# a point of seahorse valley often used for deep zooms
SEAHORSE = (-0.7436438870371587, 0.1318259042053119)


def deep_zoom(torch, native, side: int = 4096, dx: float = 1e-17, max_iter: int = 20000) -> dict:
    """Double-double render of a side x side view of pitch dx (below binary64
    resolution near |c| ~ 0.76) at a seahorse-valley point, next to the binary64
    render of the same window, whose pixel centres collapse into blocks."""
    win = (SEAHORSE[0], 0.0, SEAHORSE[1], 0.0, dx, dx)
    out = torch.empty((side, side), dtype=torch.int32, device="cuda")
    ms = timed_ms(torch, lambda: native.render_dd(win, side, side, max_iter, 2.0, out=out), 2,
                  "double-double deep zoom")
    total = int(out.sum(dtype=torch.int64).item())
    f64 = torch.empty_like(out)
    ms64 = timed_ms(torch, lambda: native.render((SEAHORSE[0], SEAHORSE[1], dx, dx), side, side,
                                                  max_iter, 2.0, out=f64), 2,
                    "binary64 same window")
    rate = total / (ms / 1e3)
    return {"workload": f"{side}x{side}, pitch {dx:g}, max_iter {max_iter}, R 2, centre "
                        f"{SEAHORSE[0]!r} + {SEAHORSE[1]!r} i",
            "ms": ms, "sum_counts": total, "pixel_iterations_per_s": rate,
            "fp64_instructions_per_iteration": DD_INSTR_PER_ITER,
            "fp64_tflops": rate * DD_FLOPS_PER_ITER / 1e12,
            "fp64_issue_frac": rate * DD_INSTR_PER_ITER / (FP64_PEAK_TFLOPS * 1e12 / 2),
            "binary64_same_window_ms": ms64,
            "distinct_counts_middle_row": {
                "double_double": int(torch.unique(out[side // 2]).numel()),
                "binary64": int(torch.unique(f64[side // 2]).numel())}}


def paper_context(torch, native, workloads) -> dict:
    """The paper's image shape on this GPU, with the window assumed to be the
    640 x 480 view's (re [-2, 1], im [-1.2, 1.2]): context, not a like-for-like figure."""
    v = workloads.paper_view()
    out = torch.empty((v.m, v.n), dtype=torch.int32, device="cuda")
    ms = timed_ms(torch, lambda: native.render(v.window, v.m, v.n, v.max_iter, v.R, out=out),
                  3, "paper-shaped view")
    total = int(out.sum(dtype=torch.int64).item())
    paper_s = sum(PAPER_ALT32_COMPUTE_S) / len(PAPER_ALT32_COMPUTE_S)
    return {"workload": f"{v.m}x{v.n}, max_iter {v.max_iter}, R {v.R}, window assumed "
                        "re[-2,1] x im[-1.2,1.2]",
            "gpu_ms": ms, "sum_counts": total,
            "gpu_pixel_iterations_per_s": total / (ms / 1e3),
            "paper_alternating_32_tasks_compute_s": paper_s,
            "paper_pixel_iterations_per_s_if_same_window": total / paper_s,
            "time_ratio": paper_s / (ms / 1e3)}


def timed_stats(torch, fn, reps: int, name: str) -> dict:
    """One untimed warm-up call, then `reps` calls each between two events:
    {"ms": minimum, "median_ms": median, "reps": reps, "all_ms": every time}."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for r in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
        log(f"  {name} rep {r}: {ts[-1]:.2f} ms")
    srt = sorted(ts)
    return {"ms": srt[0], "median_ms": srt[len(srt) // 2], "reps": reps, "all_ms": ts}


def timed_ms(torch, fn, reps: int, name: str) -> float:
    return timed_stats(torch, fn, reps, name)["ms"]


def tail_fraction(st, clock_khz):
    """From the launch timestamps: time between the first claim that found the
    queue empty and the last wavefront exit, and its share of the launch."""
    if st[6] == 0 or st[4] < 0 or st[5] < 0 or st[6] <= st[4] or st[5] < st[4]:
        return None
    return {"tail_ms": (st[6] - st[5]) / clock_khz, "span_ms": (st[6] - st[4]) / clock_khz,
            "tail_fraction": (st[6] - st[5]) / (st[6] - st[4])}


# Tiling of the batch plans whose queue orders are compared: the learned step probes
# every tile (64 probes of up to 128 updates), so coarse tiles keep that cost small,
# and 4 row parts per tile keep the queue's grain fine.  On the uneven batch the
# learned order with 64 x 8 tiles gained 1.4 of the 4.2 ms between FCFS and the
# true-cost order, with 128 x 16 tiles 3.5 of 4.7 ms (probe features 1.44 vs 0.38 ms).
# Deferred blocks of at most 128 updates: escapes are dense in these boundary zooms,
# and the batch took 305 ms in FCFS order against 316 ms with blocks of 1024.
BATCH_TUNING = {"tile_w": 128, "tile_h": 16, "tile_parts": 4, "block_iters": 128}


def train_cost_model(torch, native, workloads, costmodel, tuning=None, per_seed: int = 4):
    """Cost model for the ordered launches: tile costs logged from views of the
    uneven-batch distribution (seeds 1000-1015, per_seed views each) and four full
    views of other sizes and limits, on tiles of the given tuning; 200k tiles
    sampled, 30 epochs of Adam (all in the kernels)."""
    t0 = time.perf_counter()
    tv = workloads.training_views(range(1000, 1016), per_seed=per_seed)
    tv += [workloads.c2(side, mi) for side, mi in ((1024, 2000), (2048, 5000), (1536, 20000),
                                                   (768, 800))]
    feat, target, _, tplan = costmodel.collect(tv, tuning=tuning)
    params, losses = costmodel.train(feat, target, epochs=30, batch=512, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    info = {"train_views": len(tv), "train_tiles_logged": int(tplan.ntiles),
            "train_samples": min(int(tplan.ntiles), 200000), "epochs": 30, "batch": 512,
            "tiling": tplan.tuning, "final_train_loss": losses[-1],
            "seconds": time.perf_counter() - t0}
    tplan.close()
    return params, info


def makespans(torch, native, workloads, costmodel, reps: int, clock_khz: float,
              cus: int) -> dict:
    """Uneven 64-view batch: per-view row partitions and FCFS vs one batched launch.
    The queue orders are compared on one plan of BATCH_TUNING tiles, with a cost model
    trained on tiles of that shape; the autotuner's own pick is timed in FCFS order
    beside them."""
    res = {}
    views = workloads.c3()
    log(f"makespan: {len(views)} views, {sum(v.pixels for v in views)} px")
    params, res["cost_model_training"] = train_cost_model(torch, native, workloads, costmodel,
                                                          tuning=BATCH_TUNING, per_seed=8)
    t0 = time.perf_counter()
    tun, trials = native.autotune(views)
    res["autotune"] = {"tuning": tun, "trials": trials, "seconds": time.perf_counter() - t0}
    plan = native.Plan(views, BATCH_TUNING)
    res["tuning"] = plan.tuning
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

    # Each configuration is swept once; the best worker count is then timed `reps` times
    # (min and median reported, speed-ups on the min).
    ms = {}
    for pol in ("static", "alternating"):
        best = None
        for label, wsel in (("W=m", lambda v: v.m), ("W=m/2", lambda v: max(1, v.m // 2)),
                            ("W=m/4", lambda v: max(1, v.m // 4))):
            t = timed_ms(torch, lambda: per_view(pol, wsel), 1, f"{pol} {label}")
            if best is None or t < best[0]:
                best = (t, label, wsel)
        rec = timed_stats(torch, lambda: per_view(pol, best[2]), reps, f"{pol} {best[1]}")
        ms[f"{pol}_rows_per_view"] = dict(rec, workers=best[1])
    assert torch.equal(out, ref), "row partitions changed the counts"
    ms["fcfs_per_view"] = timed_stats(torch, lambda: per_view("fcfs", None), reps, "fcfs/view")

    # The stricter static baseline: one launch in which the rows of all 64 views,
    # concatenated, are split over W workgroups by the paper's partitions.  W = 7 per CU
    # is every worker resident at once (4 wavefronts each); more workers than that wait
    # for free slots and measured several times slower, so the sweep stops there.
    for pol in ("static", "alternating"):
        per_w = {}
        for mult in (1, 2, 4, 7):
            W = cus * mult
            out.fill_(-1)
            per_w[W] = timed_ms(torch, lambda: plan.launch(out, mode=pol, workers=W,
                                                           use_graph=True), 1,
                                f"concatenated {pol} W={W}")
            assert torch.equal(out, ref), f"concatenated {pol} changed the counts"
        W = min(per_w, key=per_w.get)
        rec = timed_stats(torch, lambda: plan.launch(out, mode=pol, workers=W, use_graph=True),
                          reps, f"concatenated {pol} W={W}")
        stats.zero_()
        plan.launch(out, mode=pol, workers=W, stats=stats)
        torch.cuda.synchronize()
        st = [int(v) for v in stats.cpu().tolist()]
        ms[f"{pol}_rows_concatenated"] = dict(rec, workers=W, ms_by_workers=per_w,
                                              tail=tail_fraction(st, clock_khz))

    res["cost_model_eval"] = costmodel.evaluate(params, plan.features(),
                                                native.cost_targets(cost))
    # the autotuner's pick, FCFS order
    aplan = native.Plan(views, tun)
    aout = torch.empty(aplan.out_size(), dtype=torch.int32, device="cuda")
    ms["batched_fcfs_autotuned"] = dict(
        timed_stats(torch, lambda: aplan.launch(aout, use_graph=True), reps,
                    "batched fcfs, autotuned plan"), tiling=aplan.tuning)
    assert torch.equal(aout, ref), "the autotuned plan changed the counts"
    aplan.close()
    del aout
    true_perm = torch.argsort(cost, descending=True).to(torch.int32)
    names = {"fcfs": "fcfs", "probe": "probe_lpt", "learned": "learned_lpt",
             "ordered": "true_cost_lpt"}
    # the queue orders differ by about 1 % of a launch: each is timed in rounds that
    # interleave the four orders (3 x reps launches each), so box drift hits all alike
    modes = (("fcfs", {}), ("probe", {}), ("learned", {"mlp": params}),
             ("ordered", {"order": true_perm}))
    times = {mode: [] for mode, _ in modes}
    for rnd in range(3):
        for mode, kw in modes:
            out.fill_(-1)
            rec = timed_stats(torch, lambda: plan.launch(out, mode=mode, use_graph=True, **kw),
                              reps, f"batched {mode} round {rnd}")
            times[mode] += rec["all_ms"]
            assert torch.equal(out, ref), f"batched {mode} changed the counts"
    for mode, kw in modes:
        ts = sorted(times[mode])
        rec = {"ms": ts[0], "median_ms": ts[len(ts) // 2], "reps": len(ts)}
        stats.zero_()
        plan.launch(out, mode=mode, stats=stats, **kw)
        torch.cuda.synchronize()
        st = [int(v) for v in stats.cpu().tolist()]
        ms[f"batched_{names[mode]}"] = dict(rec, tail=tail_fraction(st, clock_khz))
    res["makespan_ms"] = ms
    f, lrn, tru = (ms[k]["median_ms"] for k in ("batched_fcfs", "batched_learned_lpt",
                                                "batched_true_cost_lpt"))
    # what the trained network gains over its FCFS fallback on the same plan, as a share
    # of what the true-cost order (known only after a render) gains
    res["learned_gain_share_of_true_cost_gain_medians"] = ((f - lrn) / (f - tru) if f > tru
                                                           else None)
    static = min(ms["static_rows_per_view"]["ms"], ms["alternating_rows_per_view"]["ms"])
    res["speedup_batched_learned_vs_static_rows"] = static / ms["batched_learned_lpt"]["ms"]
    res["speedup_batched_fcfs_vs_static_rows"] = static / ms["batched_fcfs"]["ms"]
    concat = min(ms["static_rows_concatenated"]["ms"], ms["alternating_rows_concatenated"]["ms"])
    res["speedup_batched_learned_vs_concatenated_rows"] = concat / ms["batched_learned_lpt"]["ms"]
    res["speedup_batched_fcfs_vs_concatenated_rows"] = concat / ms["batched_fcfs"]["ms"]
    res["batched_fcfs_pixel_iterations_per_s"] = sum_counts / (ms["batched_fcfs"]["ms"] / 1e3)
    static_med = min(ms["static_rows_per_view"]["median_ms"],
                     ms["alternating_rows_per_view"]["median_ms"])
    concat_med = min(ms["static_rows_concatenated"]["median_ms"],
                     ms["alternating_rows_concatenated"]["median_ms"])
    res["speedup_medians"] = {
        "batched_learned_vs_static_rows": static_med / ms["batched_learned_lpt"]["median_ms"],
        "batched_fcfs_vs_static_rows": static_med / ms["batched_fcfs"]["median_ms"],
        "batched_learned_vs_concatenated_rows": concat_med / ms["batched_learned_lpt"]["median_ms"],
        "batched_fcfs_vs_concatenated_rows": concat_med / ms["batched_fcfs"]["median_ms"]}
    plan.close()
    return res


def profile_batch(torch, native, workloads, costmodel, steps: int) -> dict:
    """Counter runs on the uneven batch (plan of BATCH_TUNING tiles): the features,
    inference and ordered-render kernels, each launched `steps` times between events;
    returns the figures that turn per-dispatch counters into per-iteration rates."""
    views = workloads.c3()
    torch.cuda.set_device(0)
    plan = native.Plan(views, BATCH_TUNING)
    out = torch.empty(plan.out_size(), dtype=torch.int32, device="cuda")
    cost = torch.empty(plan.ntiles, dtype=torch.int64, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    plan.launch(out, tile_cost=cost)
    torch.cuda.synchronize()
    sum_counts = int(cost.sum().item())
    feat = torch.empty((plan.ntiles, native.NFEAT), dtype=torch.float32, device="cuda")
    params = costmodel.init_params(0)
    keys = torch.empty(plan.ntiles, dtype=torch.float32, device="cuda")

    def timed(fn):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    res = {"workload": "uneven 64-view batch (seed 745)", "tuning": plan.tuning,
           "tiles": plan.ntiles, "sum_counts": sum_counts}
    res["features_ms"] = timed(lambda: plan.features(feat))
    f = feat.cpu().numpy()[:, 4:].astype("float64")
    import numpy as np
    caps = np.minimum(np.array([v.max_iter for v in views]), 128)
    # probe iterations = sum of min(count, cap) over all probes, from the features
    tile_view = np.repeat(np.arange(len(views)),
                          [native.tile_count(v.m, v.n, plan.tuning["tile_w"],
                                             plan.tuning["tile_h"]) for v in views])
    cap_t = caps[tile_view][:, None].astype(np.float64)
    res["probe_iterations"] = int(np.rint(np.exp(f * np.log1p(cap_t)) - 1).sum())
    res["mlp_ms"] = timed(lambda: native.mlp_forward(params, feat, keys))
    true_perm = native.order_desc(native.cost_targets(cost))
    res["render_ms"] = timed(lambda: plan.launch(out, mode="ordered", order=true_perm,
                                                 stats=stats))
    torch.cuda.synchronize()
    st = [int(v) for v in stats.cpu().tolist()]
    res["render_wave_iterations_per_launch"] = st[0] / steps
    res["lane_occupancy"] = st[1] / (64.0 * st[0]) if st[0] else None
    assert int(out.sum(dtype=torch.int64).item()) == sum_counts
    plan.close()
    return res


# Single views of the counter table of the render kernel: what its instruction mix
# looks like with no escapes, with the headline's mix at a smaller size, with dense
# escapes, and with every pixel escaping at once.
PROFILE_VIEWS = {
    "interior": ((-0.2, 0.0, 0.2 / 2048, 0.2 / 2048), 2048, 2048, 10000),
    "full_4096": (None, 4096, 4096, 10000),
    "seahorse": ((-0.745, 0.113, 0.01 / 2048, 0.01 / 2048), 2048, 2048, 10000),
    "exterior": ((3.0, 3.0, 0.5 / 4096, 0.5 / 4096), 4096, 4096, 10000),
}


def profile_view(torch, native, workloads, name: str, steps: int) -> dict:
    """Counter runs on one view of PROFILE_VIEWS through a one-view plan (64x8 tiles):
    one FCFS launch logs the tile costs, then `steps` ordered launches in the true-cost
    order; returns the figures that turn per-dispatch counters into per-iteration rates."""
    win, m, n, max_iter = PROFILE_VIEWS[name]
    v = workloads.c2(m, max_iter) if win is None else workloads.View(win, m, n, max_iter)
    torch.cuda.set_device(0)
    plan = native.Plan([v])
    out = torch.empty(plan.out_size(), dtype=torch.int32, device="cuda")
    cost = torch.empty(plan.ntiles, dtype=torch.int64, device="cuda")
    plan.launch(out, tile_cost=cost)
    torch.cuda.synchronize()
    perm = native.order_desc(native.cost_targets(cost))
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    for _ in range(steps):
        plan.launch(out, mode="ordered", order=perm, stats=stats)
    torch.cuda.synchronize()
    st = [int(x) for x in stats.cpu().tolist()]
    sum_counts = int(cost.sum().item())
    assert st[1] == steps * sum_counts
    plan.close()
    return {"view": name, "window": list(v.window), "m": v.m, "n": v.n,
            "max_iter": v.max_iter, "sum_counts": sum_counts,
            "render_wave_iterations_per_launch": st[0] / steps,
            "lane_occupancy": st[1] / (64.0 * st[0]) if st[0] else None}


def stress_batch(torch, native, workloads, costmodel, reps: int, clock_khz: float, params,
                 cus: int, contiguous_rows: bool = False) -> dict:
    """Stress batch in one plan (64x8 tiles, blocks of at most 128 updates): a 16384 x
    16384 deep zoom of width 1e-12 at a boundary point (max_iter 50000) submitted first,
    then 4096 views of 512 x 512 drawn like the uneven batch.  Queue orders FCFS (submission order), probe, learned and true
    cost, and the paper's alternating row partition over the concatenated rows (every
    worker resident); the contiguous partition only on request (about a minute per
    launch: the deep view's rows fall to a few workers).  Every order must give the
    FCFS counts."""
    views = workloads.c5()
    # blocks of at most 128 updates, as on the uneven batch: 1859 ms against 1925 ms
    # with blocks of 1024 in FCFS order
    plan = native.Plan(views, {"block_iters": 128})
    log(f"stress: {len(views)} views, {plan.npixels} px, {plan.ntiles} tiles")
    out = torch.empty(plan.out_size(), dtype=torch.int32, device="cuda")
    cost = torch.empty(plan.ntiles, dtype=torch.int64, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    plan.launch(out, tile_cost=cost)
    torch.cuda.synchronize()
    sum_counts = int(cost.sum().item())
    ref = out.clone()
    # tiles are numbered view by view, the deep view first
    nt0 = native.tile_count(views[0].m, views[0].n, plan.tuning["tile_w"], plan.tuning["tile_h"])
    res = {"views": len(views), "pixels": plan.npixels, "tiles": plan.ntiles,
           "sum_counts": sum_counts, "deep_view_sum_counts": int(cost[:nt0].sum().item())}
    if params is not None:
        res["cost_model_eval"] = costmodel.evaluate(params, plan.features(),
                                                    native.cost_targets(cost))
    true_perm = native.order_desc(native.cost_targets(cost))
    runs = [("fcfs", "fcfs", {}), ("probe_lpt", "probe", {}),
            ("true_cost_lpt", "ordered", {"order": true_perm})]
    if params is not None:
        runs.insert(2, ("learned_lpt", "learned", {"mlp": params}))
    W = cus * 7
    if contiguous_rows:
        runs.append(("static_rows_concatenated", "static", {"workers": W}))
    runs.append(("alternating_rows_concatenated", "alternating", {"workers": W}))
    ms = {}
    for name, mode, kw in runs:
        out.fill_(-1)
        t = timed_ms(torch, lambda: plan.launch(out, mode=mode, use_graph=True, **kw), reps,
                     f"stress {name}")
        assert torch.equal(out, ref), f"stress {name} changed the counts"
        stats.zero_()
        plan.launch(out, mode=mode, stats=stats, **kw)
        torch.cuda.synchronize()
        st = [int(v) for v in stats.cpu().tolist()]
        ms[name] = {"ms": t, "pixel_iterations_per_s": sum_counts / (t / 1e3),
                    "tail": tail_fraction(st, clock_khz)}
    # The same batch with collapsed rows: the deep view's row pitch lies below the
    # spacing of doubles near its centre, so neighbouring rows share their imaginary part
    # (and counts); each distinct row is rendered once and copied out after the render.
    cplan = native.Plan(views, {"block_iters": 128, "collapse_rows": 1})
    ccost = torch.empty(cplan.ntiles, dtype=torch.int64, device="cuda")
    out.fill_(-1)
    cplan.launch(out, tile_cost=ccost)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), "collapsed rows changed the counts"
    rendered = int(ccost.sum().item())
    out.fill_(-1)
    t = timed_ms(torch, lambda: cplan.launch(out, use_graph=True), reps, "stress fcfs collapsed")
    assert torch.equal(out, ref), "collapsed rows changed the counts"
    ms["fcfs_collapsed_rows"] = {"ms": t, "tiles": cplan.ntiles,
                                 "iterations_executed": rendered,
                                 "pixel_iterations_per_s_of_the_image": sum_counts / (t / 1e3),
                                 "executed_iterations_per_s": rendered / (t / 1e3)}
    cplan.close()
    res["makespan_ms"] = ms
    res["row_workers"] = W
    best_rows = min(ms[k]["ms"] for k in ("static_rows_concatenated",
                                          "alternating_rows_concatenated") if k in ms)
    for name in ("fcfs", "learned_lpt", "true_cost_lpt"):
        if name in ms:
            res[f"speedup_{name}_vs_best_row_partition"] = best_rows / ms[name]["ms"]
    plan.close()
    return res


def comparisons(torch, native, view, plan, out, cost, sum_counts, stream, params=None) -> dict:
    """The plain mandel_render (FCFS in tile order) and the true-cost order on the
    headline view, the cost of the probe features alone, and the time to the image with
    conjugate rows rendered once (the learned step's order when a model is given)."""
    comp = {}
    plain = torch.empty((view.m, view.n), dtype=torch.int32, device="cuda")
    comp["plain_fcfs_render_ms"] = timed_ms(
        torch, lambda: native.render(view.window, view.m, view.n, view.max_iter, view.R,
                                     out=plain, stream=stream), 3, "plain FCFS")
    assert torch.equal(plain.view(-1), out), "plain FCFS and the ordered plan disagree"
    true_perm = torch.argsort(cost, descending=True).to(torch.int32)
    comp["true_cost_order_ms"] = timed_ms(
        torch, lambda: plan.launch(out, mode="ordered", order=true_perm, use_graph=True,
                                   stream=stream), 3, "true-cost order")
    comp["features_ms"] = timed_ms(torch, lambda: plan.features(stream=stream), 3, "features")
    for k in ("plain_fcfs_render_ms", "true_cost_order_ms"):
        comp[k.replace("_ms", "_pixel_iterations_per_s")] = sum_counts / (comp[k] / 1e3)
    # Time to the same image when rows that are conjugates of each other are rendered
    # once (the window is centred on the real axis, and conjugate points have equal
    # counts bit for bit): half the rows run, then they are copied.  Reported apart;
    # the headline counts every executed iteration of the whole image.
    ref = out.clone()
    mplan = native.Plan([view], {"collapse_rows": 2})
    mcost = torch.empty(mplan.ntiles, dtype=torch.int64, device="cuda")
    out.fill_(-1)
    mplan.launch(out, tile_cost=mcost, stream=stream)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), "mirrored rows changed the counts"
    executed = int(mcost.sum().item())
    out.fill_(-1)
    mkw = {"mode": "learned", "mlp": params} if params is not None else {}
    t = timed_ms(torch, lambda: mplan.launch(out, use_graph=True, stream=stream, **mkw), 3,
                 "mirrored rows")
    assert torch.equal(out, ref), "mirrored rows changed the counts"
    comp["mirrored_rows"] = {"ms": t, "mode": "learned" if mkw else "fcfs", "tiles": mplan.ntiles,
                             "iterations_executed": executed,
                             "executed_iterations_per_s": executed / (t / 1e3),
                             "time_to_image_speedup_vs_fcfs": comp["plain_fcfs_render_ms"] / t}
    mplan.close()
    return comp


def view_partitions(torch, native, view, ref, sum_counts, cus: int, clock_khz: float,
                    headline_ms: float) -> dict:
    """The paper's setting on one image, the 8192 x 8192 view: its contiguous rows
    (Sec. III-A, Eq. (stp)-(rem)) and alternating rows (Sec. III-C) over W workgroup
    workers, against the device FCFS tile queue (Sec. III-B's analogue; 64 x 8 tiles,
    claim grain swept) and the non-persistent grid launch.  Every image must equal the
    headline's."""
    res = {}
    out = torch.empty((view.m, view.n), dtype=torch.int32, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")

    def run(name, **sched):
        rec = timed_stats(torch, lambda: native.render_sched(view.window, view.m, view.n,
                                                             view.max_iter, view.R, out=out,
                                                             **sched), 3, name)
        assert torch.equal(out.view(-1), ref), f"{name} changed the counts"
        stats.zero_()
        native.render_sched(view.window, view.m, view.n, view.max_iter, view.R, out=out,
                            stats=stats, **sched)
        torch.cuda.synchronize()
        st = [int(v) for v in stats.cpu().tolist()]
        rec["pixel_iterations_per_s"] = sum_counts / (rec["ms"] / 1e3)
        rec["tail"] = tail_fraction(st, clock_khz)
        return rec

    for pol in ("static", "alternating"):
        per = {}
        for W in (256, 512, 1024, 2048, cus * 7):
            per[W] = run(f"{pol} rows W={W}", policy=pol, workers=W)
        best = min(per, key=lambda w: per[w]["ms"])
        res[f"{pol}_rows"] = {"by_workers": per, "best_workers": best, "best_ms": per[best]["ms"]}
    per = {g: run(f"fcfs grain {g}", grain=g) for g in (1, 2, 4, 8)}
    best = min(per, key=lambda g: per[g]["ms"])
    res["fcfs_tiles"] = {"by_grain": per, "best_grain": best, "best_ms": per[best]["ms"]}
    res["grid_tiles"] = run("grid", policy="grid")
    best_rows = min(res["static_rows"]["best_ms"], res["alternating_rows"]["best_ms"])
    res["speedup_fcfs_vs_best_row_partition"] = best_rows / res["fcfs_tiles"]["best_ms"]
    res["speedup_headline_step_vs_best_row_partition"] = best_rows / headline_ms
    return res


FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (FMA = 2 flops)
HBM_PEAK_GBS = 8000.0


def secondary_kernels(torch, native, plan, params, sum_probe_iters, reps: int) -> dict:
    """Each ordering kernel timed alone (events on the launching stream) against
    the roofline that bounds it: probe features (FP64 VALU), cost-model inference
    and one training step (FP32 VALU), the bucket order (HBM)."""
    import numpy as np
    nt = plan.ntiles
    res = {}
    feat = plan.features()
    ms = timed_ms(torch, lambda: plan.features(feat), reps, "features kernel")
    tflops = 7 * sum_probe_iters / (ms / 1e3) / 1e12
    res["features"] = {"ms": ms, "tiles": nt, "probe_iterations": sum_probe_iters,
                       "bound": "alu", "achieved_tflops_fp64": tflops,
                       "frac": tflops / FP64_PEAK_TFLOPS}
    keys = torch.empty(nt, dtype=torch.float32, device="cuda")
    ms = timed_ms(torch, lambda: native.mlp_forward(params, feat, keys), reps, "mlp forward")
    flops = nt * 2 * (68 * 64 + 64 * 64 + 64)
    res["mlp_forward"] = {"ms": ms, "flops": flops, "bound": "alu",
                          "achieved_tflops_fp32": flops / (ms / 1e3) / 1e12,
                          "frac": flops / (ms / 1e3) / 1e12 / FP32_PEAK_TFLOPS}
    perm = torch.empty(nt, dtype=torch.int32, device="cuda")
    ms = timed_ms(torch, lambda: native.order_desc(keys, perm), reps, "order")
    nbytes = nt * (4 + 4 + 4)  # keys read twice, permutation written once
    res["order"] = {"ms": ms, "bytes": nbytes, "bound": "hbm",
                    "achieved_gbs": nbytes / (ms / 1e3) / 1e9,
                    "frac": nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    B = 512
    p2 = params.clone()
    m = torch.zeros_like(p2)
    v = torch.zeros_like(p2)
    target = torch.zeros(nt, dtype=torch.float32, device="cuda")
    idx = torch.arange(B, dtype=torch.int32, device="cuda")
    work = torch.empty(native.mlp_work_floats(B), dtype=torch.float32, device="cuda")
    ms = timed_ms(torch, lambda: native.mlp_train_step(p2, m, v, 1, feat, target, idx, 1e-3,
                                                       work=work), reps, "train step")
    flops = B * 3 * 2 * (68 * 64 + 64 * 64 + 64)  # forward + two backward products
    res["mlp_train_step"] = {"ms": ms, "batch": B, "flops": flops, "bound": "alu",
                             "achieved_tflops_fp32": flops / (ms / 1e3) / 1e12,
                             "frac": flops / (ms / 1e3) / 1e12 / FP32_PEAK_TFLOPS}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--side", type=int, default=8192)
    ap.add_argument("--max-iter", type=int, default=10000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-makespan", action="store_true")
    ap.add_argument("--makespan-reps", type=int, default=5)
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the stress batch (16384^2 deep zoom + 4096 views of 512^2)")
    ap.add_argument("--stress-contiguous-rows", action="store_true",
                    help="also time the contiguous row partition on the stress batch (~1 min "
                         "per launch)")
    ap.add_argument("--cpu-rows-step", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--profile", action="store_true",
                    help="run for counters and traces: one FCFS launch logs the tile costs, "
                         "then the ordered render (true-cost order) is launched only as it "
                         "is timed, --steps times; no training, no steps of the whole path, "
                         "no comparisons, makespans or CPU baseline")
    ap.add_argument("--profile-batch", action="store_true",
                    help="run for counters on the uneven 64-view batch: one FCFS launch logs "
                         "the tile costs, then --steps launches each of the probe-feature "
                         "kernel, the cost-model inference kernel (untrained weights) and the "
                         "ordered render in the true-cost order, on the plan the makespan "
                         "comparison uses; prints one JSON line and nothing else runs")
    ap.add_argument("--profile-view", choices=sorted(PROFILE_VIEWS),
                    help="run for counters on one single view: one FCFS launch logs the "
                         "tile costs, then --steps ordered launches in the true-cost order; "
                         "prints one JSON line and nothing else runs")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on a single GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2007_00745_amd import costmodel, native, workloads

    native.lib()  # fails loudly when the library is missing
    if args.profile_batch:
        print(json.dumps(profile_batch(torch, native, workloads, costmodel, args.steps)),
              flush=True)
        return
    if args.profile_view:
        print(json.dumps(profile_view(torch, native, workloads, args.profile_view, args.steps)),
              flush=True)
        return
    view = workloads.c2(args.side, args.max_iter)
    torch.cuda.set_device(0)
    dinfo = native.device_info()
    clock_khz = float(dinfo["wall_clock_khz"]) or 100000.0
    stream = torch.cuda.current_stream()
    if args.profile:
        args.no_makespan = args.no_cpu_baseline = args.no_stress = True
        params, cm_info, mode = None, {}, "probe"
    else:
        log("bench: training the cost model")
        params, cm_info = train_cost_model(torch, native, workloads, costmodel)
        mode = "learned"
    plan = native.Plan([view])
    out = torch.empty(plan.out_size(), dtype=torch.int32, device="cuda")
    # Consecutive steps alternate between two streams, each with its own plan (queue,
    # features, order, graph) and output buffer: the next step's probe/MLP/order
    # kernels and the start of its render fill the compute units that the current
    # render's tail leaves idle.  Every step still computes its whole image.
    plan2 = native.Plan([view])
    out2 = torch.empty(plan2.out_size(), dtype=torch.int32, device="cuda")
    stream2 = torch.cuda.Stream()
    pipes = [(plan, out, stream), (plan2, out2, stream2)]

    def step(k: int = 0):
        p, o, s = pipes[k % 2]
        p.launch(o, mode=mode, mlp=params, use_graph=True, stream=s)

    cost = torch.empty(plan.ntiles, dtype=torch.int64, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    if args.profile:
        # Counter and trace runs: the ordered render kernel is launched only as it is
        # timed below.  The tile costs and the sum of counts come from one FCFS launch,
        # a different instantiation of the render kernel, so a trace's statistics for
        # the ordered kernel cover exactly the timed launches.
        plan.launch(out, stats=stats, tile_cost=cost, stream=stream)
        torch.cuda.synchronize()
        sum_counts = int(out.sum(dtype=torch.int64).item())
        assert sum_counts == int(cost.sum().item())
        st = [int(v) for v in stats.cpu().tolist()]
        lane_occ = st[1] / (64.0 * st[0]) if st[0] else None
        ms, serial, wall = [], None, 0.0
    else:
        log(f"bench: {view.m}x{view.n} max_iter {view.max_iter}; warmup {args.warmup}")
        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        plan.launch(out, mode=mode, mlp=params, stats=stats, tile_cost=cost, stream=stream)
        torch.cuda.synchronize()
        sum_counts = int(out.sum(dtype=torch.int64).item())
        assert sum_counts == int(cost.sum().item())
        st = [int(v) for v in stats.cpu().tolist()]
        lane_occ = st[1] / (64.0 * st[0]) if st[0] else None
        if params is not None:
            cm_info.update(costmodel.evaluate(params, plan.features(), native.cost_targets(cost)))

        log(f"bench: timing {args.steps} steps on two alternating streams")
        out.fill_(-1)
        out2.fill_(-1)
        e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e_b = torch.cuda.Event()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e_start.record(stream)
        stream2.wait_event(e_start)
        for k in range(args.steps):
            step(k)
        e_b.record(stream2)
        stream.wait_event(e_b)
        e_end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_total = e_start.elapsed_time(e_end)
        ms_mean = ms_total / args.steps
        for o in (out, out2)[:min(args.steps, 2)]:
            assert int(o.sum(dtype=torch.int64).item()) == sum_counts, "a step left an incomplete image"
        sec = ms_mean / 1e3
        value = sum_counts / sec
        tflops = FLOPS_PER_ITER * sum_counts / sec / 1e12
        log(f"bench: {ms_mean:.3f} ms/step pipelined ({wall * 1e3 / args.steps:.3f} ms/step wall), "
            f"{tflops:.2f} TFLOP/s")

        # The same steps one after another on one stream: the latency of one step.
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream)
            step(0)
            b.record(stream)
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in evs]
        serial = {"ms_mean": sum(ms) / len(ms), "ms_median": sorted(ms)[len(ms) // 2],
                  "ms_min": min(ms), "pixel_iterations_per_s": sum_counts / (sum(ms) / len(ms) / 1e3)}
        log(f"bench: one stream {serial['ms_mean']:.3f} ms/step")

    # The dominant kernel alone: the same learned order computed once through the
    # public calls, then only the ordered render (clear + render kernels) between events.
    if params is not None:
        keys = native.mlp_forward(params, plan.features(stream=stream), stream=stream)
    else:
        keys = native.cost_targets(cost, stream=stream)  # profile runs: true-cost order
    lperm = native.order_desc(keys, stream=stream)
    rev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in rev:
        a.record(stream)
        plan.launch(out, mode="ordered", order=lperm, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    render_ms = sum(a.elapsed_time(b) for a, b in rev) / len(rev)
    render_tflops = FLOPS_PER_ITER * sum_counts / (render_ms / 1e3) / 1e12
    log(f"bench: ordered render alone {render_ms:.3f} ms, {render_tflops:.2f} TFLOP/s")
    if args.profile:
        ms_mean = render_ms
        value = sum_counts / (render_ms / 1e3)
        tflops = render_tflops
    comp = None
    per = None
    outp = None
    kernels = None
    ceiling = None
    if not args.profile:
        # measured FP64 ceilings: fma chains, and the bare update loop (no test, no scheduling)
        ceiling = {"fma_chain": native.fp64_probe(0), "update_loop": native.fp64_probe(1),
                   "update_loop_2_pixels_per_lane": native.fp64_probe(2)}
        best = max(ceiling["update_loop"]["tflops"],
                   ceiling["update_loop_2_pixels_per_lane"]["tflops"])
        ceiling["render_frac_of_update_loop"] = render_tflops / best
        # independent FMA chains issue at most one FP64 FMA per lane per clock: their rate
        # over the nominal peak bounds the clock under FP64 load from below, and the
        # render's share of that rate is its fraction of the clock-adjusted peak
        ceiling["fp64_clock_ghz_lower_bound"] = 2.4 * ceiling["fma_chain"]["tflops"] / FP64_PEAK_TFLOPS
        ceiling["render_frac_of_clock_adjusted_peak"] = render_tflops / ceiling["fma_chain"]["tflops"]
        log(f"bench: fp64 ceilings fma {ceiling['fma_chain']['tflops']:.1f}, update loop "
            f"{best:.1f} TFLOP/s")
        comp = comparisons(torch, native, view, plan, out, cost, sum_counts, stream, params)
        comp["paper_partitions_one_view"] = view_partitions(
            torch, native, view, out.clone(), sum_counts, int(dinfo["compute_units"]),
            clock_khz, ms_mean)
        comp["render_kernel_ms"] = render_ms
        per = periodicity(torch, native, view, plan, out, sum_counts, serial["ms_mean"],
                          clock_khz, stream)
        if params is not None:
            comp["tail_analysis"] = tail_analysis(torch, native, plan, out, params, cost,
                                                  clock_khz, stream)
        outp = output_path(torch, native, out, view, step, stream)
        import numpy as np
        f = plan.features().cpu().numpy()[:, 4:].astype(np.float64)
        cap = min(view.max_iter, 128)
        probe_iters = int(np.rint(np.exp(f * np.log1p(cap)) - 1).sum())
        kernels = secondary_kernels(torch, native, plan, params, probe_iters, 3)

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
                   "policy": "hipGraph: probe features -> cost-model MLP -> descending "
                             "order -> persistent ordered tile queue, 64x8 tiles; "
                             "consecutive steps alternate over two streams",
                   "parallelism": "single GPU"},
        "sum_counts": sum_counts,
        "fp64_tflops": tflops,
        "pct_fp64_peak": 100.0 * tflops / FP64_PEAK_TFLOPS,
        "lane_occupancy": lane_occ,
        # the device queue replaces the paper's FCFS messages (2 per row, Eq. (fcfs_m))
        "queue_claims_per_step": st[3],
        "paper_fcfs_messages_same_rows": 2 * view.m,
        "tail": tail_fraction(st, clock_khz),
        "wall_s": wall,
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "one_stream": serial,
        "device": dinfo,
        "roofline": {"bound": "alu", "achieved": render_tflops, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": render_tflops / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "kernel": "render_kernel (ordered queue, batch, deferred tests)",
                     "flops_per_launch": FLOPS_PER_ITER * sum_counts,
                     "launch_ms": render_ms},
        "kernel_code_sha256_16": kernel_sha(),
        "profile_run": bool(args.profile),
        "cost_model": cm_info,
        "comparisons": comp,
        "secondary_kernels": kernels,
        "fp64_ceiling": ceiling,
        "periodicity_detection": per,
        "output_path": outp,
    }
    if not args.profile:
        res["paper_context"] = paper_context(torch, native, workloads)
        res["deep_zoom_double_double"] = deep_zoom(torch, native)
    if not args.no_makespan:
        res["makespan"] = makespans(torch, native, workloads, costmodel, args.makespan_reps,
                                    clock_khz, int(dinfo["compute_units"]))
    if not args.no_stress:
        res["stress_batch"] = stress_batch(torch, native, workloads, costmodel, 1, clock_khz,
                                           params, int(dinfo["compute_units"]),
                                           contiguous_rows=args.stress_contiguous_rows)
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"bench: cpu baseline on {threads} threads")
        res["cpu_baseline"] = cpu_baseline(view, args.cpu_rows_step, threads)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
