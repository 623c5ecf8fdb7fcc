"""Command line: render one view on the GPU and write it as a PPM file, reporting
the computation time and the total time including the file write (the two times
the paper reports for each run, Sec. IV).

    python -m paper_2007_00745_amd --size 8000 8000 --max-iter 2000 --radius 400 \\
        --bounds -2 1 -1.2 1.2 --out mandelbrot.ppm
    python -m paper_2007_00745_amd --size 2048 2048 --max-iter 20000 \\
        --centre -0.7436438870371587 0.1318259042053119 --pitch 1e-17 --double-double \\
        --out deep.ppm

The window is given by its bounds (re_min re_max im_min im_max) or by its centre and
pixel pitch.  --schedule picks the work partition: fcfs (device queue, default),
static or alternating rows over --workers workgroups (paper Sec. III-A, III-C).
With --periodicity the FCFS render runs from a one-view plan with row stealing.
--collapse-rows 1 renders rows that share their imaginary part in binary64 once (deep
zooms below binary64 resolution), 2 also rows that are conjugates of each other (a
window centred on the real axis); the image is the same, and the executed iterations
are reported apart from the image's sum of counts.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2007_00745_amd",
                                 description="escape-time Mandelbrot on the GPU -> PPM")
    ap.add_argument("--size", type=int, nargs=2, metavar=("ROWS", "COLS"), default=(480, 640))
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--radius", type=float, default=2.0)
    ap.add_argument("--bounds", type=float, nargs=4,
                    metavar=("RE_MIN", "RE_MAX", "IM_MIN", "IM_MAX"))
    ap.add_argument("--centre", type=float, nargs=2, metavar=("RE", "IM"))
    ap.add_argument("--pitch", type=float, help="pixel pitch (with --centre)")
    ap.add_argument("--schedule", choices=("fcfs", "static", "alternating"), default="fcfs")
    ap.add_argument("--workers", type=int, default=0, help="workgroups for row schedules")
    ap.add_argument("--periodicity", action="store_true",
                    help="exact periodicity detection (same image, less work)")
    ap.add_argument("--block-iters", type=int, default=0,
                    help="longest block of untested updates (default 1024, and 128 with "
                         "--periodicity: a cycle is found one block after the orbit reaches "
                         "it, so shorter blocks find it sooner)")
    ap.add_argument("--collapse-rows", type=int, choices=(0, 1, 2), default=0,
                    help="render rows with equal (1) or equal and opposite (2) imaginary "
                         "parts once, then copy them (same image)")
    ap.add_argument("--double-double", action="store_true",
                    help="double-double arithmetic for pitches below binary64 resolution")
    ap.add_argument("--out", default="mandelbrot.ppm")
    args = ap.parse_args(argv)

    import torch

    from . import native, workloads
    m, n = args.size
    if args.centre is not None:
        if not args.pitch:
            ap.error("--centre needs --pitch")
        cx, cy, dx, dy = args.centre[0], args.centre[1], args.pitch, args.pitch
    else:
        b = args.bounds or (-2.0, 1.0, -1.2, 1.2)
        cx, cy, dx, dy = workloads.window_from_bounds(b[0], b[1], b[2], b[3], m, n)
    if args.double_double and (args.schedule != "fcfs" or args.periodicity or
                               args.collapse_rows):
        ap.error("--double-double uses the FCFS queue without periodicity detection or "
                 "collapsed rows")
    if args.collapse_rows and args.schedule != "fcfs":
        ap.error("--collapse-rows renders from a one-view plan with the FCFS queue")
    if args.schedule != "fcfs" and args.workers < 1:
        args.workers = m

    out = torch.empty((m, n), dtype=torch.int32, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    native.lib()
    plan = None
    if (args.periodicity or args.collapse_rows) and args.schedule == "fcfs":
        # a one-view plan: for row stealing (the tiles whose orbits never settle on a
        # short cycle are the tail, and stealing spreads their rows over idle wavefronts)
        # and for collapsed rows
        plan = native.Plan([workloads.View((cx, cy, dx, dy), m, n, args.max_iter, args.radius)],
                           {"block_iters": args.block_iters or (128 if args.periodicity
                                                                else 1024),
                            "collapse_rows": args.collapse_rows,
                            # row stealing takes whole tiles; otherwise as mandel_render
                            "tile_parts": 1 if args.periodicity else native.TILE_PARTS_AUTO})
    torch.cuda.synchronize()  # device, library and plan set-up stay outside the timed part
    t0 = time.perf_counter()
    a.record()
    if plan is not None:
        per = int(args.periodicity)
        plan.launch(out.view(-1), periodicity=per, steal=per, stats=stats)
    elif args.double_double:
        native.render_dd((cx, 0.0, cy, 0.0, dx, dy), m, n, args.max_iter, args.radius, out=out,
                         stats=stats)
    else:
        kw = {"policy": args.schedule, "periodicity": int(args.periodicity), "stats": stats,
              "block_iters": args.block_iters or (128 if args.periodicity else 1024)}
        if args.schedule != "fcfs":
            kw["workers"] = args.workers
        else:
            kw["tile_parts"] = native.TILE_PARTS_AUTO  # as mandel_render does
        native.render_sched((cx, cy, dx, dy), m, n, args.max_iter, args.radius, out=out, **kw)
    b.record()
    rgb = native.colour_boolean(out, args.max_iter)
    host = rgb.cpu()
    native.write_ppm(args.out, host, m, n)
    total = time.perf_counter() - t0
    if plan is not None:
        plan.close()
    counts = int(out.sum(dtype=torch.int64).item())
    skipped = 0 if args.double_double else int(stats[7].item())
    # counts of the rendered pixels (all of them unless rows were collapsed), less the
    # updates that periodicity detection skipped
    executed = int(stats[1].item()) - skipped
    compute_ms = a.elapsed_time(b)
    print(json.dumps({"file": args.out, "rows": m, "cols": n, "max_iter": args.max_iter,
                      "sum_counts": counts, "updates_skipped": skipped,
                      "iterations_executed": executed, "compute_ms": compute_ms,
                      "executed_pixel_iterations_per_s": executed / (compute_ms / 1e3),
                      "total_s_including_write": total}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
