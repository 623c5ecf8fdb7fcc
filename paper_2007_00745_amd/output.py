"""The paper's output path on one GPU: render -> Boolean colouring -> copy to
host -> PPM file (Sec. III: the master writes the image file), for one image or
a sequence of views.

In the pipelined form the GPU renders and colours view k + 1 while a host
thread writes view k: the device work goes to one stream, the copies land in
two pinned host buffers used in turn, and the writer waits on each copy's
event.  Every step is a library call (mandel_plan_launch, mandel_colour_boolean,
mandel_write_ppm); this module only orders them.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

from . import native


def render_to_ppm(views, paths, pipelined: bool = True, mode: str = "fcfs", mlp=None,
                  stream=None) -> dict:
    """Renders each view (one single-view plan per view) and writes it to the
    matching path.  Returns the wall time of the whole sequence and of its parts
    (device time from events; host write time measured around each write)."""
    import torch
    assert len(views) == len(paths)
    dev = torch.device("cuda")
    s = stream or torch.cuda.current_stream()
    plans = [native.Plan([v]) for v in views]
    npx = max(v.pixels for v in views)
    counts = torch.empty(max(npx, 1), dtype=torch.int32, device=dev)
    rgb = torch.empty(max(3 * npx, 1), dtype=torch.uint8, device=dev)
    host = [torch.empty(max(3 * npx, 1), dtype=torch.uint8, pin_memory=True) for _ in range(2)]
    copied = [torch.cuda.Event() for _ in range(2)]
    writes = []

    def write(k, buf):
        t0 = time.perf_counter()
        native.write_ppm(paths[k], host[buf][:3 * views[k].pixels], views[k].m, views[k].n)
        writes.append(time.perf_counter() - t0)

    kw = {"mlp": mlp} if mode == "learned" else {}
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=1) as pool:
        pending = [None, None]
        for k, (v, plan) in enumerate(zip(views, plans)):
            buf = k % 2
            if pending[buf] is not None:       # the writer still reads this buffer
                pending[buf].result()
                pending[buf] = None
            with torch.cuda.stream(s):
                plan.launch(counts, mode=mode, stream=s, **kw)
                native.colour_boolean(counts[:v.pixels], v.max_iter, rgb[:3 * v.pixels],
                                      stream=s)
                host[buf][:3 * v.pixels].copy_(rgb[:3 * v.pixels], non_blocking=True)
                copied[buf].record(s)
            if pipelined:
                def job(k=k, buf=buf):
                    copied[buf].synchronize()
                    write(k, buf)
                pending[buf] = pool.submit(job)
            else:
                copied[buf].synchronize()
                write(k, buf)
        for p in pending:
            if p is not None:
                p.result()
    total = time.perf_counter() - t0
    for p in plans:
        p.close()
    return {"seconds": total, "write_seconds": sum(writes), "frames": len(views),
            "pipelined": pipelined}
