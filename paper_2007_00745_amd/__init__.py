"""Escape-time Mandelbrot generation on MI355X (gfx950).

The compute lives in ``libmandel.so`` (HIP kernels behind the C ABI of
``include/mandel.h``); this package only binds it (``native``) and describes
the synthetic workloads (``workloads``).
"""
from . import native, workloads  # noqa: F401
from .native import MandelError, render, render_sched, tile_count  # noqa: F401

__all__ = ["native", "workloads", "render", "render_sched", "tile_count", "MandelError"]
