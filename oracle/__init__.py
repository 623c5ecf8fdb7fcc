"""CPU oracle for escape-time Mandelbrot generation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module: only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use it.  It shares no code with the GPU library.

The escape-time definition itself lives in ``mandel_oracle.c`` (paper, Sec. I,
Eq. (1)-(2)); this module builds that file with gcc and wraps it with ctypes.
``partition`` holds the paper's row partitions (Sec. III-A and III-C) and
``mlp`` the FP64 reference of the tile cost model.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mandel_oracle.c")
_LIB = os.path.join(_HERE, "libmandel_oracle.so")
# -ffp-contract=off and no -march: every product and sum is rounded on its own.
CFLAGS = ["-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library next to its source."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            L = ctypes.CDLL(_LIB)
            d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
            P = ctypes.c_void_p
            L.oracle_pixel_c.argtypes = [P, i32, i32, i64, i64, P, P]
            L.oracle_pixel_c.restype = None
            L.oracle_escape_count.argtypes = [d, d, i32, d]
            L.oracle_escape_count.restype = i32
            L.oracle_render.argtypes = [P, i32, i32, i32, d, P]
            L.oracle_render.restype = None
            L.oracle_render_rows.argtypes = [P, i32, i32, i32, d, i64, i64, P]
            L.oracle_render_rows.restype = d
            L.oracle_render_pixels.argtypes = [P, i32, i32, i32, d, P, i64, P]
            L.oracle_render_pixels.restype = None
            L.oracle_escape_counts.argtypes = [P, P, i64, i32, d, P]
            L.oracle_escape_counts.restype = None
            _lib = L
    return _lib


def _win(window) -> np.ndarray:
    w = np.ascontiguousarray(np.asarray(window, dtype=np.float64).reshape(4))
    return w


def escape_count(cx: float, cy: float, max_iter: int, R: float) -> int:
    """Eq. (1)-(2) for a single point c = cx + i*cy."""
    return int(lib().oracle_escape_count(float(cx), float(cy), int(max_iter), float(R)))


def escape_counts(cx, cy, max_iter: int, R: float) -> np.ndarray:
    cx = np.ascontiguousarray(cx, dtype=np.float64).ravel()
    cy = np.ascontiguousarray(cy, dtype=np.float64).ravel()
    assert cx.shape == cy.shape
    out = np.empty(cx.shape, dtype=np.int32)
    lib().oracle_escape_counts(cx.ctypes.data, cy.ctypes.data, cx.size, int(max_iter),
                               float(R), out.ctypes.data)
    return out


def pixel_c(window, m: int, n: int, i: int, j: int) -> tuple[float, float]:
    w = _win(window)
    cx, cy = ctypes.c_double(), ctypes.c_double()
    lib().oracle_pixel_c(w.ctypes.data, m, n, i, j, ctypes.byref(cx), ctypes.byref(cy))
    return cx.value, cy.value


def render(window, m: int, n: int, max_iter: int, R: float) -> np.ndarray:
    """Whole m x n image, single thread, row-major int32."""
    w = _win(window)
    out = np.empty((m, n), dtype=np.int32)
    lib().oracle_render(w.ctypes.data, m, n, int(max_iter), float(R), out.ctypes.data)
    return out


def render_parallel(window, m: int, n: int, max_iter: int, R: float,
                    threads: int | None = None) -> tuple[np.ndarray, float]:
    """Whole image split over independent single-threaded workers on
    alternating rows (worker t takes rows t, t+T, ...).  ctypes drops the GIL
    during each foreign call, so the workers run on separate cores.
    Returns (image, wall seconds)."""
    import time
    T = threads or os.cpu_count() or 1
    w = _win(window)
    out = np.empty((m, n), dtype=np.int32)
    L = lib()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=T) as ex:
        futs = [ex.submit(L.oracle_render_rows, w.ctypes.data, m, n, int(max_iter), float(R),
                          t, T, out.ctypes.data) for t in range(T)]
        for f in futs:
            f.result()
    return out, time.perf_counter() - t0


def render_pixels(window, m: int, n: int, max_iter: int, R: float, idx,
                  threads: int = 1) -> np.ndarray:
    """Counts of selected pixels, given as flat row-major indices."""
    w = _win(window)
    idx = np.ascontiguousarray(idx, dtype=np.int64).ravel()
    out = np.empty(idx.shape, dtype=np.int32)
    L = lib()
    if threads <= 1 or idx.size < 2 * threads:
        L.oracle_render_pixels(w.ctypes.data, m, n, int(max_iter), float(R), idx.ctypes.data,
                               idx.size, out.ctypes.data)
        return out
    chunks = np.array_split(np.arange(idx.size), threads)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = []
        for ch in chunks:
            if ch.size == 0:
                continue
            a, b = int(ch[0]), int(ch[-1]) + 1
            futs.append(ex.submit(L.oracle_render_pixels, w.ctypes.data, m, n, int(max_iter),
                                  float(R), idx.ctypes.data + 8 * a, b - a,
                                  out.ctypes.data + 4 * a))
        for f in futs:
            f.result()
    return out
