"""Double-double escape-time oracle (TEST INFRASTRUCTURE ONLY: imported by the
tests, never by the library).

The arithmetic and the definition live in ``mandel_dd_oracle.c``; this module
builds that file with gcc and wraps it with ctypes.  A window is
(cx0_hi, cx0_lo, cy0_hi, cy0_lo, dx, dy): a double-double centre and binary64
pixel pitches.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mandel_dd_oracle.c")
_LIB = os.path.join(_HERE, "libmandel_dd_oracle.so")
CFLAGS = ["-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

OPS = {"two_sum": 0, "quick_two_sum": 1, "two_prod": 2, "add": 3, "sqr": 4, "mul": 5}

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            L = ctypes.CDLL(_LIB)
            d, i32, i64, P = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
            L.oracle_dd_op.argtypes = [i32, d, d, d, d, P, P]
            L.oracle_dd_op.restype = None
            L.oracle_dd_pixel_c.argtypes = [P, i32, i32, i64, i64, P]
            L.oracle_dd_pixel_c.restype = None
            L.oracle_dd_escape_count.argtypes = [P, i32, d]
            L.oracle_dd_escape_count.restype = i32
            L.oracle_dd_render_pixels.argtypes = [P, i32, i32, i32, d, P, i64, P]
            L.oracle_dd_render_pixels.restype = None
            L.oracle_dd_render.argtypes = [P, i32, i32, i32, d, P]
            L.oracle_dd_render.restype = None
            _lib = L
    return _lib


def _win(window) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(window, dtype=np.float64).reshape(6))


def op(name: str, a, b=(0.0, 0.0)) -> tuple[float, float]:
    """One double-double operation; a and b are (hi, lo) pairs (the error-free
    transformations read only the high parts)."""
    rh, rl = ctypes.c_double(), ctypes.c_double()
    lib().oracle_dd_op(OPS[name], float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                       ctypes.byref(rh), ctypes.byref(rl))
    return rh.value, rl.value


def pixel_c(window, m: int, n: int, i: int, j: int) -> tuple[float, float, float, float]:
    w = _win(window)
    c = np.empty(4, dtype=np.float64)
    lib().oracle_dd_pixel_c(w.ctypes.data, m, n, i, j, c.ctypes.data)
    return tuple(float(v) for v in c)


def escape_count(c, max_iter: int, R: float) -> int:
    """c = (cx_hi, cx_lo, cy_hi, cy_lo)."""
    cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(4))
    return int(lib().oracle_dd_escape_count(cc.ctypes.data, int(max_iter), float(R)))


def render(window, m: int, n: int, max_iter: int, R: float) -> np.ndarray:
    w = _win(window)
    out = np.empty((m, n), dtype=np.int32)
    lib().oracle_dd_render(w.ctypes.data, m, n, int(max_iter), float(R), out.ctypes.data)
    return out


def render_pixels(window, m: int, n: int, max_iter: int, R: float, idx,
                  threads: int = 1) -> np.ndarray:
    """Counts of selected pixels (flat row-major indices), split over threads."""
    w = _win(window)
    idx = np.ascontiguousarray(idx, dtype=np.int64).ravel()
    out = np.empty(idx.shape, dtype=np.int32)
    L = lib()
    chunks = [c for c in np.array_split(np.arange(idx.size), max(1, threads)) if c.size]
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        futs = [ex.submit(L.oracle_dd_render_pixels, w.ctypes.data, m, n, int(max_iter),
                          float(R), idx.ctypes.data + 8 * int(c[0]), int(c.size),
                          out.ctypes.data + 4 * int(c[0])) for c in chunks]
        for f in futs:
            f.result()
    return out
