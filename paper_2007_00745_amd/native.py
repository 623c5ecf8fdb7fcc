"""ctypes binding of libmandel.so (argument marshalling only).

Every function here checks and converts arguments and calls the C ABI declared
in include/mandel.h; all computation happens in the library's HIP kernels.
PyTorch supplies device memory and the current stream.  If the library has
not been built, ``lib()`` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmandel.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "mandel.h")

OK, EINVAL, ENOMEM, EHIP = 0, -1, -2, -3

FCFS_TILES, STATIC_ROWS, ALTERNATING_ROWS, ORDERED_TILES, GRID_TILES = 0, 1, 2, 3, 4
POLICIES = {
    "fcfs": FCFS_TILES, "static": STATIC_ROWS, "alternating": ALTERNATING_ROWS,
    "ordered": ORDERED_TILES, "grid": GRID_TILES,
}


class MandelError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mandel error {code}: {msg}")
        self.code = code


class Window(ctypes.Structure):
    _fields_ = [("cx0", ctypes.c_double), ("cy0", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double)]


class Sched(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("grain", ctypes.c_int32),
                ("workers", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("block_iters", ctypes.c_int32),
                ("young_iters", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("order", ctypes.c_void_p), ("tile_cost", ctypes.c_void_p),
                ("claims", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


_lock = threading.Lock()
_lib = None


def exported_names() -> list[str]:
    """Function names declared in include/mandel.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mandel_[a-z0-9_]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.mandel_render.argtypes = [ctypes.POINTER(Window), i32, i32, i32, d, P, P]
        L.mandel_render.restype = ctypes.c_int
        L.mandel_render_sched.argtypes = [ctypes.POINTER(Window), i32, i32, i32, d, P,
                                          ctypes.POINTER(Sched), P]
        L.mandel_render_sched.restype = ctypes.c_int
        L.mandel_tile_count.argtypes = [i32, i32, i32, i32]
        L.mandel_tile_count.restype = i64
        L.mandel_last_error.argtypes = []
        L.mandel_last_error.restype = ctypes.c_char_p
        L.mandel_version.argtypes = []
        L.mandel_version.restype = ctypes.c_char_p
        _lib = L
        return L


def check(rc: int) -> None:
    if rc != OK:
        raise MandelError(rc, lib().mandel_last_error().decode())


def _ptr(t) -> int:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _out(out, m: int, n: int, device=None):
    import torch
    if out is None:
        return torch.empty((m, n), dtype=torch.int32, device=device or "cuda")
    if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 CUDA tensor")
    if out.numel() != m * n:
        raise ValueError(f"out has {out.numel()} elements, expected {m}*{n}")
    return out


def tile_count(m: int, n: int, tile_w: int = 64, tile_h: int = 8) -> int:
    return int(lib().mandel_tile_count(m, n, tile_w, tile_h))


def render(window, m: int, n: int, max_iter: int, R: float, out=None, stream=None):
    """mandel_render: one view, FCFS tile queue.  Returns the (m, n) int32 tensor."""
    out = _out(out, m, n)
    w = Window(*[float(v) for v in window])
    check(lib().mandel_render(ctypes.byref(w), m, n, int(max_iter), float(R), _ptr(out),
                              _stream(stream)))
    return out


def make_sched(policy="fcfs", tile_w=0, tile_h=0, grain=0, workers=0, waves_per_group=0,
               check_every=0, block_iters=0, young_iters=0, order=None, tile_cost=None,
               claims=None, stats=None) -> Sched:
    pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
    return Sched(pol, tile_w, tile_h, grain, workers, waves_per_group, check_every,
                 block_iters, young_iters, 0, _ptr(order), _ptr(tile_cost), _ptr(claims),
                 _ptr(stats))


def render_sched(window, m: int, n: int, max_iter: int, R: float, out=None, stream=None,
                 **sched):
    """mandel_render_sched with the schedule fields of mandel_sched as keywords."""
    out = _out(out, m, n)
    s = make_sched(**sched)
    w = Window(*[float(v) for v in window])
    check(lib().mandel_render_sched(ctypes.byref(w), m, n, int(max_iter), float(R), _ptr(out),
                                    ctypes.byref(s), _stream(stream)))
    return out
