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

OK, EINVAL, ENOMEM, EHIP, EIO = 0, -1, -2, -3, -4

FCFS_TILES, STATIC_ROWS, ALTERNATING_ROWS, ORDERED_TILES, GRID_TILES = 0, 1, 2, 3, 4
TILE_PARTS_AUTO = -1  # mandel_sched.tile_parts: row parts chosen from the image size
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


class WindowDD(ctypes.Structure):
    _fields_ = [("cx0_hi", ctypes.c_double), ("cx0_lo", ctypes.c_double),
                ("cy0_hi", ctypes.c_double), ("cy0_lo", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double)]


class Sched(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("grain", ctypes.c_int32),
                ("workers", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("block_iters", ctypes.c_int32),
                ("young_iters", ctypes.c_int32), ("refill_lanes", ctypes.c_int32),
                ("order", ctypes.c_void_p), ("tile_cost", ctypes.c_void_p),
                ("claims", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("tile_parts", ctypes.c_int32), ("periodicity", ctypes.c_int32),
                ("first_slot", ctypes.c_int64), ("tile_time", ctypes.c_void_p)]


class ViewC(ctypes.Structure):
    _fields_ = [("w", Window), ("m", ctypes.c_int32), ("n", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("R", ctypes.c_double), ("out_offset", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("grain", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("block_iters", ctypes.c_int32), ("young_iters", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("refill_lanes", ctypes.c_int32),
                ("tile_parts", ctypes.c_int32), ("collapse_rows", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


class LaunchC(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("order", ctypes.c_void_p), ("mlp", ctypes.c_void_p),
                ("tile_cost", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("probe_cap", ctypes.c_int32), ("workers", ctypes.c_int32),
                ("first_slot", ctypes.c_int64), ("periodicity", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tile_time", ctypes.c_void_p),
                ("steal", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


PLAN_MODES = {"fcfs": 0, "ordered": 1, "probe": 2, "learned": 3, "static": 4, "alternating": 5}
NFEAT = 68
MLP_PARAMS = 8777
MLP_NORM = 136
ORDER_BUCKETS = 4096
ORDER_KEY_LO, ORDER_KEY_HI = -2.0, 50.0

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
        L.mandel_render_dd.argtypes = [ctypes.POINTER(WindowDD), i32, i32, i32, d, P, P, P]
        L.mandel_render_dd.restype = ctypes.c_int
        L.mandel_colour_boolean.argtypes = [P, i64, i32, P, P]
        L.mandel_colour_boolean.restype = ctypes.c_int
        L.mandel_write_ppm.argtypes = [ctypes.c_char_p, P, i32, i32]
        L.mandel_write_ppm.restype = ctypes.c_int
        L.mandel_render_sched.argtypes = [ctypes.POINTER(Window), i32, i32, i32, d, P,
                                          ctypes.POINTER(Sched), P]
        L.mandel_render_sched.restype = ctypes.c_int
        L.mandel_render_sched_noalloc.argtypes = [ctypes.POINTER(Window), i32, i32, i32, d, P,
                                                  ctypes.POINTER(Sched), P]
        L.mandel_render_sched_noalloc.restype = ctypes.c_int
        L.mandel_tile_count.argtypes = [i32, i32, i32, i32]
        L.mandel_tile_count.restype = i64
        L.mandel_last_error.argtypes = []
        L.mandel_last_error.restype = ctypes.c_char_p
        L.mandel_version.argtypes = []
        L.mandel_version.restype = ctypes.c_char_p
        L.mandel_plan_create.argtypes = [ctypes.POINTER(ViewC), i32, ctypes.POINTER(Tuning),
                                         ctypes.POINTER(ctypes.c_void_p)]
        L.mandel_plan_create.restype = ctypes.c_int
        L.mandel_plan_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                       ctypes.POINTER(Tuning)]
        L.mandel_plan_info.restype = ctypes.c_int
        L.mandel_plan_launch.argtypes = [P, P, ctypes.POINTER(LaunchC), P]
        L.mandel_plan_launch.restype = ctypes.c_int
        L.mandel_plan_destroy.argtypes = [P]
        L.mandel_plan_destroy.restype = ctypes.c_int
        L.mandel_plan_features.argtypes = [P, P, i32, P]
        L.mandel_plan_features.restype = ctypes.c_int
        L.mandel_mlp_forward.argtypes = [P, P, i64, P, P]
        L.mandel_mlp_forward.restype = ctypes.c_int
        L.mandel_mlp_work_floats.argtypes = [i32]
        L.mandel_mlp_work_floats.restype = i64
        L.mandel_mlp_train_step.argtypes = [P, P, P, i32, P, P, P, i32, ctypes.c_float, P, P, P]
        L.mandel_mlp_train_step.restype = ctypes.c_int
        L.mandel_order_desc.argtypes = [P, i64, P, P]
        L.mandel_order_desc.restype = ctypes.c_int
        L.mandel_mlp_set_norm.argtypes = [P, P, i64, P]
        L.mandel_mlp_set_norm.restype = ctypes.c_int
        L.mandel_cost_targets.argtypes = [P, i64, P, P]
        L.mandel_cost_targets.restype = ctypes.c_int
        L.mandel_plan_autotune.argtypes = [ctypes.POINTER(ViewC), i32, i32,
                                           ctypes.POINTER(Tuning), ctypes.POINTER(i32), P]
        L.mandel_plan_autotune.restype = ctypes.c_int
        L.mandel_device_info.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.mandel_device_info.restype = ctypes.c_int
        L.mandel_fp64_probe.argtypes = [i32, i32, i32, P, ctypes.POINTER(d),
                                        ctypes.POINTER(ctypes.c_float), P]
        L.mandel_fp64_probe.restype = ctypes.c_int
        _lib = L
        return L


def check(rc: int) -> None:
    if rc != OK:
        raise MandelError(rc, lib().mandel_last_error().decode())


def _ptr(t) -> int:
    if t is None:
        return None
    return t.data_ptr()


def _dev(t, dtype, numel: int, name: str):
    """Device pointer of an optional buffer (None -> NULL) after checking what the
    library will read or write through it: element type, contiguity, at least
    `numel` elements, GPU memory.  A wrong buffer raises here instead of reaching
    a kernel."""
    if t is None:
        return None
    dts = dtype if isinstance(dtype, tuple) else (dtype,)
    if t.dtype not in dts:
        raise ValueError(f"{name} must be {' or '.join(str(d) for d in dts)}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs at least {numel}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    return t.data_ptr()


def _i64():
    import torch
    u64 = getattr(torch, "uint64", None)
    return (torch.int64,) if u64 is None else (torch.int64, u64)


def _f32():
    import torch
    return torch.float32


def _i32():
    import torch
    return torch.int32


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


def render_dd(window, m: int, n: int, max_iter: int, R: float, out=None, stats=None,
              stream=None):
    """mandel_render_dd: double-double deep-zoom counts.  window = (cx0_hi, cx0_lo,
    cy0_hi, cy0_lo, dx, dy).  Returns the (m, n) int32 tensor."""
    out = _out(out, m, n)
    w = WindowDD(*[float(v) for v in window])
    st = _dev(stats, _i64(), 4, "stats")
    check(lib().mandel_render_dd(ctypes.byref(w), m, n, int(max_iter), float(R), _ptr(out),
                                 st, _stream(stream)))
    return out


def colour_boolean(counts, max_iter: int, rgb=None, stream=None):
    """mandel_colour_boolean: device counts (int32, any shape) -> device RGB bytes,
    shape counts.shape + (3,)."""
    import torch
    if rgb is None:
        rgb = torch.empty(tuple(counts.shape) + (3,), dtype=torch.uint8, device=counts.device)
    npix = counts.numel()
    cp = _dev(counts, torch.int32, npix, "counts")
    rp = _dev(rgb, torch.uint8, 3 * npix, "rgb")
    check(lib().mandel_colour_boolean(cp, npix, int(max_iter), rp, _stream(stream)))
    return rgb


def write_ppm(path: str, rgb, m: int, n: int) -> None:
    """mandel_write_ppm: rgb is host memory (a contiguous CPU tensor or numpy array)
    of 3 * m * n bytes."""
    ptr = rgb.data_ptr() if hasattr(rgb, "data_ptr") else rgb.ctypes.data
    check(lib().mandel_write_ppm(os.fsencode(path), ptr, int(m), int(n)))


def make_sched(policy="fcfs", tile_w=0, tile_h=0, grain=0, workers=0, waves_per_group=0,
               check_every=0, block_iters=0, young_iters=0, refill_lanes=0, order=None,
               tile_cost=None, claims=None, stats=None, tile_parts=0, first_slot=0,
               periodicity=0, tile_time=None) -> Sched:
    """The mandel_sched struct as given (pointers unchecked: render_sched checks them)."""
    pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
    return Sched(pol, tile_w, tile_h, grain, workers, waves_per_group, check_every,
                 block_iters, young_iters, refill_lanes, _ptr(order), _ptr(tile_cost),
                 _ptr(claims), _ptr(stats), tile_parts, int(periodicity), first_slot,
                 _ptr(tile_time))


def render_sched(window, m: int, n: int, max_iter: int, R: float, out=None, stream=None,
                 noalloc: bool = False, **sched):
    """mandel_render_sched with the schedule fields of mandel_sched as keywords.  The
    optional buffers are checked against the sizes this call implies.  noalloc=True
    calls mandel_render_sched_noalloc instead (queue head in the library's static
    device scratch; calls that overlap in time on one GPU race)."""
    out = _out(out, m, n)
    pol = sched.get("policy", "fcfs")
    pol = POLICIES[pol] if isinstance(pol, str) else int(pol)
    rows = pol in (STATIC_ROWS, ALTERNATING_ROWS)
    nt = 0
    if m > 0 and n > 0 and not rows:
        nt = max(tile_count(m, n, sched.get("tile_w") or 64, sched.get("tile_h") or 8), 0)
    for key, dt, size in (("order", _i32(), nt), ("tile_cost", _i64(), nt),
                          ("claims", _i32(), m if rows else nt), ("stats", _i64(), 8),
                          ("tile_time", _i64(), 2 * nt)):
        if sched.get(key) is not None:
            _dev(sched[key], dt, size, key)
    s = make_sched(**sched)
    w = Window(*[float(v) for v in window])
    fn = lib().mandel_render_sched_noalloc if noalloc else lib().mandel_render_sched
    check(fn(ctypes.byref(w), m, n, int(max_iter), float(R), _ptr(out), ctypes.byref(s),
             _stream(stream)))
    return out


# ---- batches ----------------------------------------------------------------

def _view_array(views, offs):
    arr = (ViewC * len(views))()
    for k, v in enumerate(views):
        arr[k] = ViewC(Window(*[float(t) for t in v.window]), int(v.m), int(v.n),
                       int(v.max_iter), 0, float(v.R), int(offs[k]))
    return arr


def _packed_offsets(views):
    offs, acc = [], 0
    for v in views:
        offs.append(acc)
        acc += v.m * v.n
    return offs


def autotune(views, max_sample: int = 8, stream=None) -> tuple[dict, int]:
    """mandel_plan_autotune: (chosen tuning, number of timed trial launches)."""
    arr = _view_array(views, _packed_offsets(views))
    best, trials = Tuning(), ctypes.c_int32()
    check(lib().mandel_plan_autotune(arr, len(views), int(max_sample), ctypes.byref(best),
                                     ctypes.byref(trials), _stream(stream)))
    return best.as_dict(), int(trials.value)


class Plan:
    """A batch plan (mandel_plan_*): views rendered by one persistent launch."""

    def __init__(self, views, tuning: dict | None = None, out_offsets=None):
        n = len(views)
        offs = _packed_offsets(views) if out_offsets is None else list(out_offsets)
        arr = _view_array(views, offs)
        tu = Tuning(**(tuning or {}))
        h = ctypes.c_void_p()
        check(lib().mandel_plan_create(arr, n, ctypes.byref(tu), ctypes.byref(h)))
        self._h = h
        self.views = list(views)
        self.out_offsets = list(offs)
        nt, npx, t = ctypes.c_int64(), ctypes.c_int64(), Tuning()
        check(lib().mandel_plan_info(h, ctypes.byref(nt), ctypes.byref(npx), ctypes.byref(t)))
        self.ntiles, self.npixels, self.tuning = int(nt.value), int(npx.value), t.as_dict()

    def out_size(self) -> int:
        return max((o + v.m * v.n for o, v in zip(self.out_offsets, self.views)), default=0)

    def launch(self, out, mode="fcfs", use_graph=False, order=None, mlp=None, tile_cost=None,
               stats=None, probe_cap=0, first_slot=0, workers=0, periodicity=0, tile_time=None,
               steal=0, stream=None):
        nt = self.ntiles
        la = LaunchC(PLAN_MODES[mode] if isinstance(mode, str) else int(mode), int(use_graph),
                     _dev(order, _i32(), nt, "order"), _dev(mlp, _f32(), MLP_PARAMS, "mlp"),
                     _dev(tile_cost, _i64(), nt, "tile_cost"), _dev(stats, _i64(), 8, "stats"),
                     int(probe_cap), int(workers), int(first_slot), int(periodicity), 0,
                     _dev(tile_time, _i64(), 2 * nt, "tile_time"), int(steal), 0)
        op = _dev(out, _i32(), self.out_size(), "out")
        check(lib().mandel_plan_launch(self._h, op, ctypes.byref(la), _stream(stream)))
        return out

    def features(self, feat=None, probe_cap: int = 0, stream=None):
        import torch
        if feat is None:
            feat = torch.empty((self.ntiles, NFEAT), dtype=torch.float32, device="cuda")
        fp = _dev(feat, torch.float32, self.ntiles * NFEAT, "feat")
        check(lib().mandel_plan_features(self._h, fp, int(probe_cap), _stream(stream)))
        return feat

    def view_images(self, out):
        """Split a packed output buffer into per-view (m, n) tensors."""
        return [out[o:o + v.m * v.n].view(v.m, v.n) for o, v in zip(self.out_offsets, self.views)]

    def close(self):
        if getattr(self, "_h", None):
            lib().mandel_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- cost model and ordering ----------------------------------------------------

def mlp_forward(params, x, y=None, stream=None):
    import torch
    n = x.shape[0]
    if y is None:
        y = torch.empty(n, dtype=torch.float32, device=x.device)
    check(lib().mandel_mlp_forward(_dev(params, torch.float32, MLP_PARAMS, "params"),
                                   _dev(x, torch.float32, n * NFEAT, "x"),
                                   n, _dev(y, torch.float32, n, "y"), _stream(stream)))
    return y


def mlp_work_floats(batch: int) -> int:
    return int(lib().mandel_mlp_work_floats(batch))


def mlp_train_step(params, m, v, t: int, x, target, idx, lr: float, loss=None, work=None,
                   stream=None):
    import torch
    B = idx.numel()
    if work is None:
        work = torch.empty(mlp_work_floats(B), dtype=torch.float32, device=x.device)
    f32 = torch.float32
    nx = x.shape[0]
    check(lib().mandel_mlp_train_step(
        _dev(params, f32, MLP_PARAMS, "params"), _dev(m, f32, MLP_PARAMS, "adam_m"),
        _dev(v, f32, MLP_PARAMS, "adam_v"), int(t), _dev(x, f32, nx * NFEAT, "x"),
        _dev(target, f32, nx, "target"), _dev(idx, torch.int32, B, "idx"), B, float(lr),
        _dev(loss, f32, 1, "loss"), _dev(work, f32, mlp_work_floats(B), "work"),
        _stream(stream)))
    return work


def order_desc(keys, perm=None, stream=None):
    import torch
    n = keys.numel()
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=keys.device)
    check(lib().mandel_order_desc(_dev(keys, torch.float32, n, "keys"), n,
                                  _dev(perm, torch.int32, n, "perm"), _stream(stream)))
    return perm


def mlp_set_norm(params, feat, stream=None):
    import torch
    n = feat.shape[0]
    check(lib().mandel_mlp_set_norm(_dev(params, torch.float32, MLP_PARAMS, "params"),
                                    _dev(feat, torch.float32, n * NFEAT, "feat"), n,
                                    _stream(stream)))
    return params


def cost_targets(cost, target=None, stream=None):
    import torch
    n = cost.numel()
    if target is None:
        target = torch.empty(n, dtype=torch.float32, device=cost.device)
    check(lib().mandel_cost_targets(_dev(cost, _i64(), n, "cost"), n,
                                    _dev(target, torch.float32, n, "target"), _stream(stream)))
    return target


def device_info() -> dict:
    cus, khz = ctypes.c_int32(), ctypes.c_int32()
    check(lib().mandel_device_info(ctypes.byref(cus), ctypes.byref(khz)))
    return {"compute_units": int(cus.value), "wall_clock_khz": int(khz.value)}


def fp64_probe(kind: int, iters: int = 4000, blocks_per_cu: int = 8, stream=None) -> dict:
    """mandel_fp64_probe: kind 0 fma chains, 1 the bare update, 2 the update on two
    pixels per lane.  Returns flops, milliseconds and TFLOP/s."""
    import torch
    info = device_info()
    sink = torch.empty(info["compute_units"] * blocks_per_cu * 256, dtype=torch.float64,
                       device="cuda")
    fl, ms = ctypes.c_double(), ctypes.c_float()
    check(lib().mandel_fp64_probe(kind, iters, blocks_per_cu, _ptr(sink), ctypes.byref(fl),
                                  ctypes.byref(ms), _stream(stream)))
    return {"flops": fl.value, "ms": ms.value, "tflops": fl.value / (ms.value / 1e3) / 1e12}
