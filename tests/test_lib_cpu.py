"""Host-side checks of libmandel.so that need no GPU: it loads, exports every
entry point that include/mandel.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import subprocess

import pytest

from paper_2007_00745_amd import native


def test_library_exports_header_symbols():
    L = native.lib()
    names = native.exported_names()
    assert "mandel_render" in names and "mandel_render_sched" in names
    for nm in names:
        assert hasattr(L, nm), f"{nm} declared in mandel.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [nm for nm in names if nm not in exported]
    assert not missing, missing


def test_version_and_tile_count():
    L = native.lib()
    assert L.mandel_version().startswith(b"mandel-gfx950")
    assert native.tile_count(480, 640) == 60 * 10
    assert native.tile_count(8192, 8192) == 1024 * 128
    assert native.tile_count(9, 65, 64, 8) == 2 * 2
    assert native.tile_count(0, 65) == 0


def _call(win=(-0.5, 0.0, 0.01, 0.01), m=8, n=8, mi=10, R=2.0, out=0x1000, sched=None):
    L = native.lib()
    w = native.Window(*win)
    if sched is None:
        return L.mandel_render(ctypes.byref(w), m, n, mi, R, out, None)
    return L.mandel_render_sched(ctypes.byref(w), m, n, mi, R, out, ctypes.byref(sched), None)


@pytest.mark.parametrize("kw", [
    dict(m=-1), dict(n=-5), dict(mi=0), dict(mi=(1 << 30) + 1), dict(R=0.0), dict(R=-2.0),
    dict(R=float("nan")), dict(R=float("inf")), dict(R=1e151),
    dict(win=(float("nan"), 0.0, 0.01, 0.01)), dict(win=(0.0, 0.0, 0.0, 0.01)),
    dict(win=(0.0, 0.0, 0.01, -0.01)), dict(win=(0.0, float("inf"), 0.01, 0.01)),
    dict(win=(1e308, 0.0, 1e307, 0.01), n=100), dict(m=1 << 20, n=1 << 20),
])
def test_invalid_arguments(kw):
    assert _call(**kw) == native.EINVAL
    assert native.lib().mandel_last_error()


@pytest.mark.parametrize("kw", [
    dict(m=-1), dict(mi=0), dict(R=float("nan")), dict(win=(0.0, 0.0, 0.0, 0.01)),
    dict(m=1 << 20, n=1 << 20), dict(out=None),
])
def test_noalloc_invalid_arguments(kw):
    # the allocation-free variant checks its arguments as mandel_render_sched does,
    # before it looks up its device scratch
    L = native.lib()
    a = dict(win=(-0.5, 0.0, 0.01, 0.01), m=8, n=8, mi=10, R=2.0, out=0x1000)
    a.update(kw)
    w = native.Window(*a["win"])
    s = native.make_sched()
    assert L.mandel_render_sched_noalloc(ctypes.byref(w), a["m"], a["n"], a["mi"], a["R"],
                                         a["out"], ctypes.byref(s), None) == native.EINVAL
    assert native.lib().mandel_last_error()


def test_null_pointers():
    L = native.lib()
    assert L.mandel_render(None, 8, 8, 10, 2.0, 0x1000, None) == native.EINVAL
    assert _call(out=None) == native.EINVAL


def test_empty_image_is_a_no_op():
    assert _call(m=0, out=None) == native.OK
    assert _call(n=0, out=None) == native.OK


@pytest.mark.parametrize("s", [
    dict(policy=7), dict(policy=1), dict(policy=3), dict(tile_w=-1), dict(grain=-3),
    dict(waves_per_group=17), dict(check_every=2), dict(block_iters=70000), dict(young_iters=-1),
    dict(workers=-1), dict(refill_lanes=65), dict(refill_lanes=-2), dict(tile_parts=65),
    dict(tile_parts=-2), dict(tile_parts=-1, first_slot=3), dict(first_slot=-1), dict(policy="static", workers=3, first_slot=2),
    dict(policy="grid", first_slot=1), dict(periodicity=2), dict(periodicity=1, check_every=1),
])
def test_invalid_schedules(s):
    sched = native.make_sched(**s)
    assert _call(sched=sched) == native.EINVAL


class _FakeDevicePtr:
    def data_ptr(self):
        return 0x2000


@pytest.mark.parametrize("policy", ["static", "alternating"])
def test_tile_time_rejected_for_row_policies(policy):
    sched = native.make_sched(policy=policy, workers=4, tile_time=_FakeDevicePtr())
    assert _call(sched=sched) == native.EINVAL


def test_fp64_probe_argument_checks():
    L = native.lib()
    fl, ms = ctypes.c_double(), ctypes.c_float()
    for kind, iters, bpc in ((3, 10, 1), (-1, 10, 1), (0, 0, 1), (0, (1 << 24) + 1, 1), (1, 10, 0),
                             (2, 10, 9)):
        assert L.mandel_fp64_probe(kind, iters, bpc, 0x1000, ctypes.byref(fl), ctypes.byref(ms),
                                   None) == native.EINVAL
    assert L.mandel_fp64_probe(0, 10, 1, None, ctypes.byref(fl), ctypes.byref(ms),
                               None) == native.EINVAL


def _call_dd(win=(-0.5, 0.0, 0.0, 0.0, 0.01, 0.01), m=8, n=8, mi=10, R=2.0, out=0x1000):
    w = native.WindowDD(*win)
    return native.lib().mandel_render_dd(ctypes.byref(w), m, n, mi, R, out, None, None)


@pytest.mark.parametrize("kw", [
    dict(m=-1), dict(mi=0), dict(mi=(1 << 30) + 1), dict(R=0.0), dict(R=1e151),
    dict(win=(float("nan"), 0.0, 0.0, 0.0, 0.01, 0.01)),
    dict(win=(0.0, float("inf"), 0.0, 0.0, 0.01, 0.01)),
    dict(win=(0.0, 0.0, 0.0, 0.0, 0.0, 0.01)), dict(win=(0.0, 0.0, 0.0, 0.0, 0.01, -1e-20)),
    dict(win=(1e150, 0.0, 0.0, 0.0, 1e140, 0.01)), dict(m=1 << 20, n=1 << 20), dict(out=None),
])
def test_dd_invalid_arguments(kw):
    assert _call_dd(**kw) == native.EINVAL
    assert native.lib().mandel_last_error()


def test_dd_empty_image_is_a_no_op():
    assert _call_dd(m=0, out=None) == native.OK
    assert native.lib().mandel_render_dd(None, 4, 4, 10, 2.0, 0x1000, None, None) == native.EINVAL


def test_binding_checks_buffers_before_the_library():
    # every optional device buffer is checked for element type, contiguity, size and
    # GPU residence before its pointer reaches the C ABI (None passes as NULL)
    import torch
    assert native._dev(None, torch.int64, 8, "stats") is None
    with pytest.raises(ValueError, match="stats must be"):
        native._dev(torch.zeros(8, dtype=torch.int32), native._i64(), 8, "stats")
    with pytest.raises(ValueError, match="contiguous"):
        native._dev(torch.zeros(8, 2, dtype=torch.int64).t(), native._i64(), 8, "stats")
    with pytest.raises(ValueError, match="needs at least 8"):
        native._dev(torch.zeros(7, dtype=torch.int64), native._i64(), 8, "stats")
    with pytest.raises(ValueError, match="GPU tensor"):
        native._dev(torch.zeros(8, dtype=torch.int64), native._i64(), 8, "stats")


def test_tile_count_at_extreme_sizes():
    # ceil divisions in 64 bits: m or n near 2^31 must not overflow
    big = 2 ** 31 - 1
    assert native.tile_count(big, 1, 64, 8) == (big + 7) // 8
    assert native.tile_count(1, big, 64, 8) == (big + 63) // 64
    assert native.tile_count(big, 1, 1, 2 ** 20) == (big + 2 ** 20 - 1) // 2 ** 20
    assert native.tile_count(46341, 46341, 64, 8) == 5793 * 725


def test_empty_image_needs_no_order():
    # an empty image is a no-op in every policy: no output buffer and no order array
    sched = native.make_sched(policy="ordered")
    assert _call(m=0, out=None, sched=sched) == native.OK
    assert _call(n=0, out=None, sched=sched) == native.OK
    assert _call(sched=sched) == native.EINVAL   # a real image still needs its order


def test_plan_rejects_bad_collapse_flag():
    v = native.ViewC(native.Window(-0.5, 0.0, 0.01, 0.01), 8, 8, 10, 0, 2.0, 0)
    arr = (native.ViewC * 1)(v)
    t = native.Tuning(collapse_rows=3)
    h = ctypes.c_void_p()
    assert native.lib().mandel_plan_create(arr, 1, ctypes.byref(t), ctypes.byref(h)) == native.EINVAL
    assert b"collapse_rows" in native.lib().mandel_last_error()
