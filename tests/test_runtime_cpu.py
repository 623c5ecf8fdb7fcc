"""Host runtime helpers on the CPU: the autotune cache file (a hit never calls
the library, a miss writes the file) and the stream watchdog (returns when the
stream drains, raises on timeout)."""
import json

import pytest

from paper_2007_00745_amd import native, runtime, workloads


class _FakeStream:
    def __init__(self, busy_polls):
        self.left = busy_polls

    def query(self):
        self.left -= 1
        return self.left < 0


def test_watchdog_returns_and_times_out():
    assert runtime.wait(_FakeStream(3), timeout=1.0, poll=1e-4) >= 0.0
    with pytest.raises(TimeoutError):
        runtime.wait(_FakeStream(10 ** 9), timeout=0.02, poll=1e-3)


def test_signature_keys_every_field_the_library_keys():
    # the file cache keys on what the library's in-process cache keys on (size,
    # max_iter, radius and window of the views, in order) and on the sample size, so
    # the two caches cannot hand out a tuning for different batches
    v1 = workloads.View((0.0, 0.0, 1e-3, 1e-3), 10, 20, 100)
    a = [v1, workloads.c1()]
    assert runtime.batch_signature(a) == runtime.batch_signature(list(a))
    variants = [
        [workloads.View((0.5, 0.0, 1e-3, 1e-3), 10, 20, 100), workloads.c1()],   # centre
        [workloads.View((0.0, 0.0, 1e-4, 1e-3), 10, 20, 100), workloads.c1()],   # zoom
        [workloads.View((0.0, 0.0, 1e-3, 1e-3), 10, 20, 101), workloads.c1()],   # max_iter
        [workloads.View((0.0, 0.0, 1e-3, 1e-3), 10, 20, 100, 3.0), workloads.c1()],  # R
        [workloads.View((0.0, 0.0, 1e-3, 1e-3), 11, 20, 100), workloads.c1()],   # rows
        [workloads.c1(), v1],                                                     # order
    ]
    sigs = {runtime.batch_signature(b) for b in variants}
    assert len(sigs) == len(variants) and runtime.batch_signature(a) not in sigs
    assert runtime.batch_signature(a, 8) != runtime.batch_signature(a, 4)


def test_autotune_cache_file(tmp_path, monkeypatch):
    views = [workloads.c1()]
    calls = []

    def fake_autotune(v, max_sample=8, stream=None):
        calls.append(len(v))
        return {"tile_w": 32, "tile_h": 4}, 15

    monkeypatch.setattr(native, "autotune", fake_autotune)
    path = str(tmp_path / "tune.json")
    t1, hit1 = runtime.autotune_cached(views, path, device_name="dev0")
    t2, hit2 = runtime.autotune_cached(views, path, device_name="dev0")
    t3, hit3 = runtime.autotune_cached(views, path, device_name="dev1")
    assert (hit1, hit2, hit3) == (False, True, False) and calls == [1, 1]
    assert t1 == t2 == t3 == {"tile_w": 32, "tile_h": 4}
    assert len(json.load(open(path))) == 2


def _tune_in_child(path, m, q):
    # a separate process adds its own batch to the shared cache file
    from paper_2007_00745_amd import native as nat, runtime as rt, workloads as wl
    nat.autotune = lambda v, max_sample=8, stream=None: ({"tile_w": 8 + m % 7, "tile_h": 4}, 1)
    q.put(rt.autotune_cached([wl.View((0.0, 0.0, 1e-3, 1e-3), m, 16, 100)], path,
                             device_name="dev0")[1])


def test_autotune_cache_file_shared_by_processes(tmp_path):
    # eight processes add eight different batches at once: no entry is lost
    import multiprocessing as mp
    path = str(tmp_path / "tune.json")
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    procs = [ctx.Process(target=_tune_in_child, args=(path, 10 + k, q)) for k in range(8)]
    for p in procs:
        p.start()
    for p in procs:
        p.join(60)
        assert p.exitcode == 0
    hits = [q.get(timeout=5) for _ in procs]
    assert hits == [False] * 8
    assert len(json.load(open(path))) == 8
