"""Host-side runtime helpers around the library: a persistent autotune cache and
a stream watchdog.

* ``autotune_cached(views, path)`` -- the library caches autotune results per
  device and batch signature for the life of the process; this keeps them in a
  JSON file across processes, keyed by the device name, the sample size and the
  batch signature, so a batch seen before is not re-timed.  The signature covers
  every field the library's own cache key is computed from (size, max_iter,
  radius and window of every view, in submission order), so two batches that
  share a file entry would also share the library's entry: zoom and position
  change where the work sits, so a tuning is never reused across them.
* ``wait(stream, timeout)`` -- polls a stream until its work is done or the time
  runs out (then raises TimeoutError, leaving the work running): a host watchdog
  for callers that must not block forever on a device call.
"""
from __future__ import annotations

import fcntl
import hashlib
import json
import os
import time

from . import native


def batch_signature(views, max_sample: int = 8) -> str:
    items = [(v.m, v.n, v.max_iter, float(v.R).hex(), [float(x).hex() for x in v.window])
             for v in views]
    return hashlib.sha256(json.dumps([max_sample, items]).encode()).hexdigest()[:24]


def _read_table(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def autotune_cached(views, path: str, max_sample: int = 8, device_name: str | None = None,
                    stream=None) -> tuple[dict, bool]:
    """(tuning, came_from_file).  A miss autotunes and adds the entry while holding an
    advisory lock on `path`.lock, then rewrites the file atomically, so processes
    that share the file neither lose each other's entries nor tune one batch twice."""
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name()
    key = f"{device_name}|{batch_signature(views, max_sample)}"
    table = _read_table(path)
    if key in table:
        return dict(table[key]), True
    with open(f"{path}.lock", "a") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        try:
            table = _read_table(path)          # another process may have added it
            if key in table:
                return dict(table[key]), True
            tuning, _ = native.autotune(views, max_sample=max_sample, stream=stream)
            table[key] = tuning
            tmp = f"{path}.tmp{os.getpid()}"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        finally:
            fcntl.flock(lock, fcntl.LOCK_UN)
    return tuning, False


def wait(stream, timeout: float, poll: float = 1e-3) -> float:
    """Returns the seconds waited once stream.query() is true; raises TimeoutError
    after `timeout` seconds."""
    t0 = time.perf_counter()
    while not stream.query():
        waited = time.perf_counter() - t0
        if waited > timeout:
            raise TimeoutError(f"stream still busy after {waited:.3f} s")
        time.sleep(poll)
    return time.perf_counter() - t0
