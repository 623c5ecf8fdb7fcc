"""The host runtime helpers with the GPU: the autotune cache file round trip on
a real batch, and the watchdog waiting for a real render."""
import torch
import pytest

from paper_2007_00745_amd import native, runtime, workloads

pytestmark = pytest.mark.gpu


def test_autotune_cache_round_trip(tmp_path):
    views = workloads.c3_scaled(745, 8, scale=16)
    path = str(tmp_path / "tune.json")
    t1, hit1 = runtime.autotune_cached(views, path, max_sample=4)
    t2, hit2 = runtime.autotune_cached(views, path, max_sample=4)
    assert not hit1 and hit2 and t1 == t2
    plan = native.Plan(views, t2)
    assert plan.tuning["tile_w"] == t2["tile_w"] and plan.tuning["tile_h"] == t2["tile_h"]
    plan.close()


def test_watchdog_on_a_render():
    v = workloads.c2(2048, 5000)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = native.render(v.window, v.m, v.n, v.max_iter, v.R, stream=s)
    waited = runtime.wait(s, timeout=60.0)
    assert waited >= 0.0 and int(out.min()) >= 1
