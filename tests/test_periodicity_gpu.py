"""GPU parity of exact periodicity detection, an option of the deferred-test
render.  A lane is cut short only when its FP64 state recurs bit for bit inside
a block that ended without an escape, so its orbit is a cycle of non-escaping
states and its count is max_iter: counts must equal the CPU oracle's exactly
(paper Sec. I, Eq. (1)-(2)) for every schedule.  The tests also check that the
detection happens (stats[7], the updates skipped) on orbits whose cycles are
known: the fixed point of c = 0, the 2-cycles of c = -1 and c = i, and the
attracting cycles at the centres of components of period 3, 4, 5 and 7."""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2007_00745_amd import native, workloads

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


# (c, period of the attracting cycle) -- centres of hyperbolic components
CYCLES = [((0.0, 0.0), 1), ((-1.0, 0.0), 2), ((0.0, 1.0), 2),
          ((-0.12256116687665358, 0.7448617666197442), 3), ((-1.754877666246693, 0.0), 3),
          ((-1.3107026413368328, 0.0), 4), ((0.2822713907669139, 0.5300606175785253), 4),
          ((-1.9854242530542052, 0.0), 5), ((-0.504340175446244, 0.562765761452982), 5),
          ((-0.2721024614889389, 0.8423646902941282), 7)]


def test_known_cycles_are_detected():
    mi = 1 << 26
    views = [workloads.View((cx, cy, 1e-3, 1e-3), 1, 1, mi) for (cx, cy), _ in CYCLES]
    want = [oracle.escape_count(cx, cy, mi, 2.0) for (cx, cy), _ in CYCLES]
    assert want == [mi] * len(CYCLES)
    plan = native.Plan(views)
    out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    plan.launch(out, stats=stats, periodicity=1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = stats.cpu().tolist()
    _log(f"cycles: {dt * 1e3:.1f} ms, skipped {st[7]} of {len(CYCLES) * mi}")
    assert out.cpu().tolist() == want
    # each orbit settles within a few hundred updates and is found one block later
    assert st[7] >= len(CYCLES) * (mi - 10000)
    # without detection every lane runs to its deadline and skips nothing
    stats.zero_()
    out.fill_(-1)
    plan.launch(out, stats=stats)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == want and int(stats[7]) == 0
    plan.close()


SCHEDS = [dict(policy="fcfs"), dict(policy="fcfs", tile_w=32, tile_h=4, grain=2),
          dict(policy="fcfs", block_iters=1), dict(policy="fcfs", block_iters=7, young_iters=0),
          dict(policy="fcfs", block_iters=33), dict(policy="fcfs", refill_lanes=1),
          dict(policy="fcfs", refill_lanes=64), dict(policy="fcfs", tile_parts=4),
          dict(policy="grid"), dict(policy="static", workers=37),
          dict(policy="alternating", workers=100, waves_per_group=2)]


@pytest.fixture(scope="module")
def views_and_refs():
    # (view, shortest cycle period among its pixels, or None when no orbit settles
    # within max_iter): the seahorse zoom sits on the cardioid's edge, where orbits
    # converge too slowly; the others hold parts of the cardioid (period 1), the
    # period-3 component, and the period-2 and period-4 components
    vs = [(workloads.c1(), 1),
          (workloads.View((-0.745, 0.113, 0.002 / 96, 0.002 / 96), 80, 96, 3000), None),
          (workloads.View((-0.12, 0.74, 0.05 / 70, 0.05 / 70), 70, 70, 5000), 3),
          (workloads.View((-1.3, 0.0, 0.3 / 64, 0.3 / 64), 33, 64, 2000), 2)]
    return [(v, oracle.render(v.window, v.m, v.n, v.max_iter, v.R), d) for v, d in vs]


@pytest.mark.parametrize("sched", SCHEDS, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_schedules_exact(views_and_refs, sched):
    for v, want, detects in views_and_refs:
        kw = dict(sched)
        if kw["policy"] == "ordered":
            kw["order"] = torch.arange(native.tile_count(v.m, v.n, 64, 8), dtype=torch.int32,
                                       device="cuda")
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        _log(f"periodic {v.m}x{v.n} it={v.max_iter} {sched}")
        got = native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, periodicity=1,
                                  stats=stats, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want)
        st = stats.cpu().tolist()
        assert st[1] == int(want.sum())
        # blocks of L updates compare their last min(L, 32) states: cycles of
        # period <= min(block_iters, 32) are found
        if detects is not None and detects <= min(sched.get("block_iters", 1024), 32):
            assert st[7] > 0


def test_ordered_and_reversed_orders(views_and_refs):
    for v, want, _ in views_and_refs:
        nt = native.tile_count(v.m, v.n, 64, 8)
        for order in (torch.arange(nt - 1, -1, -1), torch.randperm(nt)):
            got = native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, policy="ordered",
                                      order=order.to(torch.int32).cuda(), periodicity=1)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("R", [0.5, 1.999, 2.0, 2.5, 400.0, 1e150])
def test_escape_radii(R):
    # R < 2 has no deferred blocks, so nothing is detected; R >= 2 detects inside the
    # safe disk |c| <= (R^2 - R)(1 - 2^-20)
    win = workloads.window_from_bounds(-2.6, 1.2, -1.6, 1.6, 60, 80)
    v = workloads.View(win, 60, 80, 1500, R)
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    got = native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, periodicity=1, stats=stats)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.render(v.window, v.m, v.n, v.max_iter, R))
    st = stats.cpu().tolist()
    if R < 2.0:
        assert st[7] == 0
    else:
        assert st[7] > 0


def test_plan_modes_and_graph_replays():
    views = workloads.c3_scaled(745, 16, scale=32)
    views += [workloads.View((-0.5, 0.0, 0.01, 0.01), 0, 9, 100), workloads.c1()]
    want = [oracle.render(v.window, v.m, v.n, v.max_iter, v.R) for v in views]
    plan = native.Plan(views)
    perm = torch.randperm(plan.ntiles).to(torch.int32).cuda()
    for mode, kw in (("fcfs", {}), ("ordered", dict(order=perm)), ("probe", {}),
                     ("static", dict(workers=64)), ("alternating", dict(workers=300))):
        for use_graph in (False, True, True):
            out = torch.full((plan.out_size(),), -3, dtype=torch.int32, device="cuda")
            plan.launch(out, mode=mode, use_graph=use_graph, periodicity=1, **kw)
            torch.cuda.synchronize()
            imgs = plan.view_images(out.cpu())
            for k, (g, w) in enumerate(zip(imgs, want)):
                assert np.array_equal(g.numpy(), w), (mode, use_graph, k)
    plan.close()


def test_full_view_8192():
    # The 8192 x 8192 view: identical to the render without detection, the whole image
    # compared on the device, plus pixels against the oracle.
    v = workloads.c2()
    plain = native.render(v.window, v.m, v.n, v.max_iter, v.R)
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    got = native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, periodicity=1, stats=stats)
    torch.cuda.synchronize()
    assert torch.equal(got, plain)
    st = stats.cpu().tolist()
    total = int(plain.sum(dtype=torch.int64).item())
    _log(f"c2 periodic: skipped {st[7]} of {total} ({st[7] / total:.3f})")
    assert st[1] == total and 0 < st[7] < total
    rng = np.random.default_rng(81)
    idx = rng.integers(0, v.pixels, 2000)
    want = oracle.render_pixels(v.window, v.m, v.n, v.max_iter, v.R, idx, threads=16)
    assert np.array_equal(got.view(-1)[torch.tensor(idx, device="cuda")].cpu().numpy(), want)


def test_bench_configuration_8192_short_blocks_stealing():
    # The launch the benchmark times for detection: the 8192 x 8192 view on a plan
    # whose deferred blocks stop at 128 updates, FCFS queue, row stealing, replayed
    # from the graph.  Every pixel against the oracle's whole image (stored digest)
    # and against the render without detection; detection must skip more updates
    # than with the default 1024-update blocks.
    import hashlib
    import json
    import os
    v = workloads.c2()
    plain = native.render(v.window, v.m, v.n, v.max_iter, v.R)
    skipped = {}
    for K, steal in ((1024, 0), (128, 1)):
        plan = native.Plan([v], {"block_iters": K})
        out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
        for _ in range(2):
            out.fill_(-1)
            plan.launch(out, periodicity=1, steal=steal, use_graph=True)
            torch.cuda.synchronize()
            assert torch.equal(out.view(v.m, v.n), plain), (K, steal)
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        plan.launch(out, periodicity=1, steal=steal, stats=stats)
        torch.cuda.synchronize()
        assert torch.equal(out.view(v.m, v.n), plain), (K, steal)
        st = stats.cpu().tolist()
        skipped[K] = st[7]
        _log(f"c2 periodic, blocks {K}, steal {steal}: skipped {st[7]}")
        plan.close()
    assert skipped[128] > skipped[1024] > 0
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "oracle_digests.json")
    g = json.load(open(gold))["c2"][0]
    img = plain.cpu()
    assert int(img.sum(dtype=torch.int64)) == g["sum"]
    assert hashlib.sha256(np.ascontiguousarray(img.numpy(), dtype="<i4").tobytes()
                          ).hexdigest() == g["sha256"]
