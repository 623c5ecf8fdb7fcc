"""Randomised parity over the configuration space (seeded, so every run checks the
same cases): each case draws a small batch of views (full window, boundary zooms
down to pitch 1e-9, random regions, the all-escaping outside; ragged and empty
sizes; max_iter 1..3000; R from 1.5 to 400), a random plan tuning (tile shape,
claim grain, wavefronts per group, deferred block length, young updates, refill
lanes, row parts, group count, collapsed rows, the latter with a zoom whose row
pitch lies below the spacing of doubles) and two random launches of the same plan
(FCFS, ordered over a random permutation, probe, learned with random weights, the
paper's static and alternating rows over the concatenated rows; periodicity
detection, row stealing, eager or from the graph).  Every image must equal the
oracle's bit for bit (Sec. I, Eq. (1)-(2): the schedule never changes a count),
the statistics' count sum must equal the oracle's over the rendered rows, and in the
queue modes so must the per-tile cost log's total."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as mlp_ref
from paper_2007_00745_amd import native, workloads

pytestmark = pytest.mark.gpu

# points on or near the boundary of the set (seahorse and elephant valleys, the
# period-3 bulb's neck, an antenna point, the cardioid's cusp)
NEAR_BOUNDARY = [(-0.7436438870371587, 0.1318259042053119), (0.2850, 0.0110),
                 (-0.1592, 1.0317), (-1.7490, 0.0), (0.25, 0.0), (-0.75, 0.1)]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _view(rng):
    m = int(rng.choice([0, 1, 3]) if rng.random() < 0.08 else rng.integers(1, 150))
    n = int(rng.choice([0, 1, 5]) if rng.random() < 0.08 else rng.integers(1, 200))
    kind = int(rng.integers(0, 4))
    if kind == 0 and m > 0 and n > 0:
        win = workloads.window_from_bounds(-2.0, 1.0, -1.2, 1.2, m, n)
    elif kind == 1:
        cx, cy = NEAR_BOUNDARY[int(rng.integers(0, len(NEAR_BOUNDARY)))]
        d = 10.0 ** rng.uniform(-9, -3)
        win = (cx, cy, d, d * rng.uniform(0.5, 2.0))
    elif kind == 2:
        d = 10.0 ** rng.uniform(-4, -1.5)
        win = (rng.uniform(-2.2, 0.8), rng.uniform(-1.3, 1.3), d, d)
    else:
        d = 10.0 ** rng.uniform(-3, -1)
        win = (rng.choice([-2.6, 2.3]), rng.uniform(-1.0, 1.0), d, d)
    max_iter = int(np.exp(rng.uniform(0.0, np.log(3000.0))))
    R = float(rng.choice([2.0, 2.0, 2.0, 1.5, 4.0, 400.0]))
    return workloads.View(tuple(float(x) for x in win), m, n, max_iter, R)


def _tuning(rng):
    return dict(tile_w=int(rng.choice([8, 16, 32, 64, 128])),
                tile_h=int(rng.choice([1, 2, 4, 8, 16])),
                grain=int(rng.choice([1, 1, 2, 3, 8])),
                waves_per_group=int(rng.choice([1, 2, 4, 8])),
                block_iters=int(rng.choice([1, 8, 64, 1024])),
                young_iters=int(rng.choice([1, 4, 16])),
                refill_lanes=int(rng.choice([1, 8, 16, 64])),
                tile_parts=int(rng.choice([1, 1, 2, 4])),
                groups=int(rng.choice([0, 0, 37, 300])))


def _rendered_total(views, want, collapse):
    # the count sum over the rows a plan renders: with collapsed rows, only the first
    # row of each imaginary part (of each absolute value with collapse 2), formed as the
    # kernels form it; the other rows are copies
    total = 0
    for v, w in zip(views, want):
        if collapse == 0 or v.m < 2 or v.n == 0:
            total += int(w.sum(dtype=np.int64))
            continue
        i = np.arange(v.m, dtype=np.float64)
        cy = v.window[1] + ((i + 0.5) - v.m / 2.0) * v.window[3]
        key = np.abs(cy) if collapse == 2 else cy + 0.0
        _, first = np.unique(key, return_index=True)
        total += int(w[first].sum(dtype=np.int64))
    return total


def _launch_kw(rng, plan, params):
    mode = str(rng.choice(["fcfs", "ordered", "probe", "learned", "static", "alternating"]))
    kw = dict(mode=mode, use_graph=bool(rng.random() < 0.5),
              periodicity=int(rng.random() < 0.3))
    if mode == "ordered":
        kw["order"] = torch.tensor(rng.permutation(plan.ntiles), dtype=torch.int32,
                                   device="cuda")
    elif mode == "learned":
        kw["mlp"] = params
    elif mode in ("static", "alternating"):
        kw["workers"] = int(rng.choice([1, 7, 64, 500]))
    if mode not in ("static", "alternating") and plan.tuning["tile_parts"] == 1:
        kw["steal"] = int(rng.random() < 0.3)
    return kw


# 286: a plan with no tiles launched in ORDERED mode with an empty order (NULL pointer)
@pytest.mark.parametrize("seed", list(range(160)) + [286])
def test_random_batch_and_schedule(seed):
    rng = np.random.default_rng(9000 + seed)
    views = [_view(rng) for _ in range(int(rng.integers(1, 5)))]
    # collapsed rows from a generator of their own, so the other draws stay as they were;
    # with them, one more view whose row pitch is 0.05-1.5 times the spacing of doubles
    # near its imaginary part, so that some or most of its rows share a coordinate
    crng = np.random.default_rng(31000 + seed)
    collapse = int(crng.choice([0, 0, 1, 2]))
    if collapse:
        cx, cy = NEAR_BOUNDARY[int(crng.choice([0, 1, 2, 5]))]
        dy = float(np.spacing(cy)) * crng.uniform(0.05, 1.5)
        views.append(workloads.View((cx, cy, 10.0 ** crng.uniform(-9, -6), dy),
                                    int(crng.integers(2, 120)), int(crng.integers(1, 90)),
                                    int(np.exp(crng.uniform(0.0, np.log(3000.0)))), 2.0))
    want = [oracle.render(v.window, v.m, v.n, v.max_iter, v.R) for v in views]
    total = sum(int(w.sum(dtype=np.int64)) for w in want)
    tun = _tuning(rng)
    tun["collapse_rows"] = collapse
    rendered = _rendered_total(views, want, collapse)
    plan = native.Plan(views, tun)
    p = mlp_ref.init_params(rng, mu=rng.normal(size=68) * 0.1, sd=rng.uniform(0.5, 2.0, 68))
    params = torch.tensor(p, dtype=torch.float32, device="cuda")
    out = torch.empty((max(plan.out_size(), 1),), dtype=torch.int32, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    cost = torch.empty((max(plan.ntiles, 1),), dtype=torch.int64, device="cuda")
    for rep in range(2):
        kw = _launch_kw(rng, plan, params)
        rows = kw["mode"] in ("static", "alternating")
        desc = {k: v for k, v in kw.items() if k not in ("order", "mlp")}
        _log(f"seed {seed} rep {rep}: {len(views)} views "
             f"{[(v.m, v.n, v.max_iter, v.R) for v in views]} tuning {tun} launch {desc}")
        out.fill_(-1)
        stats.zero_()
        if not rows:
            kw["tile_cost"] = cost
        torch.cuda.synchronize()
        plan.launch(out, stats=stats, **kw)
        torch.cuda.synchronize()
        imgs = plan.view_images(out.cpu())
        for k, (g, w) in enumerate(zip(imgs, want)):
            assert np.array_equal(g.numpy(), w), f"seed {seed} rep {rep} view {k}"
        if plan.ntiles > 0:
            assert int(stats.cpu()[1]) == rendered
            if not rows:
                assert int(cost[:plan.ntiles].sum().item()) == rendered
    plan.close()


@pytest.mark.parametrize("seed", range(120))
def test_random_single_view_schedule(seed):
    # mandel_render_sched with a random schedule of every policy (the queue, a random
    # permutation, the paper's static and alternating rows, the grid launch), random
    # test mode, block length, young updates, refill lanes, row parts and claim grain:
    # the image equals the oracle's; the claim log says every tile part was claimed
    # once (tile policies) or every row was taken by the worker the paper assigns
    # (Sec. III-A, III-C); the statistics' count sum equals the oracle's.
    from oracle import partition
    rng = np.random.default_rng(12000 + seed)
    v = _view(rng)
    want = oracle.render(v.window, v.m, v.n, v.max_iter, v.R)
    policy = str(rng.choice(["fcfs", "ordered", "static", "alternating", "grid"]))
    tw = int(rng.choice([8, 16, 32, 64, 128]))
    th = int(rng.choice([1, 2, 4, 8, 16]))
    check_every = int(rng.random() < 0.3)
    kw = dict(policy=policy, tile_w=tw, tile_h=th, check_every=check_every,
              periodicity=int(check_every == 0 and rng.random() < 0.3),
              waves_per_group=int(rng.choice([1, 2, 4, 8])),
              block_iters=int(rng.choice([1, 8, 64, 1024])),
              young_iters=int(rng.choice([1, 4, 16])),
              refill_lanes=int(rng.choice([1, 8, 16, 64])))
    rows = policy in ("static", "alternating")
    nt = native.tile_count(v.m, v.n, tw, th)
    parts = 1
    auto = False
    if policy in ("fcfs", "ordered"):
        parts = int(rng.choice([1, 1, 2, 4]))
        kw.update(tile_parts=parts, grain=int(rng.choice([1, 2, 3, 8])))
        # automatic row parts from a generator of their own (the other draws unchanged)
        auto = bool(np.random.default_rng(33000 + seed).random() < 0.3)
        if auto:
            kw["tile_parts"] = native.TILE_PARTS_AUTO
    if policy == "ordered":
        kw["order"] = torch.tensor(rng.permutation(max(nt, 1)), dtype=torch.int32, device="cuda")
    W = 0
    if rows:
        W = int(rng.choice([1, 3, 64, 1000]))
        kw["workers"] = W
    elif policy != "grid" and rng.random() < 0.3:
        kw["workers"] = int(rng.choice([1, 37, 300]))
    nlog = v.m if rows else nt
    claims = torch.full((max(nlog, 1),), 99, dtype=torch.int32, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    desc = {k: x for k, x in kw.items() if k != "order"}
    _log(f"seed {seed}: view {(v.m, v.n, v.max_iter, v.R)} window {v.window} sched {desc}")
    got = native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, claims=claims, stats=stats,
                              **kw)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want), f"seed {seed}"
    if v.m == 0 or v.n == 0:
        return
    assert int(stats.cpu()[1]) == int(want.sum(dtype=np.int64))
    log = claims.cpu().numpy()[:nlog]
    if rows:
        fn = partition.naive_rows if policy == "static" else partition.alternating_rows
        owner = np.zeros(v.m, dtype=np.int64)
        for r in range(W):
            owner[fn(v.m, W, r)] = r + 1
        assert np.array_equal(log, owner)
    else:
        hs = np.minimum(th, v.m - np.arange(0, v.m, th))

        def per_tile(parts):
            per = np.array([sum(1 for p in range(parts) if ((p + 1) * h) // parts > (p * h) // parts)
                            for h in hs])
            return np.repeat(per[:, None], -(-v.n // tw), axis=1)

        got_log = log.reshape(len(hs), -1)
        if auto:
            # one part count for the launch: a power of two up to 8, or tile_h if smaller
            cands = sorted({min(p, th) for p in (1, 2, 4, 8)})
            assert any(np.array_equal(got_log, per_tile(p)) for p in cands), f"seed {seed}"
        else:
            assert np.array_equal(got_log, per_tile(parts))


@pytest.mark.parametrize("seed", range(24))
def test_random_double_double(seed):
    # mandel_render_dd on random deep windows (pitch 1e-19 .. 1e-12 at points near the
    # boundary, centre low parts drawn at the scale of an ulp of the high parts,
    # ragged sizes, max_iter up to 2000) equals the double-double oracle bit for bit.
    import oracle.dd as dd
    rng = np.random.default_rng(15000 + seed)
    cx, cy = NEAR_BOUNDARY[int(rng.integers(0, len(NEAR_BOUNDARY)))]
    d = 10.0 ** rng.uniform(-19, -12)
    win = (cx, float(rng.uniform(-1, 1) * 1e-17 * max(abs(cx), 1e-3)),
           cy, float(rng.uniform(-1, 1) * 1e-17 * max(abs(cy), 1e-3)), d, d * rng.uniform(0.5, 2))
    m, n = int(rng.integers(1, 40)), int(rng.integers(1, 70))
    max_iter = int(np.exp(rng.uniform(0.0, np.log(2000.0))))
    R = float(rng.choice([2.0, 2.0, 4.0]))
    _log(f"seed {seed}: dd window {win} size {m}x{n} max_iter {max_iter} R {R}")
    want = dd.render(win, m, n, max_iter, R)
    got = native.render_dd(win, m, n, max_iter, R)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want), f"seed {seed}"
