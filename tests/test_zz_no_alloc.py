"""GPU test of mandel_render_sched_noalloc, the entry point for callers that cannot
allocate: its images must equal mandel_render_sched's (and the CPU oracle's, Sec. I,
Eq. (1)-(2)) bit for bit, over two calls in a row on the same static scratch, the
second with a smaller image, in the queue policies that use the scratch head and
with a nonzero first slot."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2007_00745_amd import native, workloads

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


CASES = [
    # (view, schedule)
    (workloads.View(workloads.window_from_bounds(-2.0, 1.0, -1.2, 1.2, 300, 517), 300, 517,
                    800), {}),
    (workloads.View((-0.7436438870371587, 0.1318259042053119, 2e-7, 2e-7), 133, 201, 3000),
     dict(tile_w=32, tile_h=4, grain=2, tile_parts=2)),
]


@pytest.mark.parametrize("sched", [{}, dict(policy="ordered"), dict(check_every=1),
                                   dict(periodicity=1, block_iters=128),
                                   dict(tile_parts=native.TILE_PARTS_AUTO)])
def test_noalloc_matches_render_sched_twice(sched):
    # call 1: the larger image; call 2: a smaller one right after, on the same stream,
    # so the second call starts from the first one's leftover head
    for k, (v, extra) in enumerate(CASES):
        kw = dict(extra, **sched)
        if kw.get("policy") == "ordered":
            nt = native.tile_count(v.m, v.n, kw.get("tile_w", 64), kw.get("tile_h", 8))
            kw["order"] = torch.randperm(nt, device="cuda").to(torch.int32)
        _log(f"noalloc call {k + 1}: {v.m}x{v.n} max_iter {v.max_iter} {sched}")
        ref = torch.full((v.m, v.n), -1, dtype=torch.int32, device="cuda")
        got = torch.full((v.m, v.n), -2, dtype=torch.int32, device="cuda")
        native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, out=ref, **kw)
        native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, out=got, noalloc=True, **kw)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"call {k + 1}"
        want = oracle.render(v.window, v.m, v.n, v.max_iter, v.R)
        assert np.array_equal(got.cpu().numpy(), want), f"call {k + 1}"


def test_noalloc_logs_and_first_slot():
    # per-tile cost logs and a queue resumed at a later slot behave as in
    # mandel_render_sched: slots before first_slot are left untouched
    v = CASES[0][0]
    nt = native.tile_count(v.m, v.n)
    for first in (0, nt // 3):
        outs, costs = [], []
        for noalloc in (False, True):
            out = torch.full((v.m, v.n), -7, dtype=torch.int32, device="cuda")
            cost = torch.full((nt,), -1, dtype=torch.int64, device="cuda")
            native.render_sched(v.window, v.m, v.n, v.max_iter, v.R, out=out, tile_cost=cost,
                                first_slot=first, noalloc=noalloc)
            outs.append(out)
            costs.append(cost)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1]) and torch.equal(costs[0], costs[1])
        assert int((outs[1] == -7).sum().item()) == (0 if first == 0 else
                                                     int((outs[0] == -7).sum().item()))


def test_noalloc_argument_errors():
    # invalid arguments are refused as by mandel_render_sched, with nothing launched
    out = torch.full((4, 4), -1, dtype=torch.int32, device="cuda")
    for kw in (dict(max_iter=0), dict(R=-1.0), dict(R=float("nan"))):
        args = dict(window=(0.0, 0.0, 0.1, 0.1), m=4, n=4, max_iter=10, R=2.0)
        args.update(kw)
        with pytest.raises(native.MandelError):
            native.render_sched(out=out, noalloc=True, **args)
    with pytest.raises(native.MandelError):
        native.render_sched((0.0, 0.0, 0.1, 0.1), 4, 4, 10, 2.0, out=out, noalloc=True,
                            policy="ordered")   # ORDERED without an order array
    torch.cuda.synchronize()
    assert int(out.max().item()) == -1
    # an empty image is a no-op
    native.render_sched((0.0, 0.0, 0.1, 0.1), 0, 5, 10, 2.0,
                        out=torch.empty((0, 5), dtype=torch.int32, device="cuda"), noalloc=True)
