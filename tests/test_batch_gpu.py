"""GPU tests of batch plans, graph replay, probe features, the FP32 cost model
(inference and one training step) and the descending tile order.

Counts are compared with the CPU oracle bit for bit (paper Sec. I, Eq. (1)-(2));
the cost model is compared with the FP64 reference in oracle/mlp.py within
FP32 tolerances (rtol 1e-3 / atol 1e-5 of the gradient scale)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as mlp_ref
from oracle import order as order_ref
from paper_2007_00745_amd import native, workloads

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def small_batch():
    views = workloads.c3_scaled(745, 64, scale=32)
    views += [workloads.View((-0.5, 0.0, 0.01, 0.01), 0, 17, 100),   # empty view
              workloads.View((0.3, 0.1, 0.1, 0.1), 1, 1, 50),
              workloads.View(workloads.window_from_bounds(-2, 1, -1.2, 1.2, 33, 70), 33, 70, 300)]
    want = [oracle.render(v.window, v.m, v.n, v.max_iter, v.R) for v in views]
    return views, want


def _check(plan, out, want):
    imgs = plan.view_images(out.cpu())
    for k, (g, w) in enumerate(zip(imgs, want)):
        assert np.array_equal(g.numpy(), w), f"view {k}"


def _params(seed, feat=None, biases=True):
    # He-uniform weights; with biases=True every bias is drawn non-zero as well, so
    # that the kernels' bias reads are compared with the reference too
    rng = np.random.default_rng(seed)
    if feat is not None:
        f = feat.cpu().double().numpy()
        p = mlp_ref.init_params(rng, mu=f.mean(0), sd=f.std(0) + 1e-3)
    else:
        p = mlp_ref.init_params(rng, mu=rng.normal(size=68) * 0.1, sd=rng.uniform(0.5, 2, 68))
    if biases:
        d = mlp_ref.unpack(p)
        d["b1"] = rng.normal(size=64) * 0.5
        d["b2"] = rng.normal(size=64) * 0.5
        d["b3"] = rng.normal(size=1) + 3.0
        p = mlp_ref.pack(d)
    return p


@pytest.mark.parametrize("tuning", [{}, dict(tile_w=32, tile_h=4, grain=3),
                                    dict(tile_w=16, tile_h=16, waves_per_group=1, groups=37),
                                    dict(tile_parts=4, grain=2), dict(tile_h=5, tile_parts=8)])
def test_plan_fcfs(small_batch, tuning):
    views, want = small_batch
    plan = native.Plan(views, tuning)
    _log(f"plan {plan.ntiles} tiles {tuning}")
    out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
    plan.launch(out)
    torch.cuda.synchronize()
    _check(plan, out, want)
    plan.close()


@pytest.mark.parametrize("parts", [1, 4])
def test_plan_modes_and_graph_replays(small_batch, parts):
    views, want = small_batch
    plan = native.Plan(views, dict(tile_parts=parts))
    nt = plan.ntiles
    feat = plan.features()
    params = torch.tensor(_params(3, feat), dtype=torch.float32, device="cuda")
    order = torch.tensor(np.random.default_rng(5).permutation(nt), dtype=torch.int32,
                         device="cuda")
    for mode in ("fcfs", "ordered", "probe", "learned"):
        kw = dict(order=order) if mode == "ordered" else {}
        if mode == "learned":
            kw["mlp"] = params
        out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
        _log(f"mode {mode} eager")
        plan.launch(out, mode=mode, **kw)
        torch.cuda.synchronize()
        eager = out.clone()
        _check(plan, eager, want)
        gout = torch.full_like(out, -7)
        for rep in range(3):
            _log(f"mode {mode} graph replay {rep}")
            gout.fill_(-7)                      # eager work between replays
            torch.cuda.synchronize()
            plan.launch(gout, mode=mode, use_graph=True, **kw)
            torch.cuda.synchronize()
            assert torch.equal(gout, eager), (mode, rep)
    plan.close()


@pytest.mark.parametrize("mode", ["static", "alternating"])
def test_plan_row_modes(small_batch, mode):
    # The paper's row partitions over the concatenated rows of the whole batch
    # (Sec. III-A and III-C): every worker count gives the oracle's images, also
    # with fewer rows than workers, a view of zero-width rows and graph replays.
    views, want = small_batch
    views = views + [workloads.View((0.1, 0.2, 0.01, 0.01), 5, 0, 40)]
    want = want + [np.zeros((5, 0), dtype=np.int32)]
    nrows = sum(v.m for v in views)
    plan = native.Plan(views)
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    for W in (1, 3, 7, 64, 1000, nrows, nrows + 5):
        for use_graph in (False, True, True):
            _log(f"rows {mode} W={W} graph={use_graph}")
            out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
            stats.zero_()
            plan.launch(out, mode=mode, workers=W, stats=stats, use_graph=use_graph)
            torch.cuda.synchronize()
            _check(plan, out, want)
            st = stats.cpu().numpy()
            assert st[3] == nrows and st[1] == sum(int(w.sum()) for w in want)
            assert st[4] <= st[6] and st[5] <= st[6]
    for bad in (dict(workers=0), dict(workers=-2), dict(workers=4, first_slot=1),
                dict(workers=4, tile_cost=torch.zeros(plan.ntiles, dtype=torch.int64,
                                                      device="cuda"))):
        with pytest.raises(native.MandelError):
            plan.launch(out, mode=mode, **bad)
    with pytest.raises(native.MandelError):
        plan.launch(out, mode="fcfs", workers=4)
    plan.close()


def _tile_sums(views, imgs, tw, th):
    sums = []
    for v, img in zip(views, imgs):
        if v.m == 0 or v.n == 0:
            continue
        ty, tx = -(-v.m // th), -(-v.n // tw)
        pad = np.zeros((ty * th, tx * tw), dtype=np.int64)
        pad[:v.m, :v.n] = img
        sums.append(pad.reshape(ty, th, tx, tw).sum(axis=(1, 3)).ravel())
    return np.concatenate(sums)


def test_plan_tile_cost_and_stats(small_batch):
    views, want = small_batch
    plan = native.Plan(views, dict(tile_w=32, tile_h=8))
    cost = torch.full((plan.ntiles,), -5, dtype=torch.int64, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    out = torch.empty((plan.out_size(),), dtype=torch.int32, device="cuda")
    for use_graph in (False, True, True):
        cost.fill_(-5)
        stats.zero_()
        plan.launch(out, tile_cost=cost, stats=stats, use_graph=use_graph)
        torch.cuda.synchronize()
        assert np.array_equal(cost.cpu().numpy(), _tile_sums(views, want, 32, 8))
        st = stats.cpu().numpy()
        assert st[1] == sum(int(w.sum()) for w in want) and st[3] == plan.ntiles
    plan.close()


def test_plan_tile_timestamps(small_batch):
    # learned mode with graph replays: every tile stamped, claim before finish
    views, want = small_batch
    plan = native.Plan(views)
    tt = torch.zeros(2 * plan.ntiles, dtype=torch.int64, device="cuda")
    params = torch.tensor(_params(3, plan.features()), dtype=torch.float32, device="cuda")
    out = torch.empty((plan.out_size(),), dtype=torch.int32, device="cuda")
    for use_graph in (False, True, True):
        tt.fill_(3)
        plan.launch(out, mode="learned", mlp=params, tile_time=tt, use_graph=use_graph)
        torch.cuda.synchronize()
        _check(plan, out, want)
        t = tt.cpu().numpy().view(np.uint64).reshape(plan.ntiles, 2)
        assert (t[:, 0] <= t[:, 1]).all() and (t[:, 1] > 3).all()
    with pytest.raises(native.MandelError):
        plan.launch(out, mode="static", workers=4, tile_time=tt)
    plan.close()


@pytest.mark.parametrize("tuning", [{}, dict(tile_w=32, tile_h=5, grain=3),
                                    dict(tile_w=16, tile_h=16, waves_per_group=1, groups=37)])
def test_plan_row_stealing(small_batch, tuning):
    # Row stealing hands out the rows of claimed tiles through per-tile counters and
    # lets waves take rows of tiles others hold once the queue is dry.  The small batch
    # has far fewer tiles than the grid has waves, so most waves steal.  Every mode,
    # with periodicity detection, eager and graph replays: images equal the oracle's,
    # per-tile cost sums, statistics and timestamps are those of the plain queue.
    views, want = small_batch
    plan = native.Plan(views, tuning)
    nt = plan.ntiles
    tw, th = plan.tuning["tile_w"], plan.tuning["tile_h"]
    sums = _tile_sums(views, want, tw, th)
    feat = plan.features()
    params = torch.tensor(_params(3, feat), dtype=torch.float32, device="cuda")
    order = torch.tensor(np.random.default_rng(9).permutation(nt), dtype=torch.int32,
                         device="cuda")
    cost = torch.zeros(nt, dtype=torch.int64, device="cuda")
    tt = torch.zeros(2 * nt, dtype=torch.int64, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    out = torch.empty((plan.out_size(),), dtype=torch.int32, device="cuda")
    total = sum(int(w.sum()) for w in want)
    for mode in ("fcfs", "ordered", "probe", "learned"):
        kw = dict(order=order) if mode == "ordered" else {}
        if mode == "learned":
            kw["mlp"] = params
        for per in (0, 1):
            for use_graph in (False, True, True):
                _log(f"steal {tuning} mode {mode} periodicity {per} graph {use_graph}")
                out.fill_(-1)
                cost.fill_(-5)
                tt.fill_(3)
                stats.zero_()
                torch.cuda.synchronize()
                plan.launch(out, mode=mode, steal=1, periodicity=per, tile_cost=cost,
                            tile_time=tt, stats=stats, use_graph=use_graph, **kw)
                torch.cuda.synchronize()
                _check(plan, out, want)
                assert np.array_equal(cost.cpu().numpy(), sums)
                st = stats.cpu().numpy()
                assert st[1] == total and st[3] == nt
                t = tt.cpu().numpy().view(np.uint64).reshape(nt, 2)
                assert (t[:, 0] <= t[:, 1]).all() and (t[:, 1] > 3).all()
    # a queue that starts at slot k: tiles before it are neither rendered nor stolen
    for k in (1, nt // 2, nt - 1, nt, nt + 3):
        _log(f"steal {tuning} first_slot {k}")
        out.fill_(-1)
        cost.fill_(-5)
        stats.zero_()
        plan.launch(out, steal=1, first_slot=k, tile_cost=cost, stats=stats)
        torch.cuda.synchronize()
        c = cost.cpu().numpy()
        assert (c[:k] == 0).all() and np.array_equal(c[k:], sums[k:])
        o = out.cpu().numpy()
        assert int(o[o >= 0].sum()) == int(sums[k:].sum())
        assert stats.cpu().numpy()[3] == max(nt - k, 0)
    plan.close()


def test_plan_row_stealing_rejections(small_batch):
    views, _ = small_batch
    plan = native.Plan(views)
    out = torch.empty((plan.out_size(),), dtype=torch.int32, device="cuda")
    for bad in (dict(steal=2), dict(steal=-1), dict(steal=1, mode="static", workers=4),
                dict(steal=1, mode="alternating", workers=4)):
        with pytest.raises(native.MandelError):
            plan.launch(out, **bad)
    la = native.LaunchC(0, 0, None, None, None, None, 0, 0, 0, 0, 0, None, 0, 1)
    assert native.lib().mandel_plan_launch(plan._h, native._ptr(out), ctypes.byref(la),
                                           None) == native.EINVAL
    plan.close()
    parts = native.Plan(views, dict(tile_parts=4))
    with pytest.raises(native.MandelError):
        parts.launch(out, steal=1)
    parts.close()


def test_single_view_plan_equals_render():
    v = workloads.c1()
    plan = native.Plan([v])
    out = torch.empty(v.m * v.n, dtype=torch.int32, device="cuda")
    plan.launch(out, use_graph=True)
    ref = native.render(v.window, v.m, v.n, v.max_iter, v.R)
    torch.cuda.synchronize()
    assert torch.equal(out.view(v.m, v.n), ref)
    plan.close()


def test_plan_rejects_bad_views():
    bad = [workloads.View((0.0, 0.0, 0.0, 0.01), 4, 4, 10)]
    with pytest.raises(native.MandelError):
        native.Plan(bad)
    with pytest.raises(native.MandelError):
        native.Plan([workloads.View((0.0, 0.0, 0.01, 0.01), 4, 4, 0)])


def test_features_probe_counts(small_batch):
    views, _ = small_batch
    tw, th = 64, 8
    plan = native.Plan(views, dict(tile_w=tw, tile_h=th))
    # caps: the default (128), absolute ones, and shares of each view's max_iter
    # (probe_cap = -k: cap = max(1, max_iter // k)), down to a cap of 1
    for cap_arg in (0, 7, 300, -1, -16, -(1 << 20)):
        feat = plan.features(probe_cap=cap_arg).cpu().double().numpy()
        cap_req = 128 if cap_arg == 0 else cap_arg
        t = 0
        for v in views:
            if v.m == 0 or v.n == 0:
                continue
            cap = min(v.max_iter, cap_req) if cap_req > 0 else max(1, v.max_iter // -cap_req)
            ty, tx = -(-v.m // th), -(-v.n // tw)
            for a in range(ty):
                for b in range(tx):
                    x0, y0 = b * tw, a * th
                    w, h = min(tw, v.n - x0), min(th, v.m - y0)
                    cols = [x0 + ((2 * k + 1) * w) // 16 for k in range(8)]
                    rows = [y0 + ((2 * r + 1) * h) // 16 for r in range(8)]
                    idx = np.array([[i * v.n + j for j in cols] for i in rows]).ravel()
                    ref = np.minimum(oracle.render_pixels(v.window, v.m, v.n, v.max_iter, v.R,
                                                          idx), cap)
                    got = np.rint(np.exp(feat[t, 4:] * np.log1p(cap)) - 1)
                    assert np.array_equal(got.astype(np.int64), ref), (t, cap)
                    cxw = v.window[0] + ((x0 + w / 2) - v.n / 2) * v.window[2]
                    cyw = v.window[1] + ((y0 + h / 2) - v.m / 2) * v.window[3]
                    assert np.isclose(feat[t, 0], cxw, rtol=1e-6, atol=1e-7)
                    assert np.isclose(feat[t, 1], cyw, rtol=1e-6, atol=1e-7)
                    assert np.isclose(feat[t, 2], np.log10(w * v.window[2]), atol=1e-5)
                    assert np.isclose(feat[t, 3], np.log(v.max_iter), atol=1e-5)
                    t += 1
        assert t == plan.ntiles
    plan.close()


def _forward_close(p, x):
    # the FP32 kernel against the FP64 reference, evaluated at the FP32-rounded
    # parameters and inputs the kernel sees
    p32, x32 = np.float32(p), np.float32(x)
    y_ref = mlp_ref.forward(p32.astype(np.float64), x32.astype(np.float64))
    y = native.mlp_forward(torch.tensor(p32, device="cuda"), torch.tensor(x32, device="cuda"))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    assert np.allclose(y, y_ref, rtol=1e-3, atol=1e-4 * np.abs(y_ref).max()), \
        float(np.abs(y - y_ref).max())
    return y, y_ref


@pytest.mark.parametrize("biases", [False, True])
def test_mlp_forward_matches_fp64(biases):
    rng = np.random.default_rng(11)
    p = _params(12, biases=biases)
    x = rng.normal(size=(3001, 68)) * rng.uniform(0.5, 3, 68) + rng.normal(size=68)
    y, y_ref = _forward_close(p, x)
    if biases:
        # the biases move the output: a kernel that ignored them would be far off
        y0 = mlp_ref.forward(_params(12, biases=False), x)
        assert np.abs(y_ref - y0).max() > 100 * np.abs(y - y_ref).max()


def test_mlp_forward_trained_params():
    # inference on a parameter vector trained by the GPU's own training step (every
    # weight and bias moved away from its initial value) and on real tile features
    from paper_2007_00745_amd import costmodel
    views = workloads.training_views(range(1000, 1002), per_seed=8, lo=64, hi=512)
    feat, target, _, plan = costmodel.collect(views)
    params, losses = costmodel.train(feat, target, epochs=3, batch=256, lr=1e-3, seed=1)
    _log(f"trained on {feat.shape[0]} tiles, losses {[round(x, 3) for x in losses]}")
    p = params.cpu().double().numpy()
    d = mlp_ref.unpack(p)
    assert all(np.abs(d[b]).max() > 0 for b in ("b1", "b2", "b3"))
    _forward_close(p, feat.cpu().double().numpy())
    plan.close()


def test_mlp_train_step_matches_fp64():
    rng = np.random.default_rng(21)
    n, B = 2000, 512
    x = rng.normal(size=(n, 68))
    t = np.tanh(x[:, :5].sum(1)) * 4 + 10
    p = _params(22)
    dev = dict(dtype=torch.float32, device="cuda")
    P = torch.tensor(p, **dev)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    X = torch.tensor(x, **dev)
    T = torch.tensor(t, **dev)
    loss = torch.zeros(1, **dev)
    m_ref = np.zeros_like(p)
    v_ref = np.zeros_like(p)
    for step in range(1, 4):
        idx = rng.choice(n, B, replace=False)
        I = torch.tensor(idx, dtype=torch.int32, device="cuda")
        M_before = M.cpu().double().numpy()
        # reference step from the GPU's own parameters, so errors do not accumulate
        p_in = P.cpu().double().numpy()
        native.mlp_train_step(P, M, V, step, X, T, I, 1e-3, loss=loss)
        torch.cuda.synchronize()
        L_ref, g_ref = mlp_ref.loss_and_grad(p_in, x[idx], t[idx])
        assert np.isclose(loss.item(), L_ref, rtol=1e-4)
        g_gpu = (M.cpu().double().numpy() - 0.9 * M_before) / 0.1
        scale = np.abs(g_ref).max()
        s = slice(136, None)
        assert np.allclose(g_gpu[s], g_ref[s], rtol=1e-3, atol=1e-5 * scale)
        assert np.array_equal(P.cpu().numpy()[:136], np.float32(p[:136]))
        # where the gradient is well above FP32 noise, the Adam step agrees too
        pr, mr, vr = mlp_ref.adam_step(p_in, M_before, V_before if step > 1 else np.zeros_like(p_in),
                                       g_ref, step, 1e-3)
        V_before = V.cpu().double().numpy()
        big = np.abs(g_ref) > 1e-2 * scale
        big[:136] = False
        assert np.allclose(P.cpu().double().numpy()[big], pr[big], rtol=1e-4, atol=1e-6)


def test_order_constants_match_the_reference():
    assert native.ORDER_BUCKETS == order_ref.BUCKETS
    assert np.float32(native.ORDER_KEY_LO) == order_ref.KEY_LO
    assert np.float32(native.ORDER_KEY_HI) == order_ref.KEY_HI


_EDGE_KEYS = np.array([50.0, -2.0, 50.5, -2.5, 1e30, -1e30, np.inf, -np.inf, np.nan, 0.0, -0.0,
                       24.0, np.nextafter(np.float32(50), np.float32(0)),
                       np.nextafter(np.float32(-2), np.float32(0)), 1.0 / 78.75],
                      dtype=np.float32)


@pytest.mark.parametrize("n", [0, 1, 2, 15, 1000, 131072, 2_621_440])
def test_order_desc(n):
    # the device order visits exactly the bucket sequence of the reference
    # (oracle/order.py), and is a permutation; within a bucket any order is valid
    rng = np.random.default_rng(31 + n)
    keys = rng.uniform(-3, 52, n).astype(np.float32)
    if n >= 15:
        keys[rng.choice(n, 15, replace=False)] = _EDGE_KEYS
    if n > 1000:
        keys[rng.choice(n, n // 3, replace=False)] = np.float32(7.25)   # one crowded bucket
    k = torch.tensor(keys, device="cuda")
    perm = native.order_desc(k)
    torch.cuda.synchronize()
    pm = perm.cpu().numpy().astype(np.int64)
    assert pm.shape == (n,)
    assert np.array_equal(np.sort(pm), np.arange(n))
    assert np.array_equal(order_ref.bucket(keys[pm]), order_ref.bucket_sequence(keys))
    assert order_ref.is_valid_order(keys, pm)


def test_fp64_probe_runs():
    for kind in (0, 1, 2):
        r = native.fp64_probe(kind, iters=200, blocks_per_cu=2)
        assert r["ms"] > 0 and r["flops"] > 0 and r["tflops"] < 200


def test_two_plans_on_two_streams_concurrently(small_batch):
    # Consecutive steps alternate between two plans (each with its own queue head,
    # features, order and graph) on two streams with no synchronisation between them,
    # so their launches overlap on the device: every step's image must still be the
    # oracle's, in every queue mode and with graph replays.
    views, want = small_batch
    plans = [native.Plan(views), native.Plan(views)]
    params = torch.tensor(_params(3, plans[0].features()), dtype=torch.float32, device="cuda")
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    outs = [torch.full((plans[0].out_size(),), -1, dtype=torch.int32, device="cuda")
            for _ in range(2)]
    torch.cuda.synchronize()
    for mode, kw in (("fcfs", {}), ("probe", {}), ("learned", dict(mlp=params))):
        for o in outs:
            o.fill_(-1)
        torch.cuda.synchronize()
        _log(f"two streams, mode {mode}")
        for k in range(6):
            i = k % 2
            plans[i].launch(outs[i], mode=mode, use_graph=True, stream=streams[i], **kw)
        torch.cuda.synchronize()
        for i in range(2):
            _check(plans[i], outs[i], want)
    for p in plans:
        p.close()


def test_binding_rejects_wrong_buffers(small_batch):
    # wrong element types or sizes raise in the binding; nothing is launched
    views, want = small_batch
    plan = native.Plan(views)
    nt = plan.ntiles
    out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
    bad = [dict(stats=torch.zeros(8, dtype=torch.int32, device="cuda")),
           dict(stats=torch.zeros(4, dtype=torch.int64, device="cuda")),
           dict(tile_cost=torch.zeros(nt - 1, dtype=torch.int64, device="cuda")),
           dict(tile_time=torch.zeros(nt, dtype=torch.int64, device="cuda")),
           dict(mode="ordered", order=torch.arange(nt, dtype=torch.int64, device="cuda")),
           dict(mode="learned", mlp=torch.zeros(100, dtype=torch.float32, device="cuda"))]
    for kw in bad:
        with pytest.raises(ValueError):
            plan.launch(out, **kw)
    with pytest.raises(ValueError):
        plan.launch(out[:-1])
    torch.cuda.synchronize()
    assert int(out.max().item()) == -1          # nothing ran
    v = views[0]
    with pytest.raises(ValueError):
        native.render_sched(v.window, v.m, v.n, v.max_iter, v.R,
                            claims=torch.zeros(3, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        native.order_desc(torch.zeros(10, dtype=torch.float64, device="cuda"))
    plan.close()


def _collapsing_views():
    # view 0: a boundary zoom whose row pitch (1e-17) is far below the spacing of doubles
    # near its imaginary part (about 1.1e-16), so about 11 neighbouring rows share each
    # row coordinate; view 1 likewise with ragged sizes against 64x8 tiles; view 2 an
    # ordinary zoom (nothing to collapse); view 3 empty; view 4 a single row
    # (ordinary for rows that merge by value); views 5 and 6 are centred on the real
    # axis (even and odd row counts), so their rows pair up by conjugation; view 7 has a
    # pitch just below the spacing of doubles, so only a few scattered rows repeat the
    # row before them and most rows are copied from a row of another index
    cx, cy = workloads.boundary_centre(745, 0)
    return [workloads.View((cx, cy, 2e-15, 1e-17), 157, 96, 2000),
            workloads.View((cx, cy + 3e-15, 3e-15, 2.5e-17), 61, 70, 900),
            workloads.View((-0.745, 0.113, 1e-4, 1e-4), 45, 130, 700),
            workloads.View((0.3, 0.1, 0.1, 0.1), 0, 9, 50),
            workloads.View((cx, cy, 1e-15, 1e-17), 1, 33, 400),
            workloads.View(workloads.window_from_bounds(-2.0, 1.0, -1.2, 1.2, 96, 120), 96,
                           120, 600),
            workloads.View((-0.75, 0.0, 1e-3, 1e-3), 37, 81, 1500),
            workloads.View((cx, cy, 1e-14, 0.97 * float(np.spacing(cy))), 200, 40, 800)]


def _distinct_rows(v, mirror=False):
    # the row coordinates as the kernels form them, and the first row of each value
    # (of each absolute value with mirror)
    i = np.arange(v.m, dtype=np.float64)
    cy = v.window[1] + ((i + 0.5) - v.m / 2.0) * v.window[3]
    key = np.abs(cy) if mirror else cy
    _, idx = np.unique(key, return_index=True)
    first = np.zeros(v.m, bool)
    first[idx] = True
    return cy, first


@pytest.mark.parametrize("mode", ["fcfs", "probe", "learned", "ordered", "static",
                                  "alternating"])
@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("collapse", [1, 2])
def test_collapsed_rows_match_the_oracle(mode, use_graph, collapse):
    views = _collapsing_views()
    want = [oracle.render(v.window, v.m, v.n, v.max_iter, v.R) for v in views]
    flat = native.Plan(views)
    plan = native.Plan(views, {"collapse_rows": collapse})
    assert plan.tuning["collapse_rows"] == collapse
    mirror = collapse == 2
    distinct = [int(_distinct_rows(v, mirror)[1].sum()) for v in views]
    assert distinct[0] < views[0].m // 5 and distinct[2] == views[2].m
    assert views[7].m - 10 < distinct[7] < views[7].m
    if mirror:
        assert distinct[5] == 48 and distinct[6] == 19
    assert plan.ntiles < flat.ntiles
    kw = {}
    if mode == "learned":
        kw["mlp"] = torch.tensor(_params(5), dtype=torch.float32, device="cuda")
    elif mode == "ordered":
        kw["order"] = torch.randperm(plan.ntiles, device="cuda").to(torch.int32)
    elif mode in ("static", "alternating"):
        kw["workers"] = 37
    out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
    cost = None if mode in ("static", "alternating") else torch.empty(
        plan.ntiles, dtype=torch.int64, device="cuda")
    for rep in range(3):
        out.fill_(-1)
        plan.launch(out, mode=mode, use_graph=use_graph, tile_cost=cost, **kw)
        torch.cuda.synchronize()
        _check(plan, out, want)
    if cost is not None:
        # the tile costs cover each distinct row once
        rendered = sum(int(w[_distinct_rows(v, mirror)[1]].sum()) for v, w in zip(views, want))
        assert int(cost.sum().item()) == rendered
    plan.close()
    flat.close()


def test_collapsed_rows_refuse_a_resumed_queue():
    views = _collapsing_views()
    plan = native.Plan(views, {"collapse_rows": 1})
    out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(native.MandelError):
        plan.launch(out, first_slot=1)
    torch.cuda.synchronize()
    assert int(out.max().item()) == -1
    plan.close()
    # views whose rows are all distinct are rendered as without the option
    plain = [workloads.c1()]
    p = native.Plan(plain, {"collapse_rows": 1})
    assert p.ntiles == native.Plan(plain).ntiles
    out = torch.full((p.out_size(),), -1, dtype=torch.int32, device="cuda")
    p.launch(out, first_slot=0)
    torch.cuda.synchronize()
    _check(p, out, [oracle.render(plain[0].window, 480, 640, 1000, 2.0)])
    p.close()


@pytest.mark.parametrize("mode,steal", [("fcfs", 0), ("fcfs", 1), ("ordered", 0),
                                        ("probe", 0), ("learned", 0), ("static", 0),
                                        ("alternating", 0)])
def test_plan_automatic_row_parts(mode, steal):
    # tile_parts = MANDEL_TILE_PARTS_AUTO in a plan, resolved at each launch: counts equal
    # to the oracle's in every mode, eagerly and from graph replays; in the queue modes
    # without stealing the launch's work items are the non-empty row parts of every tile
    # for one part count p (a power of two up to 8); a resumed queue is refused
    views = [workloads.View(workloads.window_from_bounds(-2.0, 1.0, -1.2, 1.2, 300, 517),
                            300, 517, 800),
             workloads.View((-0.7436438870371587, 0.1318259042053119, 2e-7, 2e-7), 133, 201,
                            3000)]
    want = [oracle.render(v.window, v.m, v.n, v.max_iter, v.R) for v in views]
    plan = native.Plan(views, {"tile_parts": native.TILE_PARTS_AUTO})
    assert plan.tuning["tile_parts"] == native.TILE_PARTS_AUTO
    kw = {}
    if mode == "learned":
        kw["mlp"] = torch.tensor(_params(3), dtype=torch.float32, device="cuda")
    elif mode == "ordered":
        kw["order"] = torch.randperm(plan.ntiles, device="cuda").to(torch.int32)
    elif mode in ("static", "alternating"):
        kw["workers"] = 29
    if steal:
        kw["steal"] = 1
    out = torch.full((plan.out_size(),), -1, dtype=torch.int32, device="cuda")
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    for use_graph in (False, True, True):
        out.fill_(-1)
        stats.zero_()
        plan.launch(out, mode=mode, use_graph=use_graph, stats=stats, **kw)
        torch.cuda.synchronize()
        _check(plan, out, want)
        st = stats.cpu().numpy()
        assert st[1] == sum(int(w.sum(dtype=np.int64)) for w in want)
        if mode in ("fcfs", "ordered", "probe", "learned") and not steal:
            def items(p):
                n = 0
                for v in views:
                    hs = np.minimum(8, v.m - np.arange(0, v.m, 8))
                    per = [sum(1 for q in range(p) if ((q + 1) * h) // p > (q * h) // p)
                           for h in hs]
                    n += sum(per) * -(-v.n // 64)
                return n
            assert st[3] in {items(p) for p in (1, 2, 4, 8)}, st[3]
    if mode in ("fcfs", "ordered"):
        with pytest.raises(native.MandelError):
            plan.launch(out, mode=mode, first_slot=1, **kw)
    plan.close()
