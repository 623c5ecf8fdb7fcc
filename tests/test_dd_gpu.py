"""GPU parity of the double-double deep-zoom render (mandel_render_dd) against
the double-double CPU oracle (oracle/mandel_dd_oracle.c), element by element and
bit for bit: views at ordinary scale, deep zooms whose pixel pitch is far below
binary64 resolution (down to 1e-22), ragged and degenerate sizes, tiny and large
max_iter, several radii, and a 2048 x 2048 view 1e-13 wide at a seeded boundary
point, max_iter 50000, on sampled pixels."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import dd as dd_oracle
from paper_2007_00745_amd import native, workloads

pytestmark = pytest.mark.gpu

SEAHORSE = (-0.7436438870371587, -3.2e-17, 0.1318259042053119, 1.1e-17)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _win(centre, dx, dy=None):
    return tuple(centre) + (dx, dy if dy is not None else dx)


def _gpu(win, m, n, mi, R=2.0, stats=None):
    _log(f"dd {m}x{n} it={mi} R={R} win={win}")
    out = native.render_dd(win, m, n, mi, R, stats=stats)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_ordinary_scale_and_fp64_agreement():
    # the 640 x 480 window at 160 x 120: exact against the double-double oracle;
    # and with no rounding-sensitive pixels it agrees with binary64 almost everywhere
    win = (-0.5, 0.0, 0.0, 0.0, 3.0 / 160, 2.4 / 120)
    got = _gpu(win, 120, 160, 1000)
    assert np.array_equal(got, dd_oracle.render(win, 120, 160, 1000, 2.0))
    f64 = oracle.render((-0.5, 0.0, 3.0 / 160, 2.4 / 120), 120, 160, 1000, 2.0)
    assert np.mean(got == f64) > 0.99


@pytest.mark.parametrize("dx", [1e-15, 1e-17, 3e-19, 1e-22])
def test_deep_zoom_views(dx):
    win = _win(SEAHORSE, dx)
    m, n, mi = 40, 72, 3000
    got = _gpu(win, m, n, mi)
    assert np.array_equal(got, dd_oracle.render(win, m, n, mi, 2.0))


def test_deep_zoom_resolves_what_binary64_cannot():
    # dx = 1e-17: binary64 pixel centres collapse into blocks of equal counts, the
    # double-double ones do not
    win = _win(SEAHORSE, 1e-17)
    m, n, mi = 4, 128, 20000
    got = _gpu(win, m, n, mi)
    f64 = native.render((SEAHORSE[0], SEAHORSE[2], 1e-17, 1e-17), m, n, mi, 2.0)
    torch.cuda.synchronize()
    f64 = f64.cpu().numpy()
    runs64 = np.mean(f64[:, 1:] == f64[:, :-1])
    runsdd = np.mean(got[:, 1:] == got[:, :-1])
    _log(f"equal neighbours: binary64 {runs64:.3f}, double-double {runsdd:.3f}")
    assert np.array_equal(got, dd_oracle.render(win, m, n, mi, 2.0))
    assert runsdd < 0.5 * runs64 and len(np.unique(got)) > 4 * len(np.unique(f64))


@pytest.mark.parametrize("m,n", [(1, 1), (1, 97), (97, 1), (9, 65), (37, 53), (8, 64), (17, 129)])
def test_ragged_sizes(m, n):
    win = _win(SEAHORSE, 2e-17)
    got = _gpu(win, m, n, 1500)
    assert np.array_equal(got, dd_oracle.render(win, m, n, 1500, 2.0))


@pytest.mark.parametrize("mi", [1, 2, 3, 17])
def test_tiny_max_iter(mi):
    win = (-0.5, 0.0, 0.0, 0.0, 3.0 / 64, 2.4 / 48)
    got = _gpu(win, 48, 64, mi)
    assert np.array_equal(got, dd_oracle.render(win, 48, 64, mi, 2.0))
    if mi == 1:
        assert np.all(got == 1)


@pytest.mark.parametrize("R", [0.5, 1.999, 2.0, 400.0, 1e150])
def test_escape_radii(R):
    win = (-0.4, 0.0, 0.1, 0.0, 3.8 / 80, 3.2 / 60)
    got = _gpu(win, 60, 80, 700, R)
    assert np.array_equal(got, dd_oracle.render(win, 60, 80, 700, R))


def test_golden_orbits_and_large_max_iter():
    # 1 x 1 views at the hand-derived exact orbits, and bounded orbits at 2^22
    rows = [(1.0, 0.0, 1000, 2.0, 3), (2.0, 0.0, 1000, 2.0, 2), (0.0, 2.0, 1000, 2.0, 2),
            (0.5, 0.0, 1000, 2.0, 5), (-1.0, 1.0, 1000, 2.0, 3), (-2.5, 0.0, 1000, 2.0, 1),
            (-2.0, 0.0, 1000, 2.0, 1000), (0.0, 1.0, 1000, 2.0, 1000),
            (0.0, 0.0, 1 << 22, 2.0, 1 << 22), (-1.0, 0.0, 1 << 22, 2.0, 1 << 22)]
    for re_, im_, mi, R, exp in rows:
        got = _gpu((re_, 0.0, im_, 0.0, 1e-3, 1e-3), 1, 1, mi, R)
        assert int(got[0, 0]) == exp, (re_, im_)


def test_empty_views():
    for m, n in ((0, 5), (5, 0), (0, 0)):
        out = native.render_dd(_win(SEAHORSE, 1e-17), m, n, 100, 2.0)
        torch.cuda.synchronize()
        assert out.shape == (m, n)


def test_stats_and_streams():
    win = _win(SEAHORSE, 5e-17)
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = native.render_dd(win, 33, 70, 2500, 2.0, stats=stats, stream=s)
    s.synchronize()
    want = dd_oracle.render(win, 33, 70, 2500, 2.0)
    assert np.array_equal(out.cpu().numpy(), want)
    st = stats.cpu().tolist()
    assert st[1] == int(want.sum()) and st[3] == 2 * 5


def test_deep_view_2048_sampled():
    # 2048 x 2048, 1e-13 wide, at the stress batch's seeded boundary point,
    # max_iter 50000 (pitch 4.9e-17): sampled pixels against the oracle
    deep = workloads.c5()[0]
    dx = 1e-13 / 2048
    win = (deep.window[0], 0.0, deep.window[1], 0.0, dx, dx)
    m = n = 2048
    out = native.render_dd(win, m, n, 50000, 2.0)
    torch.cuda.synchronize()
    img = out.view(-1)
    rng = np.random.default_rng(2048)
    idx = rng.integers(0, m * n, 600)
    got = img[torch.tensor(idx, device="cuda")].cpu().numpy()
    want = dd_oracle.render_pixels(win, m, n, 50000, 2.0, idx, threads=16)
    assert np.array_equal(got, want)
    assert int(img.min()) >= 1 and int(img.max()) <= 50000


def test_deep_zoom_bench_view_whole_image():
    # The deep-zoom view the benchmark times (4096 x 4096 at pitch 1e-17, max_iter 20000):
    # every pixel against the double-double oracle's whole image, through its stored
    # digest (tests/golden/make_oracle_digests.py).
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "oracle_digests.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    if "dd_deep" not in table:
        pytest.skip("double-double digest not generated")
    g = table["dd_deep"][0]
    win = tuple(float.fromhex(x) for x in g["window"])
    got = _gpu(win, g["m"], g["n"], g["max_iter"], g["R"])
    assert int(got.sum(dtype=np.int64)) == g["sum"]
    assert hashlib.sha256(np.ascontiguousarray(got, dtype="<i4").tobytes()).hexdigest() == g["sha256"]
