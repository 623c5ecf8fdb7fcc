"""The stored whole-image digests of the oracle (tests/golden/oracle_digests.json,
written by tests/golden/make_oracle_digests.py, which calls only the oracle) are
pinned here: the 640 x 480 view's digest is recomputed with the oracle, and every
stored view's size, max_iter, R and window must still be what the seeded input
generator produces, so a changed generator cannot silently compare against stale
digests.  The committed boundary centres (tests/golden/boundary_centres.json) are
re-derived for sampled views by bisection with the oracle and must match bit for bit,
and a table written for other ray angles is refused."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2007_00745_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_digests.json")


def _table():
    return json.load(open(GOLDEN))


def test_c1_digest_recomputed_by_the_oracle():
    g = _table()["c1"][0]
    v = workloads.c1()
    img = oracle.render(v.window, v.m, v.n, v.max_iter, v.R)
    assert int(img.sum(dtype=np.int64)) == g["sum"]
    assert hashlib.sha256(np.ascontiguousarray(img, dtype="<i4").tobytes()).hexdigest() == g["sha256"]


@pytest.mark.parametrize("name,views", [("c1", lambda: [workloads.c1()]),
                                        ("c2", lambda: [workloads.c2()]),
                                        ("c3", workloads.c3)])
def test_stored_views_match_the_generator(name, views):
    table = _table()
    if name not in table:
        pytest.skip(f"{name} digests not generated")
    stored = table[name]
    vs = views()
    assert len(stored) == len(vs)
    for g, v in zip(stored, vs):
        assert (g["m"], g["n"], g["max_iter"], g["R"]) == (v.m, v.n, v.max_iter, v.R)
        assert [float.fromhex(x) for x in g["window"]] == [float(x) for x in v.window]
        assert 0 < g["sum"] <= v.m * v.n * v.max_iter


def test_stored_deep_zoom_view_matches_its_definition():
    import importlib.util
    table = _table()
    if "dd_deep" not in table:
        pytest.skip("double-double digest not generated")
    spec = importlib.util.spec_from_file_location(
        "make_oracle_digests", os.path.join(os.path.dirname(GOLDEN), "make_oracle_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    d, g = mod.DD_DEEP, table["dd_deep"][0]
    assert (g["m"], g["n"], g["max_iter"], g["R"]) == (d["m"], d["n"], d["max_iter"], d["R"])
    assert [float.fromhex(x) for x in g["window"]] == list(d["window"])
    assert 0 < g["sum"] <= d["m"] * d["n"] * d["max_iter"]


def test_stored_stress_small_views_match_the_generator():
    table = _table()
    if "c5_small" not in table:
        pytest.skip("stress-batch digest not generated")
    g = table["c5_small"][0]
    small = workloads.c5()[1:]
    assert g["views"] == len(small) and g["first_view"] == 1
    assert all((v.m, v.n) == (g["m"], g["n"]) for v in small)
    assert 0 < g["sum"] <= sum(v.m * v.n * v.max_iter for v in small)


def _centre_script():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_boundary_centres",
        os.path.join(os.path.dirname(GOLDEN), "make_boundary_centres.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("seed,k", [(745, 0), (745, 37), (747, 0), (748, 4095), (1000, 5),
                                    (1015, 63)])
def test_stored_boundary_centres_are_the_oracle_bisection(seed, k):
    # the committed centre of a view is what bisection along its ray with the oracle's
    # predicate gives, bit for bit; the bisection ends on adjacent doubles of t with the
    # inside end inside and the outside end escaping
    mod = _centre_script()
    d = workloads.draw(seed, k)
    mi = workloads.ray_max_iter(seed, k)

    def count(cx, cy):
        return oracle.escape_count(cx, cy, mi, 2.0)

    t_in, t_out, steps = mod.bisect_ray(d.theta, mi, workloads.RAY_OUTSIDE_T, count)
    assert np.nextafter(t_in, np.inf) == t_out and steps > 40
    cx, cy = mod.ray_point(t_in, d.theta)
    assert count(cx, cy) == mi and count(*mod.ray_point(t_out, d.theta)) < mi
    assert workloads.boundary_centre(seed, k) == (cx, cy)


def test_boundary_centre_table_rejects_other_draws(monkeypatch):
    # a generator whose draws no longer match the table is refused, not silently used
    workloads._checked.clear()
    real = workloads.draw

    def shifted(seed, k):
        d = real(seed, k)
        return workloads.Draw(d.theta + 1e-3, d.width, d.max_iter, d.u_cols, d.u_rows)

    monkeypatch.setattr(workloads, "draw", shifted)
    with pytest.raises(ValueError):
        workloads.boundary_centre(745, 0)
    monkeypatch.setattr(workloads, "draw", real)
    workloads._checked.clear()
    assert workloads.boundary_centre(745, 0)
