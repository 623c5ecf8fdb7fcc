"""The command line (python -m paper_2007_00745_amd) end to end: each schedule and
arithmetic writes the PPM file that the oracles' counts, colouring and byte layout
give (paper Sec. I with Eq. (2), Sec. III)."""
import json

import pytest

import oracle
from oracle import dd as dd_oracle
from oracle import output as out_oracle
from paper_2007_00745_amd import __main__ as cli
from paper_2007_00745_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("extra", [[], ["--schedule", "static", "--workers", "7"],
                                   ["--schedule", "alternating"], ["--periodicity"],
                                   ["--periodicity", "--block-iters", "7"],
                                   ["--collapse-rows", "1"], ["--collapse-rows", "2"],
                                   ["--collapse-rows", "2", "--periodicity"]])
def test_cli_binary64(tmp_path, capsys, extra):
    path = tmp_path / "img.ppm"
    assert cli.main(["--size", "60", "80", "--max-iter", "400", "--out", str(path)] + extra) == 0
    rep = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    win = workloads.window_from_bounds(-2.0, 1.0, -1.2, 1.2, 60, 80)
    counts = oracle.render(win, 60, 80, 400, 2.0)
    assert rep["sum_counts"] == int(counts.sum())
    # collapsed rows and periodicity detection only ever execute fewer updates
    assert 0 < rep["iterations_executed"] <= rep["sum_counts"]
    assert path.read_bytes() == out_oracle.ppm_bytes(out_oracle.boolean_colour(counts, 400),
                                                     60, 80)


def test_cli_mirrored_rows_render_half_the_rows(capsys, tmp_path):
    # the default window is centred on the real axis, so with mirrored rows only the
    # rows on one side of it (and the axis row, if any) are iterated
    path = tmp_path / "m.ppm"
    assert cli.main(["--size", "64", "80", "--max-iter", "300", "--collapse-rows", "2",
                     "--out", str(path)]) == 0
    rep = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    win = workloads.window_from_bounds(-2.0, 1.0, -1.2, 1.2, 64, 80)
    counts = oracle.render(win, 64, 80, 300, 2.0)
    assert rep["sum_counts"] == int(counts.sum())
    assert rep["iterations_executed"] == int(counts[32:].sum())


def test_cli_double_double(tmp_path, capsys):
    path = tmp_path / "deep.ppm"
    c = (-0.7436438870371587, 0.1318259042053119)
    assert cli.main(["--size", "24", "40", "--max-iter", "3000", "--centre", str(c[0]), str(c[1]),
                     "--pitch", "1e-17", "--double-double", "--out", str(path)]) == 0
    counts = dd_oracle.render((c[0], 0.0, c[1], 0.0, 1e-17, 1e-17), 24, 40, 3000, 2.0)
    assert path.read_bytes() == out_oracle.ppm_bytes(out_oracle.boolean_colour(counts, 3000),
                                                     24, 40)
