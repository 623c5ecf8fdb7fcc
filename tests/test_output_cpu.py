"""The output path on the host: the library's PPM writer against the oracle's
byte layout (oracle/output.py) and a small independent reader of the Netpbm
format, plus argument checks of the colouring entry point (no GPU needed)."""

import numpy as np
import pytest

from oracle import output as out_oracle
from paper_2007_00745_amd import native


def _read_ppm(data: bytes):
    # header tokens separated by whitespace, one whitespace byte before the raster
    tokens, pos = [], 0
    while len(tokens) < 4:
        while data[pos:pos + 1].isspace():
            pos += 1
        start = pos
        while not data[pos:pos + 1].isspace():
            pos += 1
        tokens.append(data[start:pos].decode())
    magic, w, h, maxval = tokens[0], int(tokens[1]), int(tokens[2]), int(tokens[3])
    raster = np.frombuffer(data[pos + 1:], dtype=np.uint8)
    return magic, w, h, maxval, raster.reshape(h, w, 3)


def test_boolean_colour_definition():
    counts = np.array([[1, 5, 10], [10, 9, 11]])
    rgb = out_oracle.boolean_colour(counts, 10)
    assert rgb.shape == (2, 3, 3)
    assert (rgb[0, 2] == 0).all() and (rgb[1, 0] == 0).all() and (rgb[1, 2] == 0).all()
    assert (rgb[0, 0] == 255).all() and (rgb[1, 1] == 255).all()


@pytest.mark.parametrize("m,n", [(1, 1), (3, 5), (48, 64), (7, 0)])
def test_write_ppm_matches_the_format(tmp_path, m, n):
    rng = np.random.default_rng(m * 100 + n)
    rgb = rng.integers(0, 256, (m, n, 3), dtype=np.uint8)
    path = tmp_path / "img.ppm"
    native.write_ppm(str(path), rgb, m, n)
    data = path.read_bytes()
    assert data == out_oracle.ppm_bytes(rgb, m, n)
    magic, w, h, maxval, raster = _read_ppm(data)
    assert (magic, w, h, maxval) == ("P6", n, m, 255)
    assert np.array_equal(raster, rgb)


def test_write_ppm_errors(tmp_path):
    rgb = np.zeros(12, dtype=np.uint8)
    with pytest.raises(native.MandelError) as e:
        native.write_ppm(str(tmp_path / "no" / "such" / "dir.ppm"), rgb, 2, 2)
    assert e.value.code == native.EIO
    L = native.lib()
    assert L.mandel_write_ppm(None, rgb.ctypes.data, 2, 2) == native.EINVAL
    assert L.mandel_write_ppm(b"/tmp/x.ppm", None, 2, 2) == native.EINVAL
    assert L.mandel_write_ppm(b"/tmp/x.ppm", rgb.ctypes.data, -1, 2) == native.EINVAL


def test_colour_argument_checks():
    L = native.lib()
    assert L.mandel_colour_boolean(0x1000, -1, 10, 0x2000, None) == native.EINVAL
    assert L.mandel_colour_boolean(0x1000, 8, 0, 0x2000, None) == native.EINVAL
    assert L.mandel_colour_boolean(None, 8, 10, 0x2000, None) == native.EINVAL
    assert L.mandel_colour_boolean(0x1000, 0, 10, None, None) == native.OK


def test_cli_argument_errors():
    from paper_2007_00745_amd import __main__ as cli
    with pytest.raises(SystemExit):
        cli.main(["--centre", "0", "0"])                      # no pitch
    with pytest.raises(SystemExit):
        cli.main(["--double-double", "--schedule", "static"])
    with pytest.raises(SystemExit):
        cli.main(["--double-double", "--collapse-rows", "1"])
    with pytest.raises(SystemExit):
        cli.main(["--collapse-rows", "2", "--schedule", "alternating"])
    with pytest.raises(SystemExit):
        cli.main(["--collapse-rows", "3"])
