"""GPU tests of the output path: the colouring kernel against the oracle's
Boolean colouring (oracle/output.py) on aligned, misaligned and ragged buffers,
and whole images written to PPM files -- counts rendered on the GPU, coloured,
copied and written, sequentially and pipelined -- against the file the oracle's
counts, colours and byte layout give."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import output as out_oracle
from paper_2007_00745_amd import native, output, workloads

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.parametrize("npix", [1, 3, 4, 5, 1000, 4097, 65539])
@pytest.mark.parametrize("offsets", [(0, 0), (1, 0), (0, 1), (3, 2)])
def test_colour_kernel(npix, offsets):
    rng = np.random.default_rng(npix)
    mi = 100
    host = rng.integers(1, mi + 1, npix + 8).astype(np.int32)
    host[rng.random(npix + 8) < 0.3] = mi
    oc, orgb = offsets
    counts = torch.tensor(host, device="cuda")[oc:oc + npix]
    rgb_buf = torch.full((3 * npix + 8,), 7, dtype=torch.uint8, device="cuda")
    rgb = rgb_buf[orgb:orgb + 3 * npix]
    _log(f"colour npix={npix} offsets={offsets}")
    native.colour_boolean(counts, mi, rgb)
    torch.cuda.synchronize()
    want = out_oracle.boolean_colour(host[oc:oc + npix], mi).ravel()
    assert np.array_equal(rgb.cpu().numpy(), want)
    rest = rgb_buf.cpu().numpy()
    assert (rest[:orgb] == 7).all() and (rest[orgb + 3 * npix:] == 7).all()


def test_colour_kernel_grid_stride():
    # more quads than one launch has threads (65536 blocks of 256): every pixel is
    # still coloured, black exactly where the count reached max_iter
    npix = 65536 * 256 * 4 + 13
    counts = torch.randint(1, 11, (npix,), dtype=torch.int32, device="cuda")
    rgb = native.colour_boolean(counts, 10)
    torch.cuda.synchronize()
    black = (counts >= 10)
    assert torch.equal(rgb[:, 0] == 0, black) and torch.equal(rgb[:, 0] == 255, ~black)
    assert torch.equal(rgb[:, 0], rgb[:, 1]) and torch.equal(rgb[:, 1], rgb[:, 2])


def test_single_image_file(tmp_path):
    v = workloads.c1()
    counts = native.render(v.window, v.m, v.n, v.max_iter, v.R)
    rgb = native.colour_boolean(counts, v.max_iter)
    path = tmp_path / "c1.ppm"
    native.write_ppm(str(path), rgb.cpu(), v.m, v.n)
    want = out_oracle.ppm_bytes(out_oracle.boolean_colour(
        oracle.render(v.window, v.m, v.n, v.max_iter, v.R), v.max_iter), v.m, v.n)
    assert path.read_bytes() == want


@pytest.mark.parametrize("pipelined", [False, True])
def test_sequence_to_files(tmp_path, pipelined):
    # a short zoom sequence of uneven sizes; every file equals the oracle's
    views = [workloads.View(workloads.window_from_bounds(-2, 1, -1.2, 1.2, 90, 120), 90, 120, 300),
             workloads.View((-0.745, 0.113, 1e-3 / 64, 1e-3 / 64), 48, 64, 2000),
             workloads.View((-0.745, 0.113, 1e-4 / 100, 1e-4 / 100), 77, 100, 3000),
             workloads.View((0.3, 0.5, 0.01, 0.01), 1, 1, 50)]
    paths = [str(tmp_path / f"f{k}.ppm") for k in range(len(views))]
    res = output.render_to_ppm(views, paths, pipelined=pipelined)
    _log(f"sequence {res}")
    for v, p in zip(views, paths):
        want = out_oracle.ppm_bytes(out_oracle.boolean_colour(
            oracle.render(v.window, v.m, v.n, v.max_iter, v.R), v.max_iter), v.m, v.n)
        assert open(p, "rb").read() == want
