"""The largest workloads against the oracle at sampled pixels: the plain frame at
2048x1024 D=256 (the stream's frame size) and a batch holding the three pair
sizes of the uneven batch, 1920x1080 D=256 included, in the graph-captured
launch the batch bench times.  The oracle computes each sampled pixel's left
costs along the eight lines into it, the right costs at x - d*_L, WTA,
sub-pixel and the LR check; every sampled output must match bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import synth  # noqa: E402
from paper_1801_04720_amd.batch import Batch  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def samples(rng, H, W, n):
    # Random pixels plus the four corners and the middle of every border.
    xs = list(rng.integers(0, W, n)) + [0, W - 1, 0, W - 1, W // 2, W // 2, 0, W - 1]
    ys = list(rng.integers(0, H, n)) + [0, 0, H - 1, H - 1, 0, H - 1, H // 2, H // 2]
    return np.array(xs, np.int32), np.array(ys, np.int32)


def check_map(orc, L, R, D, disp, valid, xs, ys):
    w, d, v = orc.disparity_at(L, R, D, xs, ys)
    assert np.array_equal(host(valid)[ys, xs], v)
    assert np.array_equal(host(disp)[ys, xs], d)


def test_frame_2048x1024_d256_sampled(orc):
    say("plain frame 2048x1024 D=256, sampled oracle")
    fr = synth.frame_planar(synth.rng_for(5, 3), 1024, 2048, 256, 200.0)
    ff = FusedFrame(1024, 2048, 256, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    xs, ys = samples(rng, 1024, 2048, 24)
    check_map(orc, fr.t0.left, fr.t0.right, 256, got["disp0"], got["valid0"], xs, ys)
    xs, ys = samples(rng, 1024, 2048, 24)
    check_map(orc, fr.t1.left, fr.t1.right, 256, got["disp1"], got["valid1"], xs, ys)


def test_uneven_batch_graph_sampled(orc):
    say("uneven batch (640x480/64, 1242x375/128, 1920x1080/256) in one graph, sampled oracle")
    sizes = [(480, 640, 64), (375, 1242, 128), (1080, 1920, 256)]
    pairs = [synth.pair_batch(i, *s) for i, s in enumerate(sizes)]
    ts = [{"left": dev(p.left), "right": dev(p.right), "D": s[2]} for p, s in zip(pairs, sizes)]
    b = Batch(ts, device=DEV)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        b.capture(st)
        out = b.launch(st)
        torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    for p, s, o in zip(pairs, sizes, out):
        H, W, D = s
        xs, ys = samples(rng, H, W, 16)
        say("  pair", s)
        check_map(orc, p.left, p.right, D, o["disp"], o["valid"], xs, ys)
