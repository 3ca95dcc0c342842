"""Aggregation with the costs computed from the census images inside the path
walk (sf_sgm_aggregate_census) against the CPU oracle (cost volume from the
oracle's Hamming costs, then the oracle's eight-path aggregation): bit-exact
for every D, both bases, both output stages, penalties, path subsets, shapes
with more disparities than columns, a census of a real image pair, and at
1242x375 D = 128 the whole volume against the cost-volume path plus sampled
oracle pixels on every path start (first and last row and column)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, synth  # noqa: E402

from gpu_util import dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_census(rng, H, W):
    """Uniform 62-bit census words (bits 62, 63 zero, as sf_census writes them)."""
    return rng.integers(0, 1 << 62, (H, W), dtype=np.uint64)


def run(cb, cm, D, right, P1, P2, mask=0xFF):
    return host(api.sgm_aggregate_census(dev(cb), dev(cm), D, right, P1, P2, mask), np.uint16)


@pytest.mark.parametrize("D", [32, 64, 96, 128, 160, 192, 224, 256])
@pytest.mark.parametrize("right", [0, 1])
@pytest.mark.parametrize("mode", [1, 2])
def test_every_D(orc, D, right, mode):
    say("census aggregate D", D, "right", right, "mode", mode)
    rng = np.random.default_rng(1000 * D + 10 * right + mode)
    H, W = 21, 300
    cb, cm = rand_census(rng, H, W), rand_census(rng, H, W)
    api.sgm_set_epilogue(mode)
    try:
        got = run(cb, cm, D, right, 10, 120)
    finally:
        api.sgm_set_epilogue(0)
    ref = orc.aggregate(orc.cost(cb, cm, D, bool(right)), 10, 120)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("H,W", [(1, 1), (1, 40), (40, 1), (2, 3), (33, 17), (17, 70), (9, 131)])
@pytest.mark.parametrize("right", [0, 1])
def test_shapes(orc, H, W, right):
    say("census aggregate shape", H, W, right)
    rng = np.random.default_rng(H * 7 + W + right)
    cb, cm = rand_census(rng, H, W), rand_census(rng, H, W)
    got = run(cb, cm, 64, right, 10, 120)
    assert np.array_equal(got, orc.aggregate(orc.cost(cb, cm, 64, bool(right)), 10, 120))


@pytest.mark.parametrize("P1,P2", [(0, 0), (1, 193), (10, 194), (50, 2000), (0, 8000)])
def test_penalties(orc, P1, P2):
    say("census aggregate penalties", P1, P2)
    rng = np.random.default_rng(P1 * 31 + P2)
    cb, cm = rand_census(rng, 19, 90), rand_census(rng, 19, 90)
    for right in (0, 1):
        got = run(cb, cm, 32, right, P1, P2)
        assert np.array_equal(got, orc.aggregate(orc.cost(cb, cm, 32, bool(right)), P1, P2)), right


@pytest.mark.parametrize("mask", [1, 2, 4, 8, 16, 32, 64, 128, 0x0F, 0xF0, 0x55])
def test_path_masks(orc, mask):
    say("census aggregate mask", mask)
    rng = np.random.default_rng(mask)
    cb, cm = rand_census(rng, 23, 71), rand_census(rng, 23, 71)
    got = run(cb, cm, 32, mask & 1, 10, 120, mask)
    assert np.array_equal(got, orc.aggregate(orc.cost(cb, cm, 32, bool(mask & 1)), 10, 120, mask))


def test_image_pair(orc):
    say("census aggregate 320x96 pair")
    p = synth.pair_rectangles(0)
    cl, cr = orc.census(p.left), orc.census(p.right)
    assert np.array_equal(run(cl, cr, 32, 0, 10, 120), orc.aggregate(orc.cost(cl, cr, 32, False), 10, 120))
    assert np.array_equal(run(cr, cl, 32, 1, 10, 120), orc.aggregate(orc.cost(cr, cl, 32, True), 10, 120))


@pytest.mark.parametrize("right", [0, 1])
def test_full_size_1242x375(orc, right):
    """The whole 375x1242x128 volume equals the cost-volume path's (itself
    bit-exact against the oracle elsewhere); oracle pixels on every path start."""
    say("census aggregate 1242x375 D=128, right", right)
    H, W, D = 375, 1242, 128
    p = synth.pair_planar(synth.rng_for(4, 7), H, W, D)
    L, R = dev(p.left), dev(p.right)
    cl, cr = api.census(L), api.census(R)
    cb, cm = (cr, cl) if right else (cl, cr)
    got = api.sgm_aggregate_census(cb, cm, D, right, 10, 120)
    ref = api.sgm_aggregate(api.cost(cb, cm, D, bool(right)), 10, 120)
    assert torch.equal(got, ref)
    g = host(got, np.uint16)
    cbh, cmh = host(cb, np.uint64), host(cm, np.uint64)
    pts = [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1), (617, 0), (617, H - 1), (0, 190), (W - 1, 190),
           (5, 3), (W - 6, H - 4), (640, 200)]
    for x, y in pts:
        assert np.array_equal(g[y, x], orc.aggregate_at(cbh, cmh, D, right, 10, 120, x, y)), (x, y)
