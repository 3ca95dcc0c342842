"""Pins of the oracle's temporal validation over three time steps."""
import numpy as np


def vec(u, v, d0, d1):
    return np.array([u, v, d0, d1], np.float32)


def empty(H, W):
    return np.full((H, W, 4), np.nan, np.float32), np.zeros((H, W), np.uint8)


def test_temporal_worked_example(orc):
    a, va = empty(1, 6)
    b, vb = empty(1, 6)
    a[0, 0], va[0, 0] = vec(2, 0, 5, 6), 1      # -> q = 2, matches b there
    a[0, 1], va[0, 1] = vec(5, 0, 5, 6), 1      # target x = 6 leaves the image
    a[0, 3], va[0, 3] = vec(1.49, 0, 5, 6), 1   # floor(4.49 + 0.5) = 4, b undefined there
    a[0, 4], va[0, 4] = vec(0.5, 0, 5, 6), 1    # floor(4.5 + 0.5) = 5
    a[0, 5], va[0, 5] = vec(-3, 0, 5, 6), 1     # q = 2, flow differs by 5 > 2
    b[0, 2], vb[0, 2] = vec(2.5, 0.1, 6, 7.2), 1  # |du| 0.5, |dv| 0.1, |1 - 1.2| = 0.2
    b[0, 5], vb[0, 5] = vec(0.5, 0, 5, 7.5), 1    # disparity change 1 vs 2.5 -> 1.5 > 1
    out = orc.temporal_check(a, va, b, vb, 2.0, 1.0)
    assert out.tolist() == [[1, 0, 0, 0, 0, 0]]
    out = orc.temporal_check(a, va, b, vb, 2.0, 1.5)  # the disparity tolerance is inclusive
    assert out.tolist() == [[1, 0, 0, 0, 1, 0]]


def test_temporal_constant_motion(orc):
    H, W = 20, 30
    a = np.zeros((H, W, 4), np.float32)
    a[...] = vec(3, -2, 10, 11)
    va = np.ones((H, W), np.uint8)
    out = orc.temporal_check(a, va, a, va, 0.0, 0.0)
    ys, xs = np.mgrid[0:H, 0:W]
    inside = (xs + 3 <= W - 1) & (ys - 2 >= 0)
    assert np.array_equal(out.astype(bool), inside)


def test_temporal_planted_inconsistency(orc):
    rng = np.random.default_rng(7)
    H, W = 16, 24
    a = np.zeros((H, W, 4), np.float32)
    a[...] = vec(1, 1, 20, 20.5)
    b = a.copy()
    b[9, 9, 3] += 2.0  # one pixel at t1 changes its disparity step by 2
    va = (rng.random((H, W)) < 0.9).astype(np.uint8)
    vb = np.ones((H, W), np.uint8)
    out = orc.temporal_check(a, va, b, vb, 2.0, 1.0)
    exp = va.copy()
    exp[H - 1, :] = 0
    exp[:, W - 1] = 0
    exp[8, 8] = 0  # (8, 8) + (1, 1) lands on the changed pixel
    assert np.array_equal(out, exp)
    assert not (out.astype(bool) & ~(va.astype(bool))).any()
