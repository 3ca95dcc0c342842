"""Pins of the oracle's optical-flow stand-in: the random generator against its
published outputs, the pyramid and the data term against direct numpy forms,
and flows with known answers (no motion, integer translations)."""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def noise(rng, H, W):
    return rng.integers(0, 256, (H, W)).astype(np.uint8)


def test_splitmix64_published_outputs(orc):
    vals = [int(l, 16) for l in open(os.path.join(HERE, "golden", "splitmix64_state0.txt"))
            if l.startswith("0x")]
    # Counter c of the stand-in is output number c + 1 of the sequence from `seed`.
    assert [orc.splitmix64(0, c) for c in range(len(vals))] == vals


def test_pyramid_is_rounded_box_mean(orc):
    rng = np.random.default_rng(1)
    for H, W in [(8, 12), (7, 9), (1, 1), (1, 6), (5, 1)]:
        a = noise(rng, H, W)
        p = np.pad(a.astype(np.int64), ((0, H % 2), (0, W % 2)), mode="edge")
        s = p[0::2, 0::2] + p[1::2, 0::2] + p[0::2, 1::2] + p[1::2, 1::2]
        assert np.array_equal(orc.pyr_down(a), ((s + 2) // 4).astype(np.uint8))


def test_flow_cost_definition(orc):
    rng = np.random.default_rng(2)
    H, W = 11, 17
    c0 = rng.integers(0, 2**62, (H, W), dtype=np.uint64)
    c1 = rng.integers(0, 2**62, (H, W), dtype=np.uint64)
    for _ in range(200):
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        fu, fv = int(rng.integers(-6, 7)), int(rng.integers(-4, 5))
        tx, ty = x + fu, y + fv
        if not (0 <= tx < W and 0 <= ty < H):
            assert orc.flow_cost(c0, c1, x, y, fu, fv) == -1
            continue
        s = 0
        for j in (-2, 0, 2):
            for i in (-2, 0, 2):
                a = int(c0[min(max(y + j, 0), H - 1), min(max(x + i, 0), W - 1)])
                b = int(c1[min(max(ty + j, 0), H - 1), min(max(tx + i, 0), W - 1)])
                s += bin(a ^ b).count("1")
        assert orc.flow_cost(c0, c1, x, y, fu, fv) == s


def test_no_motion_gives_zero_flow(orc):
    rng = np.random.default_rng(3)
    a = noise(rng, 40, 64)
    F, B, out = orc.flow(a, a, levels=3, iters=2, R=32)
    assert (F == 0).all() and (B == 0).all()
    assert (out == 0).all()


@pytest.mark.parametrize("du,dv", [(5, 0), (-7, 3), (13, -6)])
def test_integer_translation_recovered(orc, du, dv):
    rng = np.random.default_rng(10 + du)
    H, W = 64, 96
    big = noise(rng, H + 40, W + 40)
    A = big[20:20 + H, 20:20 + W].copy()
    B = big[20 + dv:20 + dv + H, 20 + du:20 + du + W].copy()  # A(x) = B(x - (du, dv))
    # B is A moved by (-du, -dv): the flow from A to B is (-du, -dv).
    F, Bk, out = orc.flow(A, B, levels=3, iters=8, R=32)
    m = 8  # census window + sample grid + clamped borders
    inner = (slice(m + abs(dv), H - m - abs(dv)), slice(m + abs(du), W - m - abs(du)))
    assert (F[inner][..., 0] == -du).all() and (F[inner][..., 1] == -dv).all()
    assert (out[inner][..., 0] == -du).all() and (out[inner][..., 1] == -dv).all()
