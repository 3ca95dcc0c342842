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


GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def published_outputs():
    return [int(l, 16) for l in open(os.path.join(HERE, "golden", "splitmix64_state0.txt"))
            if l.startswith("0x")]


def test_random_offsets_follow_published_outputs(orc):
    """The random-search offsets against the generator's published outputs.

    The stand-in's generator state for counter c is seed + (c + 1) * gamma, so
    with seed = (n - c) * gamma the state is (n + 1) * gamma and the output is
    the n-th published output from state 0, for any counter c.  Each case
    below builds c from (level, iteration, radius index, tile row, tile column)
    as the definition packs them and checks the offset the oracle draws against
    that published value: a wrong packing, a swapped u / v or a wrong modulo
    fails here.
    """
    g = published_outputs()
    assert len(g) >= 2
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 8), (0, 0, 0, 15, 0, 8), (0, 0, 0, 0, 15, 8), (1, 2, 3, 100, 40, 5),
             (4, 5, 0, 1241, 374, 128), (2, 63, 6, 600, 200, 1), (3, 1, 2, 7, 9, 2)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 16)), int(rng.integers(0, 64)), int(rng.integers(0, 8)),
                      int(rng.integers(0, 2048)), int(rng.integers(0, 1100)), int(rng.integers(1, 300))))
    for t, (level, it, k, x, y, r) in enumerate(cases):
        c = (((level * 64 + it) * 64 + k) * 65536 + y // 8) * 65536 + x // 8
        n = t % len(g)
        seed = ((n - c) * GAMMA) & M64
        h = g[n]
        want = ((h & 0xFFFF) % (2 * r + 1) - r, ((h >> 16) & 0xFFFF) % (2 * r + 1) - r)
        assert orc.pm_offset(seed, level, it, k, x, y, r) == want, (level, it, k, x, y, r)


def test_random_offsets_shared_per_tile_only(orc):
    """Pixels of one 8x8 tile draw the same offset; tiles, levels, iterations
    and radius indices draw their own."""
    seed = 1801
    base = orc.pm_offset(seed, 1, 2, 0, 16, 24, 64)
    for x in range(16, 24):
        for y in range(24, 32):
            assert orc.pm_offset(seed, 1, 2, 0, x, y, 64) == base
    others = [orc.pm_offset(seed, 1, 2, 0, 24, 24, 64), orc.pm_offset(seed, 1, 2, 0, 16, 32, 64),
              orc.pm_offset(seed, 0, 2, 0, 16, 24, 64), orc.pm_offset(seed, 1, 3, 0, 16, 24, 64),
              orc.pm_offset(seed, 1, 2, 1, 16, 24, 64)]
    assert sum(o == base for o in others) <= 1  # a coincidence is possible, not a pattern


def test_random_offsets_cover_the_box(orc):
    """Each offset lies in [-r, r]^2 and every displacement of a small box occurs."""
    r = 2
    seen = set()
    for t in range(4000):
        ou, ov = orc.pm_offset(99, 0, 0, 0, 8 * (t % 500), 8 * (t // 500), r)
        assert -r <= ou <= r and -r <= ov <= r
        seen.add((ou, ov))
    assert len(seen) == (2 * r + 1) ** 2


def test_pm_pixel_candidate_sequence(orc):
    """One search step at one pixel: own flow, the neighbours at distance 1 then
    4 (left, right, up, down; outside ones skipped), then one random candidate
    per radius R, R/2, ..., 1 around the best so far; the first lowest cost wins."""
    rng = np.random.default_rng(11)
    H, W = 23, 37
    c0 = rng.integers(0, 2**62, (H, W), dtype=np.uint64)
    c1 = rng.integers(0, 2**62, (H, W), dtype=np.uint64)
    fin = np.zeros((H, W, 2), np.int16)
    ys, xs = np.mgrid[0:H, 0:W]
    fin[..., 0] = rng.integers(-3, 4, (H, W))
    fin[..., 1] = rng.integers(-2, 3, (H, W))
    fin[..., 0] = np.clip(xs + fin[..., 0], 0, W - 1) - xs  # targets inside the image
    fin[..., 1] = np.clip(ys + fin[..., 1], 0, H - 1) - ys
    level, it, Rl, seed = 1, 3, 11, 4242
    for (x, y) in [(0, 0), (W - 1, H - 1), (3, 2), (18, 11), (4, 20), (36, 5), (10, 4)]:
        (bu, bv), tr = orc.pm_pixel(c0, c1, level, it, Rl, seed, fin, x, y)
        want = [(int(fin[y, x, 0]), int(fin[y, x, 1]))]
        for dist in (1, 4):
            for ddx, ddy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                nx, ny = x + dist * ddx, y + dist * ddy
                if 0 <= nx < W and 0 <= ny < H:
                    want.append((int(fin[ny, nx, 0]), int(fin[ny, nx, 1])))
        nfixed = len(want)
        assert [tuple(map(int, t[:2])) for t in tr[:nfixed]] == want
        nrand = len(tr) - nfixed
        assert nrand == int(np.floor(np.log2(Rl))) + 1
        for n, t in enumerate(tr):
            assert t[2] == orc.flow_cost(c0, c1, x, y, int(t[0]), int(t[1]))
        for k in range(nrand):
            prev = tr[:nfixed + k]
            ok = [i for i in range(len(prev)) if prev[i, 2] >= 0]
            best = min(ok, key=lambda i: (prev[i, 2], i))
            ou, ov = orc.pm_offset(seed, level, it, k, x, y, Rl >> k)
            assert tuple(map(int, tr[nfixed + k, :2])) == (int(prev[best, 0]) + ou, int(prev[best, 1]) + ov)
        ok = [i for i in range(len(tr)) if tr[i, 2] >= 0]
        win = min(ok, key=lambda i: (tr[i, 2], i))
        assert (bu, bv) == (int(tr[win, 0]), int(tr[win, 1]))


def test_pm_flow_one_level_is_the_pixel_step(orc):
    """One level and one iteration of the whole stand-in equals the per-pixel
    step applied to the zero field with level 0, iteration 0 and radius R."""
    rng = np.random.default_rng(12)
    H, W, R, seed = 19, 27, 6, 77
    A = noise(rng, H, W)
    B = noise(rng, H, W)
    F = orc.pm_flow(A, B, levels=1, iters=1, R=R, seed=seed)
    c0, c1 = orc.census(A), orc.census(B)
    zero = np.zeros((H, W, 2), np.int16)
    for y in range(H):
        for x in range(W):
            (bu, bv), _ = orc.pm_pixel(c0, c1, 0, 0, R, seed, zero, x, y)
            assert (int(F[y, x, 0]), int(F[y, x, 1])) == (bu, bv)
