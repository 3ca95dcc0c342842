"""Pins of the oracle's densification of the sparse scene-flow map: worked
examples, the trivial cases and properties every output must have."""
import numpy as np


def vec(u, v, d0, d1):
    return np.array([u, v, d0, d1], np.float32)


def test_densify_worked_example(orc):
    H, W = 3, 6
    sf4 = np.full((H, W, 4), np.nan, np.float32)
    valid = np.zeros((H, W), np.uint8)
    A, B, C = vec(1, 2, 10, 11), vec(3, 4, 5, 6), vec(7, 8, 20, 21)
    sf4[0, 0], valid[0, 0] = A, 1
    sf4[0, 3], valid[0, 3] = B, 1
    sf4[2, 4], valid[2, 4] = C, 1
    out, fill = orc.densify(sf4, valid)
    # Row 0: x=1,2 lie between A (d0 10) and B (d0 5): the farther surface B wins;
    # x=4,5 have only B on their left.
    for x, e in zip(range(6), [A, B, B, B, B, B]):
        assert np.array_equal(out[0, x], e), x
    assert fill[0].tolist() == [1, 2, 2, 1, 2, 2]
    # Row 2: everything takes C (the only defined pixel).
    assert all(np.array_equal(out[2, x], C) for x in range(W))
    # Row 1 has nothing: rows 0 and 2 are equally near, the row above wins.
    assert np.array_equal(out[1], out[0]) and (fill[1] == 3).all()


def test_densify_ties_go_left(orc):
    sf4 = np.full((1, 5, 4), np.nan, np.float32)
    valid = np.zeros((1, 5), np.uint8)
    sf4[0, 0], sf4[0, 4] = vec(1, 1, 9, 9), vec(2, 2, 9, 9)
    valid[0, [0, 4]] = 1
    out, _ = orc.densify(sf4, valid)
    assert all(np.array_equal(out[0, x], vec(1, 1, 9, 9)) for x in range(4))


def test_densify_trivial_cases(orc):
    rng = np.random.default_rng(3)
    sf4 = rng.normal(0, 5, (7, 9, 4)).astype(np.float32)
    out, fill = orc.densify(sf4, np.ones((7, 9), np.uint8))
    assert np.array_equal(out, sf4) and (fill == 1).all()
    out, fill = orc.densify(sf4, np.zeros((7, 9), np.uint8))
    assert np.isnan(out).all() and (fill == 0).all()


def test_densify_properties_random(orc):
    rng = np.random.default_rng(4)
    for density in (0.02, 0.3, 0.9):
        H, W = 23, 41
        valid = (rng.random((H, W)) < density).astype(np.uint8)
        valid[rng.integers(0, H, 3)] = 0  # some empty rows
        sf4 = rng.normal(0, 20, (H, W, 4)).astype(np.float32)
        sf4[valid == 0] = np.nan
        out, fill = orc.densify(sf4, valid)
        rows = valid.any(axis=1)
        assert (fill[valid == 1] == 1).all() and np.array_equal(out[valid == 1], sf4[valid == 1])
        assert not np.isnan(out).any()
        for y in range(H):
            if not rows[y]:
                assert (fill[y] == 3).all()
                # the copied row is the nearest non-empty one (above on ties)
                src = min((r for r in range(H) if rows[r]), key=lambda r: (abs(y - r), r))
                assert np.array_equal(out[y], out[src])
                continue
            xs = np.nonzero(valid[y])[0]
            for x in np.nonzero(valid[y] == 0)[0]:
                assert fill[y, x] == 2
                left = xs[xs < x]
                right = xs[xs > x]
                cands = ([left[-1]] if len(left) else []) + ([right[0]] if len(right) else [])
                # the value is one of the boundary pixels', and the one with the smaller d0
                assert any(np.array_equal(out[y, x], sf4[y, c]) for c in cands)
                assert out[y, x, 2] == min(sf4[y, c, 2] for c in cands)
