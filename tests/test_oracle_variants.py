"""Pins of the oracle's SGM variants (the cited method's right map by diagonal
search, 3x3 median post-filter, intensity-adaptive P2) against brute force,
library routines and special cases that reduce to the plain method."""
import itertools

import numpy as np
import pytest

from paper_1801_04720_amd import synth

CMAX = 62


def rule_p2(g, P1, P2):
    # The reading under test: the penalty across an intensity step g (>= 0).
    return P2 if g == 0 else max(P1, P2 // g)


def brute_path_varying(C, I, P1, P2):
    """Lr along a 1-D path by enumerating every disparity sequence, with the
    large-jump penalty of step k taken from the intensity step I[k] - I[k-1]."""
    n, D = C.shape
    p2 = [None] + [rule_p2(abs(int(I[k]) - int(I[k - 1])), P1, P2) for k in range(1, n)]

    def V(k, a, b):
        return 0 if a == b else (P1 if abs(a - b) == 1 else p2[k])

    E = []
    for k in range(n):
        Ek = [None] * D
        for seq in itertools.product(range(D), repeat=k + 1):
            e = sum(int(C[i, seq[i]]) for i in range(k + 1)) + sum(V(i, seq[i - 1], seq[i]) for i in range(1, k + 1))
            if Ek[seq[-1]] is None or e < Ek[seq[-1]]:
                Ek[seq[-1]] = e
        E.append(Ek)
    L = np.zeros((n, D), np.int64)
    L[0] = C[0]
    for k in range(1, n):
        L[k] = np.array(E[k]) - min(E[k - 1])
    return L


# --- intensity-adaptive P2 ---------------------------------------------------------------

def test_adaptive_brute_force_dp(orc):
    rng = np.random.default_rng(41)
    for case in range(50):
        D = int(rng.integers(1, 5))
        n = int(rng.integers(1, 7 if D <= 3 else 6))
        P1 = int(rng.integers(0, 30))
        P2 = int(rng.integers(P1, 150))
        C = rng.integers(0, CMAX + 1, (n, D)).astype(np.uint8)
        # Intensities with a mix of zero, small and large steps.
        I = np.cumsum(rng.choice([0, 0, 1, 2, 5, 40], n)).astype(np.int64) % 256
        I = I.astype(np.uint8)
        exp = brute_path_varying(C, I, P1, P2)
        assert np.array_equal(orc.path_cost_adaptive(C[None], I[None], P1, P2, 0)[0], exp)
        got = orc.path_cost_adaptive(C[::-1][None].copy(), I[::-1][None].copy(), P1, P2, 1)[0][::-1]
        assert np.array_equal(got, exp)
        assert np.array_equal(orc.path_cost_adaptive(C[:, None, :].copy(), I[:, None].copy(), P1, P2, 2)[:, 0], exp)
        diag = np.zeros((n, n, D), np.uint8)
        img = np.zeros((n, n), np.uint8)
        for i in range(n):
            diag[i, i] = C[i]
            img[i, i] = I[i]
        got = orc.path_cost_adaptive(diag, img, P1, P2, 4)
        assert np.array_equal(np.array([got[i, i] for i in range(n)]), exp)


def test_adaptive_constant_image_is_plain(orc):
    rng = np.random.default_rng(42)
    C = rng.integers(0, CMAX + 1, (9, 13, 6)).astype(np.uint8)
    img = np.full((9, 13), 77, np.uint8)
    assert np.array_equal(orc.aggregate_adaptive(C, img, 10, 120), orc.aggregate(C, 10, 120))


def test_adaptive_unit_steps_keep_p2(orc):
    # A 0/1 checkerboard: every path step changes the intensity by 0 or 1, and
    # P2 / 1 = P2, so the result is the plain aggregation.
    rng = np.random.default_rng(43)
    C = rng.integers(0, CMAX + 1, (8, 11, 7)).astype(np.uint8)
    ys, xs = np.mgrid[0:8, 0:11]
    img = ((xs + ys) % 2).astype(np.uint8)
    assert np.array_equal(orc.aggregate_adaptive(C, img, 10, 120), orc.aggregate(C, 10, 120))


def test_adaptive_strong_edges_give_p1(orc):
    # Four intensities on a 2x2 colouring: every pair of 8-neighbours differs by
    # 60, 120 or 180, so floor(120 / g) <= 2 and the penalty is clamped to P1.
    rng = np.random.default_rng(44)
    C = rng.integers(0, CMAX + 1, (10, 12, 6)).astype(np.uint8)
    ys, xs = np.mgrid[0:10, 0:12]
    img = (60 * (xs % 2) + 120 * (ys % 2)).astype(np.uint8)
    assert np.array_equal(orc.aggregate_adaptive(C, img, 10, 120), orc.aggregate(C, 10, 10))


# --- right map by diagonal search ------------------------------------------------------------

def test_diag_hand_example(orc):
    S = np.array([[[5, 9, 9], [7, 2, 9], [1, 8, 4], [6, 6, 0]],
                  [[3, 3, 3], [3, 3, 3], [3, 3, 3], [3, 3, 3]]], np.uint16)
    # q=0: S(0,0)=5, S(1,1)=2, S(2,2)=4 -> 1;  q=1: 7, 8, 0 -> 2;  q=2: 1, 6 -> 0;
    # q=3: only d=0 -> 0.  Second row: all equal -> smallest d.
    assert np.array_equal(orc.wta_right_diag(S), np.array([[1, 2, 0, 0], [0, 0, 0, 0]], np.int16))


@pytest.mark.parametrize("D", [8, 32])
def test_diag_equals_right_pass_without_smoothing(orc, D):
    # P1 = P2 = 0: S = 8 C, and the right-base cost C_R(q, d) equals C_L(q + d, d),
    # so the diagonal search in S_L reproduces the right view's own WTA wherever
    # every d keeps q + d inside the image.
    p = synth.pair_rectangles(3)
    cl, cr = orc.census(p.left), orc.census(p.right)
    SL = orc.aggregate(orc.cost(cl, cr, D, False), 0, 0)
    SR = orc.aggregate(orc.cost(cr, cl, D, True), 0, 0)
    wr, _ = orc.wta(SR)
    W = p.left.shape[1]
    got = orc.wta_right_diag(SL)
    assert np.array_equal(got[:, :W - D + 1], wr[:, :W - D + 1])


def test_diag_range_respects_image_end(orc):
    rng = np.random.default_rng(45)
    S = rng.integers(0, 1000, (5, 20, 16)).astype(np.uint16)
    w = orc.wta_right_diag(S)
    xs = np.arange(20)[None, :]
    assert (w >= 0).all() and ((xs + w) <= 19).all()


# --- 3x3 median ------------------------------------------------------------------------------

def test_median_matches_library(orc):
    scipy_nd = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(46)
    for H, W in [(1, 1), (1, 7), (6, 1), (13, 17), (40, 53)]:
        m = (rng.random((H, W)) * 100).astype(np.float32)
        m[rng.random((H, W)) < 0.2] = -1.0  # repeated values
        ref = scipy_nd.median_filter(m, size=3, mode="nearest")
        assert np.array_equal(orc.median3x3(m), ref)


def test_median_removes_isolated_outlier(orc):
    m = np.full((9, 9), 4.25, np.float32)
    m[4, 4] = 90.0
    assert np.array_equal(orc.median3x3(m), np.full((9, 9), 4.25, np.float32))


# --- whole map with variants -----------------------------------------------------------------

def test_disparity_ex_no_flags_is_plain(orc):
    p = synth.pair_rectangles(1)
    a = orc.disparity(p.left, p.right, 32)
    b = orc.disparity_ex(p.left, p.right, 32, 0)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_disparity_ex_median_and_diag_wiring(orc):
    p = synth.pair_rectangles(2)
    cl, cr = orc.census(p.left), orc.census(p.right)
    SL = orc.aggregate(orc.cost(cl, cr, 32, False), 10, 120)
    wl, ds = orc.wta(SL)
    wr_diag = orc.wta_right_diag(SL)
    valid, disp = orc.lr_check(wl, wr_diag, orc.median3x3(ds), 1)
    w, d2, v2 = orc.disparity_ex(p.left, p.right, 32, orc.DIAG | orc.MEDIAN)
    assert np.array_equal(w, wl) and np.array_equal(v2, valid) and np.array_equal(d2, disp)


def test_disparity_ex_adaptive_uses_each_views_base_image(orc):
    p = synth.pair_rectangles(0)
    cl, cr = orc.census(p.left), orc.census(p.right)
    SR = orc.aggregate_adaptive(orc.cost(cr, cl, 32, True), p.right, 10, 120)
    SL = orc.aggregate_adaptive(orc.cost(cl, cr, 32, False), p.left, 10, 120)
    wl, ds = orc.wta(SL)
    wr, _ = orc.wta(SR)
    valid, disp = orc.lr_check(wl, wr, ds, 1)
    w, d2, v2 = orc.disparity_ex(p.left, p.right, 32, orc.ADAPTIVE)
    assert np.array_equal(w, wl) and np.array_equal(v2, valid) and np.array_equal(d2, disp)


@pytest.mark.parametrize("idx", [0, 1])
def test_diag_lr_keeps_most_of_the_clean_interior(orc, idx):
    # The diagonal search compares S of different left pixels, so it is not exact;
    # on piecewise-constant pairs it still keeps nearly all of the clean interior.
    from test_oracle_sgm import clean_interior

    p = synth.pair_rectangles(idx)
    w, disp, valid = orc.disparity_ex(p.left, p.right, 32, orc.DIAG)
    ok = clean_interior(p)
    assert np.array_equal(w[ok], p.gt_disp[ok].astype(np.int16))
    assert valid[ok].mean() >= 0.95
