"""Pins of the CPU oracle's SGM and combination stages against facts fixed by
the mathematics (brute force, closed forms, invariants, special cases, exact
recovery), never against the oracle's own formulas retyped."""
import itertools

import numpy as np
import pytest

from paper_1801_04720_amd import synth

CMAX = 62


# --- census ---------------------------------------------------------------------------

def census_brute(img):
    """9x7 window, row-major neighbours, centre skipped, bit = neighbour < centre,
    clamp-to-edge; first neighbour is the most significant of 62 bits."""
    H, W = img.shape
    out = np.zeros((H, W), np.uint64)
    for y in range(H):
        for x in range(W):
            bits = []
            for dy in range(-3, 4):
                for dx in range(-4, 5):
                    if dx == 0 and dy == 0:
                        continue
                    yy = min(max(y + dy, 0), H - 1)
                    xx = min(max(x + dx, 0), W - 1)
                    bits.append(1 if img[yy, xx] < img[y, x] else 0)
            out[y, x] = int("".join(map(str, bits)), 2)
    return out


def test_census_brute_force(orc):
    rng = np.random.default_rng(1)
    for H, W in [(9, 13), (1, 1), (1, 7), (6, 1), (3, 4)]:
        img = rng.integers(0, 256, (H, W)).astype(np.uint8)
        assert np.array_equal(orc.census(img), census_brute(img))


def test_census_constant_and_impulse(orc):
    assert not orc.census(np.full((10, 12), 77, np.uint8)).any()
    img = np.full((11, 11), 100, np.uint8)
    img[5, 5] = 10  # a dark impulse: every other pixel whose window holds it sees bit 1
    c = orc.census(img)
    assert c[5, 5] == 0
    # Pixel (5, 5 + 1): the impulse is neighbour (dy=0, dx=-1); neighbours before it in
    # row-major order: 3 rows of 9 + 3 = 30 -> it is the 31st of 62 -> bit 62 - 31 = 31.
    assert c[5, 6] == np.uint64(1) << np.uint64(31)
    # Pixel (2, 1): impulse at dy=+3, dx=+4 -> the last neighbour -> bit 0.
    assert c[2, 1] == 1
    # Pixel (8, 9): impulse at dy=-3, dx=-4 -> the first neighbour -> bit 61.
    assert c[8, 9] == np.uint64(1) << np.uint64(61)
    assert int(c.max()) < (1 << 62)


def test_census_monotone_invariance(orc):
    rng = np.random.default_rng(2)
    img = rng.integers(0, 200, (20, 25)).astype(np.uint8)
    base = orc.census(img)
    assert np.array_equal(orc.census(img + 55), base)
    # A random strictly increasing map of 0..199 into 0..255.
    lut = np.sort(rng.choice(256, 200, replace=False)).astype(np.uint8)
    assert np.array_equal(orc.census(lut[img]), base)


# --- cost -----------------------------------------------------------------------------

def test_cost_bitcount_and_oob(orc):
    rng = np.random.default_rng(3)
    H, W, D = 4, 17, 9
    cb = rng.integers(0, 1 << 62, (H, W), dtype=np.uint64)
    cm = rng.integers(0, 1 << 62, (H, W), dtype=np.uint64)
    for right in (False, True):
        c = orc.cost(cb, cm, D, right)
        for y in range(H):
            for x in range(W):
                for d in range(D):
                    xm = x + d if right else x - d
                    exp = CMAX if not (0 <= xm < W) else (int(cb[y, x]) ^ int(cm[y, xm])).bit_count()
                    assert c[y, x, d] == exp


def test_cost_left_right_relation(orc):
    p = synth.pair_rectangles(3)
    cl, cr = orc.census(p.left), orc.census(p.right)
    D = 32
    CL = orc.cost(cl, cr, D, False)
    CR = orc.cost(cr, cl, D, True)
    H, W = p.left.shape
    for d in range(D):
        # C_R(x, y, d) == C_L(x + d, y, d) wherever x + d is inside the image.
        assert np.array_equal(CR[:, : W - d, d], CL[:, d:, d])


# --- path aggregation -----------------------------------------------------------------

def brute_path(C, P1, P2):
    """Lr along a 1-D path by enumerating every disparity sequence."""
    n, D = C.shape

    def V(a, b):
        return 0 if a == b else (P1 if abs(a - b) == 1 else P2)

    E = []
    for k in range(n):
        Ek = [None] * D
        for seq in itertools.product(range(D), repeat=k + 1):
            e = sum(int(C[i, seq[i]]) for i in range(k + 1)) + sum(V(seq[i - 1], seq[i]) for i in range(1, k + 1))
            if Ek[seq[-1]] is None or e < Ek[seq[-1]]:
                Ek[seq[-1]] = e
        E.append(Ek)
    L = np.zeros((n, D), np.int64)
    L[0] = C[0]
    for k in range(1, n):
        L[k] = np.array(E[k]) - min(E[k - 1])
    return L


def test_path_cost_brute_force_dp(orc):
    rng = np.random.default_rng(4)
    for case in range(60):
        D = int(rng.integers(1, 6))
        n = int(rng.integers(1, 8 if D <= 3 else (7 if D == 4 else 6)))
        P1 = int(rng.integers(0, 40))
        P2 = int(rng.integers(P1, 150))
        C = rng.integers(0, CMAX + 1, (n, D)).astype(np.uint8)
        exp = brute_path(C, P1, P2)
        # Left-to-right along a 1xn image (direction 0), right-to-left (1) on the reversed path.
        assert np.array_equal(orc.path_cost(C[None], P1, P2, 0)[0], exp)
        assert np.array_equal(orc.path_cost(C[::-1][None].copy(), P1, P2, 1)[0][::-1], exp)
        # Top-to-bottom along an nx1 image (direction 2) and the diagonal of an nxn image (4).
        assert np.array_equal(orc.path_cost(C[:, None, :].copy(), P1, P2, 2)[:, 0], exp)
        diag = np.full((n, n, D), 0, np.uint8)
        for i in range(n):
            diag[i, i] = C[i]
        got = orc.path_cost(diag, P1, P2, 4)
        assert np.array_equal(np.array([got[i, i] for i in range(n)]), exp)


def test_path_cost_bound(orc):
    p = synth.pair_rectangles(5)
    cl, cr = orc.census(p.left), orc.census(p.right)
    C = orc.cost(cl, cr, 32, False)
    for P1, P2 in [(10, 120), (5, 30), (0, 200)]:
        for r in range(8):
            L = orc.path_cost(C, P1, P2, r)
            assert L.min() >= 0
            assert L.max() <= CMAX + P2
            assert (L - L.min(axis=2, keepdims=True)).max() <= CMAX + P2


def test_aggregate_special_cases(orc):
    rng = np.random.default_rng(6)
    C = rng.integers(0, CMAX + 1, (7, 9, 5)).astype(np.uint8)
    # P1 = P2 = 0: every path cost equals the matching cost.
    assert np.array_equal(orc.aggregate(C, 0, 0).astype(np.int64), 8 * C.astype(np.int64))
    # Constant cost c: S == 8c everywhere and WTA picks d = 0.
    Cc = np.full((6, 8, 7), 13, np.uint8)
    S = orc.aggregate(Cc, 10, 120)
    assert (S == 8 * 13).all()
    w, ds = orc.wta(S)
    assert (w == 0).all() and (ds == 0).all()
    # 1x1 image.
    C1 = rng.integers(0, CMAX + 1, (1, 1, 6)).astype(np.uint8)
    assert np.array_equal(orc.aggregate(C1, 10, 120), 8 * C1.astype(np.uint16))
    # 1xW image: six directions restart at every pixel (paths checked by brute force).
    Cr = rng.integers(0, CMAX + 1, (1, 6, 4)).astype(np.uint8)
    exp = 6 * Cr.astype(np.int64) + brute_path(Cr[0], 10, 120)[None] + brute_path(Cr[0][::-1], 10, 120)[::-1][None]
    assert np.array_equal(orc.aggregate(Cr, 10, 120).astype(np.int64), exp)
    # Hx1 image.
    Cv = rng.integers(0, CMAX + 1, (6, 1, 4)).astype(np.uint8)
    exp = 6 * Cv.astype(np.int64)[:, 0] + brute_path(Cv[:, 0], 7, 50) + brute_path(Cv[::-1, 0], 7, 50)[::-1]
    assert np.array_equal(orc.aggregate(Cv, 7, 50).astype(np.int64)[:, 0], exp)


MIRROR_X = [1, 0, 2, 3, 5, 4, 7, 6]      # (rx, ry) -> (-rx, ry)
MIRROR_Y = [0, 1, 3, 2, 6, 7, 4, 5]      # (rx, ry) -> (rx, -ry)
TRANSPOSE = [2, 3, 0, 1, 4, 6, 5, 7]     # (rx, ry) -> (ry, rx)


def test_aggregate_symmetries(orc):
    rng = np.random.default_rng(7)
    C = rng.integers(0, CMAX + 1, (9, 12, 6)).astype(np.uint8)
    P1, P2 = 9, 70
    S = orc.aggregate(C, P1, P2)
    assert np.array_equal(orc.aggregate(C[:, ::-1].copy(), P1, P2), S[:, ::-1])
    assert np.array_equal(orc.aggregate(C[::-1].copy(), P1, P2), S[::-1])
    assert np.array_equal(orc.aggregate(C.transpose(1, 0, 2).copy(), P1, P2), S.transpose(1, 0, 2))
    for r in range(8):
        L = orc.path_cost(C, P1, P2, r)
        assert np.array_equal(orc.path_cost(C[:, ::-1].copy(), P1, P2, MIRROR_X[r]), L[:, ::-1])
        assert np.array_equal(orc.path_cost(C[::-1].copy(), P1, P2, MIRROR_Y[r]), L[::-1])
        assert np.array_equal(orc.path_cost(C.transpose(1, 0, 2).copy(), P1, P2, TRANSPOSE[r]),
                              L.transpose(1, 0, 2))


def test_path_mask_is_sum_of_directions(orc):
    rng = np.random.default_rng(8)
    C = rng.integers(0, CMAX + 1, (5, 7, 4)).astype(np.uint8)
    tot = sum(orc.path_cost(C, 10, 120, r).astype(np.int64) for r in range(8))
    assert np.array_equal(orc.aggregate(C, 10, 120).astype(np.int64), tot)
    assert np.array_equal(orc.aggregate(C, 10, 120, 1 << 3).astype(np.int64), orc.path_cost(C, 10, 120, 3))


# --- WTA and sub-pixel ------------------------------------------------------------------

def test_subpixel_closed_form(orc):
    rng = np.random.default_rng(9)
    n = 500
    b = rng.integers(0, 1000, n)
    a = b + rng.integers(1, 400, n)   # strictly above the minimum (smallest argmin is d=1)
    c = b + rng.integers(0, 400, n)
    S = np.stack([a, b, c], -1).astype(np.uint16)[None]
    w, ds = orc.wta(S)
    assert (w == 1).all()
    # Vertex of the parabola through (0, a), (1, b), (2, c).
    vertex = 1.0 + (a - c) / (2.0 * (a - 2 * b + c))
    assert np.allclose(ds[0], vertex, rtol=0, atol=1e-6)
    assert (np.abs(ds - 1.0) <= 0.5).all()
    sym = np.array([[[50, 20, 50, 90]]], np.uint16)
    assert orc.wta(sym)[1][0, 0] == 1.0
    # Ties go to the smallest d; no refinement at the range ends.
    tie = np.array([[[9, 3, 3, 8], [1, 5, 6, 7], [9, 9, 9, 0]]], np.uint16)
    w, ds = orc.wta(tie)
    assert list(w[0]) == [1, 0, 3] and ds[0, 1] == 0.0 and ds[0, 2] == 3.0


# --- whole disparity maps -----------------------------------------------------------------

def chebyshev_far(mask, r):
    """True where no True pixel of mask lies within Chebyshev distance < r."""
    H, W = mask.shape
    pad = np.pad(mask, r - 1, constant_values=False)
    near = np.zeros((H, W), bool)
    for dy in range(2 * r - 1):
        for dx in range(2 * r - 1):
            near |= pad[dy:dy + H, dx:dx + W]
    return ~near


def clean_interior(p, margin=5):
    H, W = p.left.shape
    border = np.zeros((H, W), bool)
    border[0, :] = border[-1, :] = True
    border[:, 0] = border[:, -1] = True
    bad = p.disc | p.occluded | border
    ok = chebyshev_far(bad, margin)
    xs = np.arange(W)[None, :]
    ok &= (xs - p.gt_disp.astype(np.int64)) >= margin
    return ok


@pytest.mark.parametrize("idx", [0, 1, 2, 3])
def test_exact_recovery_piecewise_constant(orc, idx):
    p = synth.pair_rectangles(idx)
    w, disp, valid = orc.disparity(p.left, p.right, 32, 10, 120)
    ok = clean_interior(p)
    assert ok.sum() > 0.5 * ok.size
    assert np.array_equal(w[ok], p.gt_disp[ok].astype(np.int16))
    assert valid[ok].all()
    # Integer ground truth, interior minimum: the parabola vertex stays within half a pixel.
    assert (np.abs(disp[ok] - p.gt_disp[ok]) <= 0.5).all()


def test_lr_constant_disparity(orc):
    for d in (0, 5, 17):
        p = synth.constant_pair(d, 24, 80)
        w, disp, valid = orc.disparity(p.left, p.right, 32, 10, 120)
        sl = slice(d + 4, 80 - 4)
        assert (w[:, sl] == d).all()
        assert valid[:, sl].all()
        # Pixels with x - d* < 0 can never pass the check.
        xs = np.arange(80)[None, :]
        assert not valid[(xs - w) < 0].any()
        assert (disp[valid == 0] == -1.0).all()


def test_lr_check_rules(orc):
    wl = np.array([[0, 1, 3, 2, 4, 6]], np.int16)
    wr = np.array([[0, 2, 2, 4, 9, 9]], np.int16)
    ds = wl.astype(np.float32) + 0.25
    valid, disp = orc.lr_check(wl, wr, ds, 1)
    # x=0: q=0, |0-0|=0 ok; x=1: q=0, |1-0|=1 ok; x=2: q=-1 invalid; x=3: q=1, |2-2| ok;
    # x=4: q=0, |4-0|=4 bad; x=5: q=-1 invalid.
    assert list(valid[0]) == [1, 1, 0, 1, 0, 0]
    assert list(disp[0]) == [0.25, 1.25, -1.0, 2.25, -1.0, -1.0]


# --- combination and triangulation ----------------------------------------------------------

def test_bilinear_affine_field(orc):
    rng = np.random.default_rng(10)
    H, W = 30, 40
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    al, be, ga = 20.0, 0.3, -0.2
    d1 = (al + be * xs + ga * ys).astype(np.float32)
    d0 = np.full((H, W), 10.0, np.float32)
    v = np.ones((H, W), np.uint8)
    flow = rng.uniform(-3, 3, (H, W, 2)).astype(np.float32)
    sf4, valid = orc.combine(d0, v, d1, v, flow)
    xp = xs + flow[..., 0].astype(np.float64)
    yp = ys + flow[..., 1].astype(np.float64)
    inside = (xp >= 0) & (xp <= W - 1) & (yp >= 0) & (yp <= H - 1)
    assert np.array_equal(valid.astype(bool), inside)
    exp = al + be * xp + ga * yp
    assert np.allclose(sf4[..., 3][inside], exp[inside], atol=1e-4, rtol=0)
    assert np.array_equal(sf4[..., 0][inside], flow[..., 0][inside])
    assert np.isnan(sf4[~inside]).all()


def test_bilinear_integer_flow_and_identity(orc):
    rng = np.random.default_rng(11)
    H, W = 12, 15
    d1 = rng.uniform(0, 50, (H, W)).astype(np.float32)
    v = np.ones((H, W), np.uint8)
    flow = rng.integers(-2, 3, (H, W, 2)).astype(np.float32)
    sf4, valid = orc.combine(d1, v, d1, v, flow)
    ys, xs = np.mgrid[0:H, 0:W]
    xt, yt = xs + flow[..., 0].astype(int), ys + flow[..., 1].astype(int)
    ins = (xt >= 0) & (xt < W) & (yt >= 0) & (yt < H)
    assert np.array_equal(sf4[..., 3][ins], d1[yt[ins], xt[ins]])
    sf4, valid = orc.combine(d1, v, d1, v, np.zeros((H, W, 2), np.float32))
    assert valid.all() and np.array_equal(sf4[..., 3], d1) and np.array_equal(sf4[..., 2], d1)


def test_combine_validity_rules(orc):
    H, W = 6, 8
    d = np.full((H, W), 7.0, np.float32)
    v1 = np.ones((H, W), np.uint8)
    v1[2, 3] = 0
    v0 = np.ones((H, W), np.uint8)
    v0[0, 0] = 0
    flow = np.zeros((H, W, 2), np.float32)
    flow[1, 1] = (1.5, 0.5)          # taps (2,1),(3,1),(2,2),(3,2): (3,2)=x3,y2 invalid -> undefined
    flow[4, 4] = (3.0, 1.0)          # lands on (7,5) exactly: last column and row, +1 taps clamp
    flow[3, 3] = (np.nan, 0.0)       # NaN flow -> undefined
    flow[5, 0] = (-0.001, 0.0)       # just outside
    sf4, valid = orc.combine(d, v0, d, v1, flow)
    assert valid[0, 0] == 0
    assert valid[1, 1] == 0
    assert valid[4, 4] == 1 and sf4[4, 4, 3] == 7.0
    assert valid[3, 3] == 0 and valid[5, 0] == 0
    # Zero flow at (2, 2): taps (2,2), (3,2), (2,3), (3,3); (3,2) is invalid even though its
    # weight is zero, so S is undefined under the all-four-taps reading.
    assert valid[2, 2] == 0
    assert valid[0, 1] == 1


def test_triangulation_closed_forms(orc):
    H, W = 4, 5
    f, B = 721.5, 0.54
    cx, cy = (W - 1) / 2, (H - 1) / 2
    fB = np.float32(np.float32(f) * np.float32(B))
    assert abs(float(fB) - 389.61) < 1e-4
    d0 = np.ones((H, W), np.float32)
    v = np.ones((H, W), np.uint8)
    sf4, valid, xyz0, motion = orc.combine(d0, v, d0, v, np.zeros((H, W, 2), np.float32), (f, B, cx, cy))
    assert (valid == 3).all()
    assert np.all(xyz0[..., 2] == fB)
    assert np.all(motion == 0.0)
    # Half the disparity at t1: depth doubles.
    d1 = np.full((H, W), 0.5, np.float32)
    sf4, valid, xyz0, motion = orc.combine(d0, v, d1, v, np.zeros((H, W, 2), np.float32), (f, B, cx, cy))
    assert np.allclose(motion[..., 2], xyz0[..., 2], rtol=1e-6)
    # X of the principal point is 0; X grows linearly with x at fixed depth.
    assert np.all(xyz0[1, 2, 0] == 0.0) if W % 2 == 1 else True
    assert np.allclose(xyz0[0, :, 0], (np.arange(W) - cx) * fB / f, rtol=1e-6)
    # Non-positive disparity: no 3-D point, S still defined.
    d0z = d0.copy()
    d0z[0, 0] = 0.0
    sf4, valid, xyz0, motion = orc.combine(d0z, v, d0, v, np.zeros((H, W, 2), np.float32), (f, B, cx, cy))
    assert valid[0, 0] == 1 and np.isnan(xyz0[0, 0]).all() and np.isnan(motion[0, 0]).all()


# --- sampled oracle (for images too large for the full oracle) ----------------------------

def test_aggregate_at_equals_full_aggregation(orc):
    rng = np.random.default_rng(31)
    H, W, D = 9, 23, 8
    L = rng.integers(0, 256, (H, W)).astype(np.uint8)
    R = rng.integers(0, 256, (H, W)).astype(np.uint8)
    cl, cr = orc.census(L), orc.census(R)
    for right in (False, True):
        base, match = (cr, cl) if right else (cl, cr)
        S = orc.aggregate(orc.cost(base, match, D, right), 10, 40)
        for y in range(H):
            for x in range(W):
                assert np.array_equal(orc.aggregate_at(base, match, D, right, 10, 40, x, y), S[y, x]), (x, y)
    for mask in (0x01, 0x22, 0xC0):
        S = orc.aggregate(orc.cost(cl, cr, D, False), 5, 30, mask)
        assert np.array_equal(orc.aggregate_at(cl, cr, D, False, 5, 30, 11, 4, mask), S[4, 11])


def test_disparity_at_equals_full_map(orc):
    p = synth.pair_rectangles(2)
    w, disp, valid = orc.disparity(p.left, p.right, 32)
    rng = np.random.default_rng(32)
    ys = rng.integers(0, 96, 60)
    xs = rng.integers(0, 320, 60)
    ws, ds, vs = orc.disparity_at(p.left, p.right, 32, xs, ys)
    assert np.array_equal(ws, w[ys, xs]) and np.array_equal(vs, valid[ys, xs])
    assert np.array_equal(ds, disp[ys, xs])
