"""Parity of every C-ABI stage with the CPU oracle on the same seeded inputs:
bit-exact for census, costs, aggregated costs, WTA disparities and masks;
|gpu - oracle| <= 1e-5 * max(|oracle|, scale) for FP32 outputs."""
import ctypes as ct
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, synth, _lib  # noqa: E402

from gpu_util import DEV, assert_close_rel, dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# --- census ---------------------------------------------------------------------------

@pytest.mark.parametrize("H,W", [(96, 320), (1, 1), (5, 8), (7, 9), (13, 70), (64, 65), (375, 1242)])
def test_census(orc, H, W):
    say("census", H, W)
    rng = np.random.default_rng(H * 1000 + W)
    img = rng.integers(0, 256, (H, W)).astype(np.uint8)
    got = host(api.census(dev(img)), np.uint64)
    assert np.array_equal(got, orc.census(img))


@pytest.mark.parametrize("H,W,pitch,offset", [(40, 1024, 1024, 0), (17, 900, 903, 1), (9, 1300, 1301, 3),
                                               (12, 1242, 1250, 2)])
def test_census_interior_tiles(orc, H, W, pitch, offset):
    """Images wide enough for tiles away from both edges (dword fill from any base and pitch alignment)."""
    say("census interior", H, W, pitch, offset)
    rng = np.random.default_rng(W + offset)
    buf = rng.integers(0, 256, H * pitch + 8).astype(np.uint8)
    t = dev(buf)
    out = torch.empty((H, W), dtype=torch.int64, device=DEV)
    _lib.check(_lib.lib().sf_census(ct.c_void_p(t.data_ptr() + offset), H, W, pitch,
                                    ct.c_void_p(out.data_ptr()),
                                    ct.c_void_p(torch.cuda.current_stream().cuda_stream)))
    img = np.ascontiguousarray(buf[offset:offset + H * pitch].reshape(H, pitch)[:, :W])
    assert np.array_equal(host(out, np.uint64), orc.census(img))


def test_census_pitch(orc):
    say("census pitch")
    rng = np.random.default_rng(5)
    H, W, pitch = 19, 41, 64
    wide = rng.integers(0, 256, (H, pitch)).astype(np.uint8)
    t = dev(wide)
    out = torch.empty((H, W), dtype=torch.int64, device=DEV)
    _lib.check(_lib.lib().sf_census(ct.c_void_p(t.data_ptr()), H, W, pitch, ct.c_void_p(out.data_ptr()),
                                    ct.c_void_p(torch.cuda.current_stream().cuda_stream)))
    assert np.array_equal(host(out, np.uint64), orc.census(np.ascontiguousarray(wide[:, :W])))


# --- cost -----------------------------------------------------------------------------

@pytest.mark.parametrize("D", [1, 3, 5, 16, 32, 48, 96, 100, 128, 256])
@pytest.mark.parametrize("right", [False, True])
def test_cost(orc, D, right):
    say("cost", D, right)
    p = synth.pair_rectangles(1)
    cl, cr = orc.census(p.left), orc.census(p.right)
    base, match = (cr, cl) if right else (cl, cr)
    got = host(api.cost(dev(base), dev(match), D, right))
    assert np.array_equal(got, orc.cost(base, match, D, right))


@pytest.mark.parametrize("offset", [1, 4, 8])
def test_cost_unaligned_output(orc, offset):
    """Output pointers that are not 16-byte aligned take the narrower stores."""
    say("cost unaligned", offset)
    p = synth.pair_rectangles(2)
    cl, cr = orc.census(p.left), orc.census(p.right)
    H, W, D = p.left.shape[0], p.left.shape[1], 32
    buf = torch.full((H * W * D + 16,), 255, dtype=torch.uint8, device=DEV)
    tl, tr = dev(cl), dev(cr)
    _lib.check(_lib.lib().sf_cost(ct.c_void_p(tl.data_ptr()), ct.c_void_p(tr.data_ptr()), H, W, D, 0,
                                  ct.c_void_p(buf.data_ptr() + offset),
                                  ct.c_void_p(torch.cuda.current_stream().cuda_stream)))
    got = host(buf)
    assert np.array_equal(got[offset:offset + H * W * D].reshape(H, W, D), orc.cost(cl, cr, D, False))
    assert (got[:offset] == 255).all() and (got[offset + H * W * D:] == 255).all()


# --- aggregation ------------------------------------------------------------------------

def rand_cost(rng, H, W, D):
    return rng.integers(0, 63, (H, W, D)).astype(np.uint8)


@pytest.mark.parametrize("D", [32, 64, 96, 128, 160, 192, 224, 256])
@pytest.mark.parametrize("mode", [1, 2])
def test_aggregate_every_D(orc, D, mode):
    say("aggregate D", D, "mode", mode)
    rng = np.random.default_rng(D + mode)
    H, W = 21, 37
    C = rand_cost(rng, H, W, D)
    api.sgm_set_epilogue(mode)
    try:
        got = host(api.sgm_aggregate(dev(C), 10, 120), np.uint16)
    finally:
        api.sgm_set_epilogue(0)
    assert np.array_equal(got, orc.aggregate(C, 10, 120))


@pytest.mark.parametrize("H,W", [(1, 1), (1, 40), (40, 1), (2, 3), (33, 17), (17, 70)])
def test_aggregate_shapes(orc, H, W):
    say("aggregate shape", H, W)
    rng = np.random.default_rng(H * 7 + W)
    C = rand_cost(rng, H, W, 64)
    got = host(api.sgm_aggregate(dev(C), 10, 120), np.uint16)
    assert np.array_equal(got, orc.aggregate(C, 10, 120))


@pytest.mark.parametrize("P1,P2", [(0, 0), (10, 120), (1, 193), (30, 30), (10, 194), (50, 2000)])
def test_aggregate_penalties(orc, P1, P2):
    say("aggregate penalties", P1, P2)
    rng = np.random.default_rng(P1 * 31 + P2)
    C = rand_cost(rng, 19, 29, 32)
    got = host(api.sgm_aggregate(dev(C), P1, P2), np.uint16)
    assert np.array_equal(got, orc.aggregate(C, P1, P2))


@pytest.mark.parametrize("mask", [1, 2, 4, 8, 16, 32, 64, 128, 0x0F, 0xF0, 0x55, 0xFF])
def test_aggregate_path_masks(orc, mask):
    say("aggregate mask", mask)
    rng = np.random.default_rng(mask)
    C = rand_cost(rng, 23, 31, 32)
    got = host(api.sgm_aggregate(dev(C), 10, 120, mask), np.uint16)
    assert np.array_equal(got, orc.aggregate(C, 10, 120, mask))


def test_aggregate_c1_pair(orc):
    say("aggregate 320x96")
    p = synth.pair_rectangles(0)
    C = orc.cost(orc.census(p.left), orc.census(p.right), 32, False)
    got = host(api.sgm_aggregate(dev(C), 10, 120), np.uint16)
    assert np.array_equal(got, orc.aggregate(C, 10, 120))


# --- WTA / LR / features ------------------------------------------------------------------

@pytest.mark.parametrize("D", [1, 2, 3, 32, 100, 128, 256])
def test_wta_lr_features(orc, D):
    say("wta D", D)
    rng = np.random.default_rng(D)
    H, W = 17, 45
    # Small value range so ties are frequent.
    Sl = rng.integers(0, 40, (H, W, D)).astype(np.uint16)
    Sr = rng.integers(0, 40, (H, W, D)).astype(np.uint16)
    img = rng.integers(0, 256, (H, W)).astype(np.uint8)
    out = api.wta_lr(dev(Sl), dev(Sr), dev(img), P2=120, lr_tol=1, want_feat=True)
    wl, dsl = orc.wta(Sl)
    wr, _ = orc.wta(Sr)
    valid, disp = orc.lr_check(wl, wr, dsl, 1)
    assert np.array_equal(host(out["wta_left"]), wl)
    assert np.array_equal(host(out["wta_right"]), wr)
    assert np.array_equal(host(out["valid"]), valid)
    assert_close_rel(host(out["disp"]), disp, 1.0, what="disp")
    feat = orc.features(img, Sl, wl, 120)
    assert_close_rel(host(out["feat"]), feat, 1e-3, what="feat")
    # No right view: every pixel kept with its sub-pixel disparity.
    out2 = api.wta_lr(dev(Sl), None, None, lr_tol=1)
    v2, d2 = orc.no_check(dsl)
    assert np.array_equal(host(out2["valid"]), v2)
    assert_close_rel(host(out2["disp"]), d2, 1.0, what="disp no check")


@pytest.mark.parametrize("tol", [0, 1, 3])
def test_lr_tolerance(orc, tol):
    say("lr tol", tol)
    p = synth.pair_rectangles(2)
    cl, cr = orc.census(p.left), orc.census(p.right)
    Sl = orc.aggregate(orc.cost(cl, cr, 32, False), 10, 120)
    Sr = orc.aggregate(orc.cost(cr, cl, 32, True), 10, 120)
    out = api.wta_lr(dev(Sl), dev(Sr), lr_tol=tol)
    wl, dsl = orc.wta(Sl)
    wr, _ = orc.wta(Sr)
    valid, disp = orc.lr_check(wl, wr, dsl, tol)
    assert np.array_equal(host(out["valid"]), valid)
    assert_close_rel(host(out["disp"]), disp, 1.0)


# --- combination ------------------------------------------------------------------------------

@pytest.mark.parametrize("H,W", [(1, 1), (9, 14), (96, 320), (375, 1242)])
def test_combine(orc, H, W):
    say("combine", H, W)
    rng = np.random.default_rng(H + W)
    d0 = rng.uniform(-1, 80, (H, W)).astype(np.float32)
    d1 = rng.uniform(-1, 80, (H, W)).astype(np.float32)
    v0 = (rng.uniform(size=(H, W)) < 0.85).astype(np.uint8)
    v1 = (rng.uniform(size=(H, W)) < 0.9).astype(np.uint8)
    flow = rng.normal(0, 0.3 * max(H, W), (H, W, 2)).astype(np.float32)
    k = rng.uniform(size=(H, W)) < 0.1
    flow[k] = np.round(flow[k])                       # integer flows
    flow[rng.uniform(size=(H, W)) < 0.02] = np.nan    # NaN flows
    # Flows that land exactly on the last column / row (the +1 taps clamp there).
    ys, xs = np.mgrid[0:H, 0:W]
    e = rng.uniform(size=(H, W)) < 0.05
    flow[e, 0] = (W - 1 - xs[e]).astype(np.float32)
    flow[e, 1] = (H - 1 - ys[e]).astype(np.float32)
    cam = (721.5, 0.54, (W - 1) / 2, (H - 1) / 2)
    out = api.combine(dev(d0), dev(v0), dev(d1), dev(v1), dev(flow), cam)
    sf4, valid, xyz0, motion = orc.combine(d0, v0, d1, v1, flow, cam)
    assert np.array_equal(host(out["valid"]), valid)
    g = host(out["sf4"])
    assert_close_rel(g, sf4, 1.0, what="sf4")
    P0 = np.linalg.norm(np.nan_to_num(xyz0), axis=-1, keepdims=True)
    assert_close_rel(host(out["xyz0"]), xyz0, np.maximum(P0, 1e-30), what="xyz0")
    P1 = np.linalg.norm(np.nan_to_num(xyz0 + motion), axis=-1, keepdims=True)
    assert_close_rel(host(out["motion"]), motion, np.maximum(np.maximum(P0, P1), 1e-30), what="motion")
    # Without a camera only S and bit 0 are produced.
    out2 = api.combine(dev(d0), dev(v0), dev(d1), dev(v1), dev(flow))
    sf4b, validb = orc.combine(d0, v0, d1, v1, flow)
    assert np.array_equal(host(out2["valid"]), validb)
    assert_close_rel(host(out2["sf4"]), sf4b, 1.0)
