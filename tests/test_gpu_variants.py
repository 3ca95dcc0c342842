"""SGM variants on the GPU against the CPU oracle: right map by the diagonal
search in S_L, the LR check of given maps, the 3x3 median, and whole frames
using them (fused entry point and per-stage path)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, synth  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame, PlainFrame  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402
from test_gpu_frame import check_frame  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("H,W,D", [(1, 1, 1), (3, 5, 8), (7, 40, 5), (9, 70, 32), (5, 300, 100),
                                   (4, 200, 128), (3, 300, 256)])
def test_wta_right_diag(orc, H, W, D):
    say("wta_right_diag", H, W, D)
    rng = np.random.default_rng(H * 1000 + W + D)
    S = rng.integers(0, 1457, (H, W, D)).astype(np.uint16)
    S[rng.random((H, W, D)) < 0.3] = 700  # ties
    got = host(api.wta_right_diag(dev(S)))
    assert np.array_equal(got, orc.wta_right_diag(S))


@pytest.mark.parametrize("tol", [0, 1, 3])
def test_lr_check(orc, tol):
    say("lr_check", tol)
    rng = np.random.default_rng(70 + tol)
    H, W, D = 23, 91, 40
    wl = rng.integers(0, D, (H, W)).astype(np.int16)
    wr = np.clip(np.roll(wl, -3, axis=1) + rng.integers(-2, 3, (H, W)), 0, D - 1).astype(np.int16)
    ds = (wl + rng.uniform(-0.5, 0.5, (H, W))).astype(np.float32)
    out = api.lr_check(dev(wl), dev(wr), dev(ds), tol)
    ev, ed = orc.lr_check(wl, wr, ds, tol)
    assert np.array_equal(host(out["valid"]), ev)
    assert np.array_equal(host(out["disp"]), ed)


@pytest.mark.parametrize("H,W", [(1, 1), (1, 7), (6, 1), (17, 33), (100, 37), (375, 1242)])
@pytest.mark.parametrize("masked", [False, True])
def test_median3x3(orc, H, W, masked):
    say("median3x3", H, W, masked)
    rng = np.random.default_rng(H * 7 + W)
    m = (rng.random((H, W)) * 128).astype(np.float32)
    m[rng.random((H, W)) < 0.25] = 3.5  # repeated values
    mask = (rng.random((H, W)) < 0.8).astype(np.uint8)
    got = host(api.median3x3(dev(m), dev(mask) if masked else None))
    exp = orc.median3x3(m)
    if masked:
        exp = np.where(mask == 1, exp, np.float32(-1.0))
    assert np.array_equal(got, exp)


def oracle_frame_ex(orc, fr, D, cam, flags):
    w0, d0, v0 = orc.disparity_ex(fr.t0.left, fr.t0.right, D, flags)
    w1, d1, v1 = orc.disparity_ex(fr.t1.left, fr.t1.right, D, flags)
    sf4, valid, xyz0, motion = orc.combine(d0, v0, d1, v1, fr.flow, cam)
    return dict(disp0=d0, valid0=v0, disp1=d1, valid1=v1, sf4=sf4, valid=valid, xyz0=xyz0, motion=motion)


VARIANTS = [(True, False), (False, True), (True, True)]  # (diag, median)


@pytest.mark.parametrize("diag,median", VARIANTS)
@pytest.mark.parametrize("H,W,D", [(48, 160, 32), (61, 203, 64), (33, 300, 256), (1, 50, 32), (7, 9, 32)])
def test_fused_frame_variants_small(orc, diag, median, H, W, D):
    say("fused frame variant", diag, median, H, W, D)
    fr = synth.frame_planar(synth.rng_for(8, D + H), H, W, D, 20.0)
    ff = FusedFrame(H, W, D, diag=diag, median=median, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    torch.cuda.synchronize()
    flags = (orc.DIAG if diag else 0) | (orc.MEDIAN if median else 0)
    check_frame(got, oracle_frame_ex(orc, fr, D, ff.cam, flags))


@pytest.mark.parametrize("diag,median", VARIANTS)
def test_fused_frame_variants_c2_vs_oracle(orc, diag, median):
    say("fused frame variant 1242x375 D=128", diag, median)
    fr = synth.frame_1242x375(3)
    ff = FusedFrame(375, 1242, 128, diag=diag, median=median, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    torch.cuda.synchronize()
    flags = (orc.DIAG if diag else 0) | (orc.MEDIAN if median else 0)
    check_frame(got, oracle_frame_ex(orc, fr, 128, ff.cam, flags))


@pytest.mark.parametrize("diag,median", VARIANTS)
def test_fused_equals_stagewise_variants(diag, median):
    say("fused vs per-stage variant", diag, median)
    fr = synth.frame_1242x375(4)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    a = FusedFrame(375, 1242, 128, diag=diag, median=median, persistent=True, device=DEV).run(*args)
    a = {k: host(v).copy() for k, v in a.items()}
    m0, m1, c = PlainFrame(375, 1242, 128, diag=diag, median=median, device=DEV).run(*args)
    torch.cuda.synchronize()
    assert np.array_equal(a["valid0"], host(m0["valid"]))
    assert np.array_equal(a["disp0"], host(m0["disp"]))
    assert np.array_equal(a["valid1"], host(m1["valid"]))
    assert np.array_equal(a["disp1"], host(m1["disp"]))
    for k in ("sf4", "valid", "xyz0", "motion"):
        assert np.array_equal(a[k], host(c[k]), equal_nan=True), k


def test_learned_frame_median_equals_stagewise():
    from paper_1801_04720_amd import lrnet

    say("learned frame + median vs stages")
    H, W, D = 64, 200, 64
    fr = synth.frame_planar(synth.rng_for(8, 13), H, W, D, 25.0)
    prm = dev(lrnet.init_params(7))
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    got = FusedFrame(H, W, D, learned_params=prm, median=True, device=DEV).run(*args)
    got = {k: host(v).copy() for k, v in got.items()}
    for t, key in ((0, "0"), (1, "1")):
        L, R = args[2 * t], args[2 * t + 1]
        Sl = api.sgm_aggregate(api.cost(api.census(L), api.census(R), D, False), 10, 120)
        m = api.wta_lr(Sl, None, L, 120, 1, want_feat=True)
        logits = lrnet.forward(prm, m["feat"][None].contiguous())
        valid, _ = lrnet.mask(logits[0], m["wta_left"], m["disp"])
        disp = api.median3x3(m["disp"], valid)
        torch.cuda.synchronize()
        assert np.array_equal(got["valid" + key], host(valid))
        assert np.array_equal(got["disp" + key], host(disp))


def test_diag_right_map_matches_right_pass_without_smoothing(orc):
    """P1 = P2 = 0 on census costs: the diagonal search in S_L equals the right
    view's own WTA wherever q + d stays inside the image for every d."""
    say("diag == right pass at P1 = P2 = 0")
    p = synth.pair_rectangles(2)
    D = 32
    L, R = dev(p.left), dev(p.right)
    cl, cr = api.census(L), api.census(R)
    Sl = api.sgm_aggregate(api.cost(cl, cr, D, False), 0, 0)
    Sr = api.sgm_aggregate(api.cost(cr, cl, D, True), 0, 0)
    wr = host(api.wta_lr(Sr, None, None, 0, 1)["wta_left"])
    wd = host(api.wta_right_diag(Sl))
    W = p.left.shape[1]
    assert np.array_equal(wd[:, :W - D + 1], wr[:, :W - D + 1])


# --- intensity-adaptive P2 ---------------------------------------------------------------------

def adaptive_image(rng, H, W, pitch):
    # Flat patches (g = 0), unit steps and strong edges.
    base = rng.choice(np.array([0, 1, 3, 40, 200], np.int64), (H // 3 + 1, W // 3 + 1))
    img = np.kron(base, np.ones((3, 3), np.int64))[:H, :W]
    img = (img + rng.integers(0, 2, (H, W))) % 256
    wide = np.zeros((H, pitch), np.uint8)
    wide[:, :W] = img
    wide[:, W:] = 255
    return wide


@pytest.mark.parametrize("H,W,D", [(1, 1, 32), (5, 37, 32), (21, 37, 64), (9, 70, 128), (6, 45, 256)])
@pytest.mark.parametrize("P1,P2", [(10, 120), (7, 40), (5, 300)])
def test_aggregate_adaptive_vs_oracle(orc, H, W, D, P1, P2):
    say("aggregate adaptive", H, W, D, P1, P2)
    rng = np.random.default_rng(H * 31 + W + D + P2)
    C = rng.integers(0, 63, (H, W, D)).astype(np.uint8)
    wide = adaptive_image(rng, H, W, W + 5)
    got = host(api.sgm_aggregate_adaptive(dev(C), dev(wide), P1, P2), np.uint16)
    assert np.array_equal(got, orc.aggregate_adaptive(C, np.ascontiguousarray(wide[:, :W]), P1, P2))


def test_aggregate_adaptive_pitch_and_masks(orc):
    import ctypes as ct

    from paper_1801_04720_amd import _lib

    say("aggregate adaptive pitch / masks")
    rng = np.random.default_rng(91)
    H, W, D, pitch = 23, 41, 64, 64
    C = rng.integers(0, 63, (H, W, D)).astype(np.uint8)
    wide = adaptive_image(rng, H, W, pitch)
    img_t = dev(wide)  # [H][pitch]; the entry point reads only the first W bytes of each row
    for mask in (0x01, 0x0C, 0x30, 0xC0, 0xFF):
        S = torch.empty((H, W, D), dtype=torch.int16, device=DEV)
        ws = torch.empty(api.sgm_workspace_bytes(H, W, D), dtype=torch.uint8, device=DEV)
        Ct = dev(C)
        _lib.check(_lib.lib().sf_sgm_aggregate_adaptive(
            ct.c_void_p(Ct.data_ptr()), ct.c_void_p(img_t.data_ptr()), pitch, H, W, D, 10, 120, mask,
            ct.c_void_p(S.data_ptr()), ct.c_void_p(ws.data_ptr()), ws.numel(),
            ct.c_void_p(torch.cuda.current_stream().cuda_stream)))
        exp = orc.aggregate_adaptive(C, np.ascontiguousarray(wide[:, :W]), 10, 120, mask)
        assert np.array_equal(host(S, np.uint16), exp), mask


AVARIANTS = [(False, False), (True, False), (False, True)]  # (diag, median) with adaptive P2


@pytest.mark.parametrize("diag,median", AVARIANTS)
@pytest.mark.parametrize("H,W,D", [(48, 160, 32), (33, 300, 256)])
def test_fused_frame_adaptive_small(orc, diag, median, H, W, D):
    say("fused frame adaptive", diag, median, H, W, D)
    fr = synth.frame_planar(synth.rng_for(8, D + 2 * H), H, W, D, 20.0)
    ff = FusedFrame(H, W, D, diag=diag, median=median, adaptive_p2=True, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    torch.cuda.synchronize()
    flags = orc.ADAPTIVE | (orc.DIAG if diag else 0) | (orc.MEDIAN if median else 0)
    check_frame(got, oracle_frame_ex(orc, fr, D, ff.cam, flags))


def test_fused_frame_adaptive_c2_vs_oracle(orc):
    say("fused frame adaptive 1242x375 D=128")
    fr = synth.frame_1242x375(5)
    ff = FusedFrame(375, 1242, 128, adaptive_p2=True, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    torch.cuda.synchronize()
    check_frame(got, oracle_frame_ex(orc, fr, 128, ff.cam, orc.ADAPTIVE))


@pytest.mark.parametrize("diag", [False, True])
def test_fused_equals_stagewise_adaptive(diag):
    say("fused vs per-stage adaptive", diag)
    fr = synth.frame_1242x375(6)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    a = FusedFrame(375, 1242, 128, diag=diag, adaptive_p2=True, device=DEV).run(*args)
    a = {k: host(v).copy() for k, v in a.items()}
    m0, m1, c = PlainFrame(375, 1242, 128, diag=diag, adaptive_p2=True, device=DEV).run(*args)
    torch.cuda.synchronize()
    assert np.array_equal(a["valid0"], host(m0["valid"]))
    assert np.array_equal(a["disp1"], host(m1["disp"]))
    for k in ("sf4", "valid", "xyz0", "motion"):
        assert np.array_equal(a[k], host(c[k]), equal_nan=True), k


def test_learned_frame_adaptive_equals_stagewise():
    from paper_1801_04720_amd import lrnet

    say("learned frame adaptive vs stages")
    H, W, D = 64, 200, 64
    fr = synth.frame_planar(synth.rng_for(8, 17), H, W, D, 25.0)
    prm = dev(lrnet.init_params(9))
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    got = FusedFrame(H, W, D, learned_params=prm, adaptive_p2=True, device=DEV).run(*args)
    got = {k: host(v).copy() for k, v in got.items()}
    for t, key in ((0, "0"), (1, "1")):
        L, R = args[2 * t], args[2 * t + 1]
        Sl = api.sgm_aggregate_adaptive(api.cost(api.census(L), api.census(R), D, False), L, 10, 120)
        m = api.wta_lr(Sl, None, L, 120, 1, want_feat=True)
        logits = lrnet.forward(prm, m["feat"][None].contiguous())
        valid, disp = lrnet.mask(logits[0], m["wta_left"], m["disp"])
        torch.cuda.synchronize()
        assert np.array_equal(got["valid" + key], host(valid))
        assert np.array_equal(got["disp" + key], host(disp))


def steps_image(H, W):
    """Intensities whose horizontal and vertical steps take every value 1..255."""
    x = np.arange(W, dtype=np.int64)[None, :]
    y = np.arange(H, dtype=np.int64)[:, None]
    return ((x * (x + 1) // 2 + 3 * (y * (y + 1) // 2)) % 256).astype(np.uint8)


@pytest.mark.parametrize("D", [32, 64])
def test_aggregate_adaptive_largest_p2_all_steps(orc, D):
    """P2 = 8000 (the largest the entry points accept) on an image whose path
    steps cover g = 1..255: the quotient floor(P2 / g) is exact in every
    direction (S then needs the packed 16-bit accumulation: 62 + P2 > 255)."""
    say("aggregate adaptive P2 = 8000, all steps, D =", D)
    H, W = 270, 300
    img = steps_image(H, W)
    gh = set(np.abs(np.diff(img.astype(np.int64), axis=1)).ravel().tolist())
    gv = set(np.abs(np.diff(img.astype(np.int64), axis=0)).ravel().tolist())
    assert set(range(1, 256)) <= gh and set(range(1, 256)) <= gv
    rng = np.random.default_rng(8000 + D)
    C = rng.integers(0, 63, (H, W, D)).astype(np.uint8)
    got = host(api.sgm_aggregate_adaptive(dev(C), dev(img), 10, 8000), np.uint16)
    assert np.array_equal(got, orc.aggregate_adaptive(C, img, 10, 8000))
