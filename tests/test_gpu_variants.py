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
    fr = synth.frame_c2(3)
    ff = FusedFrame(375, 1242, 128, diag=diag, median=median, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    torch.cuda.synchronize()
    flags = (orc.DIAG if diag else 0) | (orc.MEDIAN if median else 0)
    check_frame(got, oracle_frame_ex(orc, fr, 128, ff.cam, flags))


@pytest.mark.parametrize("diag,median", VARIANTS)
def test_fused_equals_stagewise_variants(diag, median):
    say("fused vs per-stage variant", diag, median)
    fr = synth.frame_c2(4)
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
    p = synth.pair_c1(2)
    D = 32
    L, R = dev(p.left), dev(p.right)
    cl, cr = api.census(L), api.census(R)
    Sl = api.sgm_aggregate(api.cost(cl, cr, D, False), 0, 0)
    Sr = api.sgm_aggregate(api.cost(cr, cl, D, True), 0, 0)
    wr = host(api.wta_lr(Sr, None, None, 0, 1)["wta_left"])
    wd = host(api.wta_right_diag(Sl))
    W = p.left.shape[1]
    assert np.array_equal(wd[:, :W - D + 1], wr[:, :W - D + 1])
