"""Whole scene-flow frames on the GPU against the CPU oracle: the fused frame
entry point (all four aggregations in one launch, slabs summed inside WTA),
its persistent variant, and the per-stage path, at a small size and at the
full 1242x375 / D=128 size."""
import ctypes as ct
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import _lib, synth  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame, PlainFrame  # noqa: E402

from gpu_util import DEV, assert_close_rel, dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_frame(orc, fr, D, cam):
    w0, d0, v0 = orc.disparity(fr.t0.left, fr.t0.right, D)
    w1, d1, v1 = orc.disparity(fr.t1.left, fr.t1.right, D)
    sf4, valid, xyz0, motion = orc.combine(d0, v0, d1, v1, fr.flow, cam)
    return dict(disp0=d0, valid0=v0, disp1=d1, valid1=v1, sf4=sf4, valid=valid, xyz0=xyz0, motion=motion)


def check_frame(got, ref):
    for k in ("valid0", "valid1", "valid"):
        assert np.array_equal(host(got[k]), ref[k]), k
    assert_close_rel(host(got["disp0"]), ref["disp0"], 1.0, what="disp0")
    assert_close_rel(host(got["disp1"]), ref["disp1"], 1.0, what="disp1")
    assert_close_rel(host(got["sf4"]), ref["sf4"], 1.0, what="sf4")
    xyz0, motion = ref["xyz0"], ref["motion"]
    P0 = np.linalg.norm(np.nan_to_num(xyz0), axis=-1, keepdims=True)
    P1 = np.linalg.norm(np.nan_to_num(xyz0 + motion), axis=-1, keepdims=True)
    assert_close_rel(host(got["xyz0"]), xyz0, np.maximum(P0, 1e-30), what="xyz0")
    assert_close_rel(host(got["motion"]), motion, np.maximum(np.maximum(P0, P1), 1e-30), what="motion")


@pytest.mark.parametrize("H,W,D,persistent", [(48, 160, 32, False), (61, 203, 64, True),
                                              (40, 97, 96, False), (29, 211, 128, False),
                                              (33, 300, 256, True)])
def test_fused_frame_small(orc, H, W, D, persistent):
    say("fused frame", H, W, D, persistent)
    fr = synth.frame_planar(synth.rng_for(8, D), H, W, D, 20.0)
    ff = FusedFrame(H, W, D, persistent=persistent, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    torch.cuda.synchronize()
    check_frame(got, oracle_frame(orc, fr, D, ff.cam))


def oracle_frame_par(orc, fr, D, cam):
    """oracle_frame with the four views in parallel threads (large frames)."""
    import oracle_maps

    m = oracle_maps.maps(orc, [(fr.t0.left, fr.t0.right), (fr.t1.left, fr.t1.right)], D)
    sf4, valid, xyz0, motion = orc.combine(m[0]["disp"], m[0]["valid"], m[1]["disp"], m[1]["valid"], fr.flow, cam)
    return dict(disp0=m[0]["disp"], valid0=m[0]["valid"], disp1=m[1]["disp"], valid1=m[1]["valid"], sf4=sf4,
                valid=valid, xyz0=xyz0, motion=motion)


# Aggregation tunings of the full-size frame: the plan default (byte costs, one
# block per task), the 6-bit packed costs the frame tuner picks for 4-view
# frames, packed with persistent blocks, and byte costs persistent in view order.
FRAME_TUNINGS = [("bytes", None), ("packed", (16, 8, 0, 0, 1)), ("packed persistent", (4, 8, 0, 8, 1)),
                 ("bytes persistent view-order", (8, 4, 1, 4, 0))]


def test_fused_frame_1242x375_vs_oracle(orc):
    """The full 1242x375 D=128 frame against the oracle, whole arrays, under each
    aggregation tuning (persistent ones run twice: their task counter must be
    back at zero)."""
    from paper_1801_04720_amd._lib import SfAggTuning

    fr = synth.frame_1242x375(0)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    ref = None
    for name, t in FRAME_TUNINGS:
        tuning = SfAggTuning(*t) if t else None
        ff = FusedFrame(375, 1242, 128, tuning=tuning, device=DEV)
        if ref is None:
            say("oracle for the 1242x375 D=128 frame")
            ref = oracle_frame_par(orc, fr, 128, ff.cam)
        for rep in range(2 if t and t[3] else 1):
            say("fused frame 1242x375 D=128 vs oracle, tuning", name, "run", rep)
            for v in ff.out.values():
                v.fill_(7)
            got = ff.run(*args)
            torch.cuda.synchronize()
            check_frame(got, ref)


def test_learned_frame_1242x375_packed_costs(orc):
    """The learned frame at full size with 6-bit packed costs (and persistent
    blocks) equals the learned frame with byte costs bit for bit, and every
    pixel its mask keeps carries the oracle's sub-pixel disparity of the left
    view (the aggregation and WTA under packed costs against the oracle)."""
    import oracle_maps
    from paper_1801_04720_amd._lib import SfAggTuning

    fr = synth.frame_1242x375(3)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with np.load(os.path.join(root, "paper_1801_04720_amd", "data", "lrnet_1242x375.npz"), allow_pickle=False) as z:
        prm = dev(z["params"].astype(np.float32))
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    say("learned frame 1242x375, byte costs")
    ref = {k: host(v).copy() for k, v in FusedFrame(375, 1242, 128, learned_params=prm, device=DEV).run(*args).items()}
    for t in [(16, 8, 0, 0, 1), (4, 8, 1, 8, 1)]:
        say("learned frame 1242x375, tuning", t)
        ff = FusedFrame(375, 1242, 128, learned_params=prm, tuning=SfAggTuning(*t), device=DEV)
        for rep in range(2 if t[3] else 1):
            got = {k: host(v).copy() for k, v in ff.run(*args).items()}
            torch.cuda.synchronize()
            for k in ref:
                assert np.array_equal(got[k], ref[k], equal_nan=True), (t, rep, k)
    say("oracle left views")
    om = oracle_maps.maps(orc, [(fr.t0.left, fr.t0.right), (fr.t1.left, fr.t1.right)], 128, left_only=True)
    xs = np.arange(1242)[None, :]
    for t, m in enumerate(om):
        v = ref["valid%d" % t].astype(bool)
        d = ref["disp%d" % t]
        assert v.mean() > 0.8
        assert np.array_equal(d[v], m["dsub"][v]), t
        assert (d[~v] == -1.0).all()
        assert not (v & ((xs - m["wta_left"]) < 0)).any()


def test_fused_equals_stagewise_and_persistent_1242x375():
    say("fused vs per-stage vs persistent, 1242x375 D=128")
    fr = synth.frame_1242x375(1)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    a = FusedFrame(375, 1242, 128, device=DEV).run(*args)
    a = {k: host(v).copy() for k, v in a.items()}
    b = FusedFrame(375, 1242, 128, persistent=True, device=DEV).run(*args)
    m0, m1, c = PlainFrame(375, 1242, 128, device=DEV).run(*args)
    torch.cuda.synchronize()
    for k in a:
        assert np.array_equal(a[k], host(b[k]), equal_nan=True), k
    assert np.array_equal(a["valid0"], host(m0["valid"]))
    assert np.array_equal(a["disp1"], host(m1["disp"]))
    for k in ("sf4", "valid", "xyz0", "motion"):
        assert np.array_equal(a[k], host(c[k]), equal_nan=True), k


@pytest.mark.parametrize("learned", [False, True])
def test_frame_images_at_odd_offsets_and_pitch(learned):
    """The four images inside wider rows (pitch W + 13) at byte offsets 1, 2, 3
    and 5 give the same frame as compact copies: the census launch stages image
    rows with aligned reads (interior tiles at this width) or byte by byte (the
    row ends), for any alignment, and every later stage reads the images (the
    learned features) with the same pitch."""
    from paper_1801_04720_amd import lrnet

    say("frame with odd image offsets and pitch, learned =", learned)
    H, W, D = 40, 800, 128
    fr = synth.frame_planar(synth.rng_for(8, 43), H, W, D, 20.0)
    imgs = [fr.t0.left, fr.t0.right, fr.t1.left, fr.t1.right]
    compact = [dev(a) for a in imgs]
    wide = []
    for a, off in zip(imgs, (1, 2, 3, 5)):
        buf = np.full((H, W + 13), 77, np.uint8)
        buf[:, off:off + W] = a
        wide.append(dev(buf)[:, off:off + W])
    assert wide[0].stride(0) == W + 13
    flow = dev(fr.flow)
    prm = dev(lrnet.init_params(3)) if learned else None
    ref = {k: host(v).copy() for k, v in FusedFrame(H, W, D, learned_params=prm, device=DEV).run(*compact, flow).items()}
    # The pitch is a C-ABI argument (the Python binding takes compact tensors).
    ff = FusedFrame(H, W, D, learned_params=prm, device=DEV)
    P = lambda t: ct.c_void_p(t.data_ptr())  # noqa: E731
    o = ff.out
    cam = ct.byref(_lib.SfCamera(*[float(c) for c in ff.cam]))
    head = [ff.plan.handle] + [P(a) for a in wide] + [W + 13, P(flow), cam]
    tail = [P(o[k]) for k in ("disp0", "valid0", "disp1", "valid1", "sf4", "valid", "xyz0", "motion")]
    tail += [P(ff.ws), ff.ws.numel(), None]
    if learned:
        _lib.check(_lib.lib().sf_frame_run_learned(*head, P(prm), *tail))
    else:
        _lib.check(_lib.lib().sf_frame_run(*head, *tail))
    torch.cuda.synchronize()
    for k in ref:
        assert np.array_equal(host(o[k]), ref[k], equal_nan=True), k


def test_fused_frame_repeatable():
    """A persistent plan run four times in a row (its task counter returns to
    zero at the end of every launch, with no clearing launch in between) equals
    the one-block-per-task plan every time."""
    say("fused persistent frame run four times")
    fr = synth.frame_planar(synth.rng_for(8, 5), 64, 200, 64, 30.0)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    ref = {k: host(v).copy() for k, v in FusedFrame(64, 200, 64, device=DEV).run(*args).items()}
    ff = FusedFrame(64, 200, 64, persistent=True, device=DEV)
    for rep in range(4):
        for v in ff.out.values():
            v.fill_(7)
        got = {k: host(v).copy() for k, v in ff.run(*args).items()}
        for k in ref:
            assert np.array_equal(got[k], ref[k], equal_nan=True), (rep, k)


@pytest.mark.parametrize("D", [64, 128])
def test_learned_frame_equals_stagewise(orc, D):
    """Learned frame == its stages called one by one through the C ABI (each stage is
    pinned against the oracle in its own tests); the plain left maps agree with the
    oracle's WTA, and the learned masks never keep a pixel with x - d* < 0."""
    from paper_1801_04720_amd import api, lrnet

    say("learned frame vs stage-by-stage, D =", D)
    H, W = 64, 200
    fr = synth.frame_planar(synth.rng_for(8, 11), H, W, D, 25.0)
    prm = dev(lrnet.init_params(5))
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    ff = FusedFrame(H, W, D, learned_params=prm, device=DEV)
    got = {k: host(v).copy() for k, v in ff.run(*args).items()}
    maps = []
    for t in range(2):
        L, R = args[2 * t], args[2 * t + 1]
        cl, cr = api.census(L), api.census(R)
        Sl = api.sgm_aggregate(api.cost(cl, cr, D, False), 10, 120)
        m = api.wta_lr(Sl, None, L, 120, 1, want_feat=True)
        logits = lrnet.forward(prm, m["feat"][None].contiguous())
        valid, disp = lrnet.mask(logits[0], m["wta_left"], m["disp"])
        maps.append((valid, disp, m["wta_left"]))
    c = api.combine(maps[0][1], maps[0][0], maps[1][1], maps[1][0], args[4], ff.cam)
    torch.cuda.synchronize()
    assert np.array_equal(got["valid0"], host(maps[0][0]))
    assert np.array_equal(got["disp1"], host(maps[1][1]))
    for k in ("sf4", "valid", "xyz0", "motion"):
        assert np.array_equal(got[k], host(c[k]), equal_nan=True), k
    w0, _ = orc.wta(orc.aggregate(orc.cost(orc.census(fr.t0.left), orc.census(fr.t0.right), D, False), 10, 120))
    assert np.array_equal(host(maps[0][2]), w0)
    xs = np.arange(W)[None, :]
    assert not (got["valid0"].astype(bool) & ((xs - w0) < 0)).any()


@pytest.mark.parametrize("D", [32, 128])
@pytest.mark.parametrize("H,W", [(1, 1), (1, 50), (50, 1), (7, 9)])
def test_fused_frame_degenerate_shapes(orc, H, W, D):
    """Frames smaller than one tile; at D = 128 with packed costs and a persistent
    launch, whose task count is then below the block count it asks for."""
    from paper_1801_04720_amd._lib import SfAggTuning

    say("fused frame degenerate", H, W, D)
    rng = np.random.default_rng(H * 100 + W)
    imgs = [rng.integers(0, 256, (H, W)).astype(np.uint8) for _ in range(4)]
    flow = rng.normal(0, 2, (H, W, 2)).astype(np.float32)

    class F:
        pass

    fr = F()
    fr.t0, fr.t1 = F(), F()
    fr.t0.left, fr.t0.right, fr.t1.left, fr.t1.right = imgs
    fr.flow = flow
    tuning = SfAggTuning(16, 8, 0, 4, 1) if D == 128 else None
    ff = FusedFrame(H, W, D, tuning=tuning, device=DEV)
    for _ in range(2):  # twice: the persistent counter must be back at zero
        got = ff.run(dev(imgs[0]), dev(imgs[1]), dev(imgs[2]), dev(imgs[3]), dev(flow))
        torch.cuda.synchronize()
        check_frame(got, oracle_frame(orc, fr, D, ff.cam))


def test_fused_frame_max_size_vs_stagewise():
    """2048x1024, D = 256 (the largest workload): fused frame == per-stage path."""
    say("fused frame 2048x1024 D=256 vs per-stage")
    fr = synth.frame_planar(synth.rng_for(5, 0), 1024, 2048, 256, 200.0)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    a = FusedFrame(1024, 2048, 256, device=DEV).run(*args)
    a = {k: host(v).copy() for k, v in a.items()}
    m0, m1, c = PlainFrame(1024, 2048, 256, device=DEV).run(*args)
    torch.cuda.synchronize()
    assert np.array_equal(a["valid0"], host(m0["valid"]))
    assert np.array_equal(a["disp0"], host(m0["disp"]))
    assert np.array_equal(a["valid1"], host(m1["valid"]))
    for k in ("sf4", "valid", "xyz0", "motion"):
        assert np.array_equal(a[k], host(c[k]), equal_nan=True), k


@pytest.mark.parametrize("idx", [0, 1, 2, 3])
def test_gpu_exact_recovery_piecewise_constant(idx):
    """On the 320x96 D=32 piecewise-constant pairs the GPU path recovers the ground
    truth on the clean interior (the property the oracle is pinned to)."""
    from test_oracle_sgm import clean_interior
    from paper_1801_04720_amd import api

    say("gpu exact recovery", idx)
    p = synth.pair_rectangles(idx)
    L, R = dev(p.left), dev(p.right)
    cl, cr = api.census(L), api.census(R)
    Sr = api.sgm_aggregate(api.cost(cr, cl, 32, True), 10, 120)
    Sl = api.sgm_aggregate(api.cost(cl, cr, 32, False), 10, 120)
    out = api.wta_lr(Sl, Sr, None, 120, 1)
    ok = clean_interior(p)
    assert np.array_equal(host(out["wta_left"])[ok], p.gt_disp[ok].astype(np.int16))
    assert host(out["valid"])[ok].all()


def test_learned_frame_network_vs_oracle_1242x375(orc):
    """Full-size learned frame: features and logits of the t0 map against the
    oracle's (features bit-exact; every logit within its own propagated error
    bound, lrnet_bounds; the masks agree wherever the oracle's logit is farther
    from zero than that bound)."""
    import lrnet_bounds as lb

    from paper_1801_04720_amd import api, lrnet

    say("learned network vs oracle at 1242x375")
    fr = synth.frame_1242x375(2)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with np.load(os.path.join(root, "paper_1801_04720_amd", "data", "lrnet_1242x375.npz"), allow_pickle=False) as z:
        prm = z["params"].astype(np.float32)
    L, R = dev(fr.t0.left), dev(fr.t0.right)
    cl, cr = api.census(L), api.census(R)
    Sl = api.sgm_aggregate(api.cost(cl, cr, 128, False), 10, 120)
    m = api.wta_lr(Sl, None, L, 120, 1, want_feat=True)
    logits = host(lrnet.forward(dev(prm), m["feat"][None].contiguous()))[0]
    S = orc.aggregate(orc.cost(orc.census(fr.t0.left), orc.census(fr.t0.right), 128, False), 10, 120)
    w, _ = orc.wta(S)
    feat = orc.features(fr.t0.left, S, w, 120)
    assert np.array_equal(host(m["feat"]), feat)
    _, ref, _ = orc.lrnet(feat, prm)
    ref = ref[0]
    dz, _ = lb.forward_bounds(lb.evaluate(feat, prm))
    bound = dz[3][0, 0]
    err = np.abs(logits.astype(np.float64) - ref)
    bad = err > bound
    assert not bad.any(), f"{bad.sum()} logits beyond their bound, worst ratio {(err / bound).max()}"
    far = np.abs(ref) > bound
    say(f"  mask decided by the bound on {100 * far.mean():.3f} % of pixels")
    assert far.mean() > 0.99
    assert np.array_equal(logits[far] > 0, ref[far] > 0)


def test_kernel_timer_filter():
    """sf_prof_only: while a name is set, only that kernel's launches are timed."""
    import ctypes as ct

    say("kernel timer filter")
    lib = _lib.lib()
    H, W, D = 40, 96, 32
    fr = synth.frame_planar(synth.rng_for(8, 41), H, W, D, 10.0)
    args = [dev(a) for a in (fr.t0.left, fr.t0.right, fr.t1.left, fr.t1.right, fr.flow)]
    ff = FusedFrame(H, W, D, device=DEV)

    def count(name):
        tot, n = ct.c_double(0.0), ct.c_int(0)
        _lib.check(lib.sf_prof_query(name.encode(), ct.byref(tot), ct.byref(n)))
        return n.value, tot.value

    try:
        _lib.check(lib.sf_prof_enable(256))
        _lib.check(lib.sf_prof_only(b"sgm_tasks"))
        for _ in range(3):
            ff.run(*args)
        torch.cuda.synchronize()
        lib.sf_prof_disable()
        n_agg, t_agg = count("sgm_tasks")
        assert n_agg == 3 and t_agg > 0
        assert count("census")[0] == 0 and count("wta_slab_left")[0] == 0
        _lib.check(lib.sf_prof_only(None))
        _lib.check(lib.sf_prof_enable(256))
        ff.run(*args)
        torch.cuda.synchronize()
        lib.sf_prof_disable()
        assert count("sgm_tasks")[0] == 1 and count("census")[0] == 1
    finally:
        lib.sf_prof_disable()
        lib.sf_prof_only(None)
