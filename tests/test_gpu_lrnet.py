"""The learned LR stand-in on the GPU against the CPU oracle: exact logits and
exact gradients on dyadic inputs (every FP32 sum exact, so summation order
cannot matter), logits and gradients on random data each within its own
propagated error bound (lrnet_bounds), bit-exact Adam, run-to-run determinism,
checkpoint/resume, and a short training run that beats the method without
the network."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, lrnet, synth  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402

NP = 5377


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dyadic_setup(rng, B, H, W):
    feat = (rng.integers(0, 17, (B, H, W, 4)) / 16.0).astype(np.float32)
    prm = (rng.integers(-4, 5, NP) / 16.0).astype(np.float32)
    for off in (576, 2896, 5216):
        prm[off:off + 16] = rng.integers(-64, 257, 16) / 256.0
    prm[5376] = rng.integers(-256, 257) / 256.0
    return feat, prm


@pytest.mark.parametrize("B,H,W", [(1, 8, 8), (2, 19, 45), (1, 33, 70)])
def test_forward_exact_on_dyadic_grid(orc, B, H, W):
    say("lrnet exact forward", B, H, W)
    rng = np.random.default_rng(B * 100 + H)
    feat, prm = dyadic_setup(rng, B, H, W)
    got = host(lrnet.forward(dev(prm), dev(feat)))
    _, ref, _ = orc.lrnet(feat, prm)
    assert np.array_equal(got, ref)


def test_forward_nonfinite_features(orc):
    """NaN and infinite features: the oracle's rules (ReLU maps a NaN to 0, a
    zero weight times an infinity is a NaN, opposite infinities sum to a NaN)
    hold on the GPU; the other logits stay exact on the dyadic grid."""
    say("lrnet forward, non-finite features")
    rng = np.random.default_rng(77)
    B, H, W = 2, 19, 45
    feat, prm = dyadic_setup(rng, B, H, W)
    feat[0, 3, 5, 1] = np.nan
    feat[0, 10, 20, 2] = np.inf
    feat[1, 15, 30, 0] = -np.inf
    feat[1, 0, 44, 3] = np.inf
    got = host(lrnet.forward(dev(prm), dev(feat)))
    _, ref, _ = orc.lrnet(feat, prm)
    assert not np.isfinite(ref).all()
    assert np.array_equal(got, ref, equal_nan=True)


def _trained():
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with np.load(os.path.join(root, "paper_1801_04720_amd", "data", "lrnet_1242x375.npz"), allow_pickle=False) as z:
        return z["params"].astype(np.float32)


@pytest.mark.parametrize("params", ["init", "trained"])
def test_forward_within_bound_random(orc, params):
    """Random inputs: every logit within its own bound of the oracle's (FP32
    sums in another order, the BF16 roundings they can change, propagated
    through the layers; lrnet_bounds)."""
    import lrnet_bounds as lb

    say("lrnet random forward, params", params)
    rng = np.random.default_rng(3)
    B, H, W = 2, 37, 53
    feat = rng.uniform(0, 2, (B, H, W, 4)).astype(np.float32)
    prm = lrnet.init_params(1) if params == "init" else _trained()
    got = host(lrnet.forward(dev(prm), dev(feat)))
    _, ref, _ = orc.lrnet(feat, prm)
    dz, _ = lb.forward_bounds(lb.evaluate(feat, prm))
    bound = dz[3][:, 0]
    err = np.abs(got.astype(np.float64) - ref)
    bad = err > bound
    assert not bad.any(), f"{bad.sum()} logits beyond their bound, worst ratio {(err / bound).max()}"


@pytest.mark.parametrize("B,H,W", [(1, 8, 8), (2, 12, 16), (2, 19, 45), (1, 33, 70)])
def test_backward_exact_on_dyadic_grid(orc, B, H, W):
    """Backward from a given dL/dz4 on inputs whose every sum is exact (checked
    on the CPU first): the GPU's gradient equals the oracle's bit for bit."""
    import lrnet_bounds as lb

    say("lrnet exact backward", B, H, W)
    feat, prm, dz4 = lb.dyadic_case(100 * B + H, B, H, W)
    got = host(lrnet.backward(dev(prm), dev(feat), dev(dz4)))
    ref = orc.lrnet_backward(feat, dz4, prm)
    assert np.count_nonzero(ref) > 100
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, f"{bad.size} gradient elements differ, first at {bad[:5]}"


@pytest.mark.parametrize("seed,params", [(0, "init"), (1, "init"), (0, "trained")])
def test_gradient_within_bound(orc, seed, params):
    """Loss gradient on random data: every one of the 5377 elements within its
    own bound of the oracle's (lrnet_bounds), and the loss within 1e-5."""
    import lrnet_bounds as lb

    say("lrnet gradient", seed, params)
    rng = np.random.default_rng(10 + seed)
    B, H, W = 2, 24, 40
    feat = rng.uniform(0, 1.5, (B, H, W, 4)).astype(np.float32)
    label = (rng.uniform(size=(B, H, W)) < 0.8).astype(np.uint8)
    if params == "init":
        prm = lrnet.init_params(seed)
        prm[5376] = 0.3
    else:
        prm = _trained()
    g, loss = lrnet.grad(dev(prm), dev(feat), dev(label))
    g = host(g)
    ref_loss, ref_logits, ref = orc.lrnet(feat, prm, label, want_grad=True)
    assert abs(float(host(loss)[0]) - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
    s = 1.0 / (1.0 + np.exp(-ref_logits.astype(np.float64)))
    dz4 = ((s - label) / label.size).astype(np.float32)
    ev = lb.evaluate(feat, prm, dz4)
    dz, da = lb.forward_bounds(ev)
    bound = lb.gradient_bounds(ev, dz, da, lb.loss_gradient_bound(ev, dz[3][:, 0]))
    err = np.abs(g.astype(np.float64) - ref)
    bad = np.flatnonzero(err > bound)
    assert bad.size == 0, f"{bad.size} elements beyond their bound, first {bad[:5]}"
    informative = (bound < 0.5 * np.abs(ref)).mean()
    say(f"  bound below half the gradient on {100 * informative:.1f} % of elements")


def test_gradient_deterministic():
    say("lrnet gradient twice")
    rng = np.random.default_rng(4)
    feat = dev(rng.uniform(0, 1, (3, 40, 70, 4)).astype(np.float32))
    label = dev((rng.uniform(size=(3, 40, 70)) < 0.7).astype(np.uint8))
    prm = dev(lrnet.init_params(2))
    g1, l1 = lrnet.grad(prm, feat, label)
    a1, b1 = host(g1).copy(), host(l1).copy()
    g2, l2 = lrnet.grad(prm, feat, label)
    assert np.array_equal(a1, host(g2)) and np.array_equal(b1, host(l2))


def test_adam_bit_exact(orc):
    say("adam")
    rng = np.random.default_rng(5)
    w = rng.standard_normal(NP).astype(np.float32)
    m = (rng.standard_normal(NP) * 0.01).astype(np.float32)
    v = (rng.uniform(0, 1e-3, NP)).astype(np.float32)
    g = rng.standard_normal(NP).astype(np.float32)
    tw, tm, tv = dev(w), dev(m), dev(v)
    lrnet.adam(tw, tm, tv, dev(g), 1e-3, 0.9, 0.999, 1e-8, 7)
    orc.adam(w, m, v, g, 1e-3, 0.9, 0.999, 1e-8, 7)
    assert np.array_equal(host(tw), w) and np.array_equal(host(tm), m) and np.array_equal(host(tv), v)


def test_mask_rule():
    say("lrnet mask")
    H, W = 3, 6
    logits = np.array([[1, -1, 2, 0.5, -0.1, 3]] * H, np.float32)
    wta = np.array([[0, 0, 3, 1, 0, 6]] * H, np.int16)
    dsub = wta.astype(np.float32) + 0.25
    valid, disp = lrnet.mask(dev(logits), dev(wta), dev(dsub))
    # x - d* >= 0 and logit > 0
    assert list(host(valid)[0]) == [1, 0, 0, 1, 0, 0]
    assert list(host(disp)[0]) == [0.25, -1.0, -1.0, 1.25, -1.0, -1.0]


def make_training_data(n_pairs, H, W, D, seed0):
    """Features and plain-LR labels of t0 pairs, produced by the GPU plain path."""
    feats, labels, wtas = [], [], []
    for i in range(n_pairs):
        p = synth.pair_planar(synth.rng_for(4, seed0 + i), H, W, D)
        L, R = dev(p.left), dev(p.right)
        cl, cr = api.census(L), api.census(R)
        Sr = api.sgm_aggregate(api.cost(cr, cl, D, True), 10, 120)
        Sl = api.sgm_aggregate(api.cost(cl, cr, D, False), 10, 120)
        out = api.wta_lr(Sl, Sr, L, 120, 1, want_feat=True)
        feats.append(out["feat"])
        labels.append(out["valid"])
        wtas.append(out["wta_left"])
    return torch.stack(feats), torch.stack(labels), torch.stack(wtas)


def test_training_beats_method_without_network():
    say("lrnet training")
    H, W, D = 96, 320, 64
    feat, label, wta = make_training_data(12, H, W, D, 0)
    vfeat, vlabel, vwta = make_training_data(3, H, W, D, 1000)
    tr = lrnet.Trainer(lrnet.init_params(0), lr=3e-3)
    losses = []
    for step in range(300):
        i = step % 3
        losses.append(float(tr.step(feat[4 * i:4 * i + 4], label[4 * i:4 * i + 4]).item()))
    assert np.mean(losses[-20:]) < 0.7 * np.mean(losses[:5])
    logits = lrnet.forward(tr.params, vfeat)
    lab = host(vlabel).astype(bool)
    xs = np.arange(W)[None, None, :]
    geo = (xs - host(vwta).astype(np.int64)) >= 0
    learned = (host(logits) > 0) & geo
    acc_none = (lab == np.ones_like(lab)).mean()
    acc_geo = (lab == geo).mean()
    acc_learned = (lab == learned).mean()
    say(f"agreement: no check {acc_none:.4f}, geometric rule {acc_geo:.4f}, learned {acc_learned:.4f}")
    assert acc_learned > acc_geo >= acc_none


def test_checkpoint_resume_bit_exact():
    say("lrnet checkpoint")
    rng = np.random.default_rng(9)
    feat = dev(rng.uniform(0, 1, (2, 32, 48, 4)).astype(np.float32))
    label = dev((rng.uniform(size=(2, 32, 48)) < 0.8).astype(np.uint8))
    a = lrnet.Trainer(lrnet.init_params(3))
    for _ in range(5):
        a.step(feat, label)
    st = a.state()
    b = lrnet.Trainer(lrnet.init_params(99))
    b.load_state(st)
    la = float(a.step(feat, label).item())
    lb = float(b.step(feat, label).item())
    assert la == lb
    assert np.array_equal(host(a.params), host(b.params))


def test_training_resume_bit_exact(tmp_path):
    """train_lrnet: a run stopped at a checkpoint and resumed from it ends with
    the same weights and moments as the uninterrupted run (the checkpoint holds
    the Adam state, the step, the seed and the crop sampler's generator state)."""
    from paper_1801_04720_amd import train_lrnet as tl

    say("lrnet training resume")
    cfg = {"t0": 2, "t1": 1, "big": 0, "val_t0": 1, "val_t1": 1, "val_big": 0, "steps": 12, "batch": 2,
           "crop": [64, 128], "lr": 3e-3, "seed": 5, "workers": 2, "ckpt": None, "ckpt_every": 0}
    full, ev = tl.train(dict(cfg), log=say)
    assert ev["val"]["t0"]["maps"] == 1 and ev["val"]["t1"]["maps"] == 1
    ck = str(tmp_path / "ck.npz")
    part, _ = tl.train(dict(cfg, ckpt=ck, ckpt_every=5), log=say, stop_after=7)
    with np.load(ck, allow_pickle=False) as z:
        assert int(z["next_step"]) == 5 and int(z["seed"]) == 5
    resumed, _ = tl.train(dict(cfg, ckpt=ck, ckpt_every=5), log=say, resume=ck)
    a, b = full.state(), resumed.state()
    assert a["step"] == b["step"] == 12
    for k in ("params", "m", "v"):
        assert np.array_equal(a[k], b[k]), k
