"""CPU checks of the network error analysis used by the GPU tests: its float64
evaluation reproduces the oracle exactly where every sum is exact, the exactness
condition holds for the dyadic test inputs, and its per-element bounds cover a
second FP32 evaluation that sums in another order."""
import numpy as np
import pytest

import lrnet_bounds as lb

NP = 5377


def grads_from_eval(ev):
    out = []
    for l in range(4):
        out += [lb.wgrad(ev["gz"][l], ev["a"][l]).reshape(-1), ev["gz"][l].sum(axis=(0, 2, 3))]
    return np.concatenate(out).astype(np.float32)


@pytest.mark.parametrize("B,H,W", [(1, 8, 8), (2, 12, 16), (2, 19, 45), (1, 33, 70)])
def test_evaluation_matches_oracle_on_exact_cases(orc, B, H, W):
    feat, prm, dz4 = lb.dyadic_case(100 * B + H, B, H, W)
    assert np.count_nonzero(dz4) >= B
    ev = lb.evaluate(feat, prm, dz4)
    _, logits, _ = orc.lrnet(feat, prm)
    assert np.array_equal(ev["z"][3][:, 0].astype(np.float32), logits)
    assert np.array_equal(grads_from_eval(ev), orc.lrnet_backward(feat, dz4, prm))


def test_exactness_condition_rejects_wide_ranges():
    rng = np.random.default_rng(5)
    feat = rng.uniform(0, 1, (1, 12, 12, 4)).astype(np.float32)
    prm = (rng.standard_normal(NP) * 0.3).astype(np.float32)
    assert not lb.sums_exact(feat, prm)


def test_boundary_distance():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 1.0 - 2.0 ** -9, 3.0, 0.75], np.float64)
    d = lb.boundary_distance(v)
    # 1.0: the boundaries are 1 + 2^-8 above and 1 - 2^-9 below (the finer
    # spacing under a power of two); 1 + 2^-8 is a boundary itself.
    assert d[0] == 2.0 ** -9 and d[1] == 0.0
    assert d[2] == 2.0 ** -9 and d[3] == 0.0
    assert d[4] == 2.0 ** -7 and d[5] == 2.0 ** -9


def _fp32_eval(feat, prm, dz4):
    """The network in float32 with every sum in another order (taps reversed,
    numpy's own reduction order): a stand-in for a second implementation.
    Returns the logits and, with dz4, the parameter gradient."""
    f = np.asarray(feat, np.float32)
    layers = [(lb.bf16(w), b) for w, b in lb.unpack(prm)]
    a = [lb.bf16(np.transpose(f, (0, 3, 1, 2)))]
    z = []
    taps = [(ky, kx) for ky in range(3) for kx in range(3)][::-1]

    def conv32(x, w):
        B, C, H, W = x.shape
        xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
        acc = np.zeros((B, w.shape[0], H, W), np.float32)
        for ky, kx in taps:
            acc += np.einsum("oc,bchw->bohw", w[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + W]).astype(np.float32)
        return acc

    def convt32(g, w):
        B, O, H, W = g.shape
        gp = np.pad(g, ((0, 0), (0, 0), (1, 1), (1, 1)))
        acc = np.zeros((B, w.shape[1], H, W), np.float32)
        for ky, kx in taps:
            acc += np.einsum("oc,bohw->bchw", w[:, :, ky, kx], gp[:, :, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W]).astype(np.float32)
        return acc

    def wgrad32(g, x):
        B, C, H, W = x.shape
        xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
        dw = np.zeros((g.shape[1], C, 3, 3), np.float32)
        for ky, kx in taps:
            dw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", g[..., ::-1], xp[:, :, ky:ky + H, kx:kx + W][..., ::-1])
        return dw

    for l, (w, b) in enumerate(layers):
        zl = conv32(a[-1], w) + b[None, :, None, None]
        z.append(zl)
        if l < 3:
            a.append(lb.bf16(np.maximum(zl, 0)))
    if dz4 is None:
        return z[3][:, 0], None
    gz = [None, None, None, np.asarray(dz4, np.float32)[:, None]]
    for l in (3, 2, 1):
        ga = convt32(gz[l], layers[l][0])
        gz[l - 1] = lb.bf16(np.where(z[l - 1] > 0, ga, np.float32(0)))
    out = []
    for l in range(4):
        out += [wgrad32(gz[l], a[l]).reshape(-1), gz[l].sum(axis=(0, 2, 3), dtype=np.float32)]
    return z[3][:, 0], np.concatenate(out)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_bound_covers_reordered_fp32(orc, seed):
    from paper_1801_04720_amd import lrnet

    rng = np.random.default_rng(10 + seed)
    B, H, W = 2, 17, 29
    feat = rng.uniform(0, 1.5, (B, H, W, 4)).astype(np.float32)
    prm = lrnet.init_params(seed)
    prm[5376] = 0.3
    dz4 = (rng.standard_normal((B, H, W)) / (B * H * W)).astype(np.float32)
    ref = orc.lrnet_backward(feat, dz4, prm)
    ev = lb.evaluate(feat, prm, dz4)
    dz, da = lb.forward_bounds(ev)
    bound = lb.gradient_bounds(ev, dz, da, 0.0)
    _, other = _fp32_eval(feat, prm, dz4)
    err = np.abs(other.astype(np.float64) - ref)
    assert (err <= bound).all(), (err / np.maximum(bound, 1e-30)).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forward_bound_covers_reordered_fp32(orc, seed):
    from paper_1801_04720_amd import lrnet

    rng = np.random.default_rng(seed)
    B, H, W = 2, 21, 34
    feat = rng.uniform(0, 2, (B, H, W, 4)).astype(np.float32)
    prm = lrnet.init_params(seed)
    prm[5376] = 0.5
    _, ref, _ = orc.lrnet(feat, prm)
    ev = lb.evaluate(feat, prm)
    dz, _ = lb.forward_bounds(ev)
    other, _ = _fp32_eval(feat, prm, None)
    err = np.abs(other.astype(np.float64) - ref)
    assert (err <= dz[3][:, 0]).all()
    # The bound is not vacuous: well below the logits' own scale.
    assert np.median(dz[3]) < 0.2 * np.median(np.abs(ref))
