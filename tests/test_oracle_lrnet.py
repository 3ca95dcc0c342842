"""Pins of the learned LR stand-in's CPU oracle: finite differences, the BCE
gradient's closed form, kernel orientation by a delta input, BF16 rounding
against the format definition, Adam's first-step closed form, and the feature
definitions on hand-built cost volumes."""
import numpy as np
import pytest

from paper_1801_04720_amd import synth

NP = 5377
OFF_W1, OFF_B1 = 0, 576
OFF_W2, OFF_B2 = 592, 592 + 2304
OFF_W3, OFF_B3 = 2912, 2912 + 2304
OFF_W4, OFF_B4 = 5232, 5376


def rand_params(rng, scale=0.3):
    return (rng.standard_normal(NP) * scale).astype(np.float32)


def test_param_count(orc):
    assert orc.lib().oracle_lrnet_nparams() == NP == OFF_B4 + 1


def test_bf16_rounding_definition(orc):
    # Values on the BF16 grid are kept; halfway cases go to the even neighbour.
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    cases = {
        1.0: 1.0,
        float(one + ulp / 2): 1.0,                   # tie -> even (1.0)
        float(one + ulp + ulp / 2): float(one + 2 * ulp),  # tie -> even (1 + 2 ulp)
        float(one + ulp / 2 + np.float32(2.0 ** -20)): float(one + ulp),
        -3.0: -3.0,
        0.0: 0.0,
    }
    for x, exp in cases.items():
        assert orc.bf16(np.array([x], np.float32))[0] == np.float32(exp)
    big = np.array([np.finfo(np.float32).max], np.float32)  # past the largest finite BF16
    assert orc.bf16(np.array([3.3895314e38], np.float32))[0] == np.float32(3.3895314e38)
    assert np.isinf(orc.bf16(big)[0])
    assert np.isnan(orc.bf16(np.array([np.nan], np.float32))[0])
    rng = np.random.default_rng(1)
    x = rng.standard_normal(2000).astype(np.float32)
    r = orc.bf16(x)
    assert (r.view(np.uint32) & 0xFFFF == 0).all()
    # Nearest: no other BF16 value is closer.
    up = (r.view(np.uint32) + 0x10000).view(np.float32)
    dn = (r.view(np.uint32) - 0x10000).view(np.float32)
    err = np.abs(r.astype(np.float64) - x)
    assert (err <= np.abs(up.astype(np.float64) - x)).all()
    assert (err <= np.abs(dn.astype(np.float64) - x)).all()


def test_gradient_finite_differences(orc):
    rng = np.random.default_rng(2)
    B, H, W = 2, 5, 6
    feat = rng.uniform(0, 1, (B, H, W, 4)).astype(np.float32)
    label = rng.integers(0, 2, (B, H, W)).astype(np.uint8)
    prm = rand_params(rng)
    for off in (OFF_B1, OFF_B2, OFF_B3):
        prm[off:off + 16] = 0.2  # keep most ReLUs away from their kink
    loss, _, g = orc.lrnet(feat, prm, label, round_bf16=False, want_grad=True)
    idx = np.concatenate([rng.choice(np.arange(OFF_W1, OFF_B1), 6, replace=False),
                          np.arange(OFF_B1, OFF_B1 + 2),
                          rng.choice(np.arange(OFF_W2, OFF_B2), 6, replace=False),
                          rng.choice(np.arange(OFF_W3, OFF_B3), 6, replace=False),
                          rng.choice(np.arange(OFF_W4, OFF_B4), 6, replace=False), [OFF_B4]])
    # The oracle rounds each pre-activation to FP32, so the loss carries ~1e-8 noise; a
    # wrong index or transpose would be off by far more than the 1 % allowed here.
    h = 3e-3
    for i in idx:
        p1 = prm.copy()
        p2 = prm.copy()
        p1[i] += np.float32(h)
        p2[i] -= np.float32(h)
        l1 = orc.lrnet(feat, p1, label, round_bf16=False)[0]
        l2 = orc.lrnet(feat, p2, label, round_bf16=False)[0]
        fd = (l1 - l2) / (float(p1[i]) - float(p2[i]))
        assert abs(fd - g[i]) <= 0.01 * abs(fd) + 2e-5, (i, fd, g[i])


def test_bce_gradient_closed_form(orc):
    # With all weights zero the logit is b4 everywhere: dL/db4 = mean(sigmoid(b4) - y).
    rng = np.random.default_rng(3)
    B, H, W = 1, 7, 9
    feat = rng.uniform(0, 1, (B, H, W, 4)).astype(np.float32)
    label = rng.integers(0, 2, (B, H, W)).astype(np.uint8)
    prm = np.zeros(NP, np.float32)
    prm[OFF_B4] = 0.7
    loss, logits, g = orc.lrnet(feat, prm, label, want_grad=True)
    z = float(np.float32(0.7))
    s = 1.0 / (1.0 + np.exp(-z))
    assert np.all(logits == np.float32(0.7))
    assert abs(g[OFF_B4] - (s - label.mean())) < 1e-6
    exp_loss = np.mean(np.log1p(np.exp(z)) - label * z)
    assert abs(loss - exp_loss) < 1e-9


def test_delta_input_reproduces_kernel(orc):
    # Channel 0 of the features is a unit impulse; layer 1 maps channel 0 through kernel K
    # into channel 0, layers 2-3 pass channel 0 through their centre tap, layer 4 reads it.
    K = np.array([[0.125, 0.25, 0.375], [0.5, 0.625, 0.75], [0.875, 1.0, 1.25]], np.float32)
    prm = np.zeros(NP, np.float32)
    prm[OFF_W1:OFF_W1 + 9] = K.reshape(-1)          # W1[0][0]
    prm[OFF_W2 + 4] = 1.0                            # W2[0][0][1][1]
    prm[OFF_W3 + 4] = 1.0                            # W3[0][0][1][1]
    prm[OFF_W4 + 4] = 1.0                            # W4[0][0][1][1]
    H, W = 7, 8
    y0, x0 = 3, 4
    feat = np.zeros((1, H, W, 4), np.float32)
    feat[0, y0, x0, 0] = 1.0
    _, logits, _ = orc.lrnet(feat, prm)
    z = logits[0]
    for ky in range(3):
        for kx in range(3):
            # Cross-correlation: output (y, x) sees input (y + ky - 1, x + kx - 1).
            assert z[y0 - ky + 1, x0 - kx + 1] == K[ky, kx]
    assert np.count_nonzero(z) == 9


def test_rounding_changes_little(orc):
    rng = np.random.default_rng(4)
    feat = rng.uniform(0, 1, (1, 8, 8, 4)).astype(np.float32)
    prm = rand_params(rng, 0.2)
    _, z_exact, _ = orc.lrnet(feat, prm, round_bf16=False)
    _, z_bf16, _ = orc.lrnet(feat, prm, round_bf16=True)
    assert np.allclose(z_exact, z_bf16, atol=0.05 * np.abs(z_exact).max())
    assert not np.array_equal(z_exact, z_bf16)


def test_adam_first_step_closed_form(orc):
    # First step with bias correction: m_hat = g, v_hat = g^2 -> dw = -lr * g / (|g| + eps).
    rng = np.random.default_rng(5)
    n = 64
    g = rng.standard_normal(n).astype(np.float32)
    w = rng.standard_normal(n).astype(np.float32)
    w0 = w.copy()
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    lr, eps = 1e-2, 1e-8
    orc.adam(w, m, v, g, lr, 0.9, 0.999, eps, 1)
    assert np.allclose(w - w0, -lr * g / (np.abs(g) + eps), rtol=1e-5, atol=1e-9)
    # A zero gradient leaves the weights unchanged.
    w1 = w.copy()
    orc.adam(w, m * 0, v * 0, np.zeros(n, np.float32), lr, 0.9, 0.999, eps, 2)
    assert np.array_equal(w, w1)


def test_features_definitions(orc):
    D = 6
    S = np.array([[[30, 20, 10, 25, 40, 12],     # d*=2, S2 = min over d in {0,4,5} = 12
                   [5, 9, 9, 9, 9, 9],           # d*=0, S2 = min over d>=2 = 9
                   [7, 0, 7, 7, 7, 7]]], np.uint16)  # d*=1, S_min=0 -> ratio uses max(S_min,1)
    img = np.array([[0, 255, 51]], np.uint8)
    w, _ = orc.wta(S)
    f = orc.features(img, S, w, P2=120)
    norm = 8 * (62 + 120)
    assert list(w[0]) == [2, 0, 1]
    assert np.allclose(f[0, :, 0], [0.0, 1.0, 0.2])
    assert np.allclose(f[0, :, 1], [2 / 5, 0.0, 1 / 5])
    assert np.allclose(f[0, :, 2], [10 / norm, 5 / norm, 0.0])
    assert np.allclose(f[0, :, 3], [12 / 10, 9 / 5, 7 / 1])
    # D = 2: no disparity is two away from d*, so S2 = S_min and the ratio is 1.
    S2 = np.array([[[4, 9]]], np.uint16)
    w2, _ = orc.wta(S2)
    f2 = orc.features(np.zeros((1, 1), np.uint8), S2, w2)
    assert f2[0, 0, 3] == 1.0


def test_network_separates_simple_labels(orc):
    # Sanity of the whole oracle loop: a few hundred Adam steps on a label that is a
    # threshold of one feature drive the loss well below its starting value.
    rng = np.random.default_rng(6)
    p = synth.pair_rectangles(0, H=16, W=24, D=8)
    feat = rng.uniform(0, 1, (2, 8, 8, 4)).astype(np.float32)
    label = (feat[..., 2] > 0.5).astype(np.uint8)
    prm = rand_params(rng, 0.2)
    m = np.zeros(NP, np.float32)
    v = np.zeros(NP, np.float32)
    first = None
    for step in range(1, 151):
        loss, _, g = orc.lrnet(feat, prm, label, want_grad=True)
        first = loss if first is None else first
        orc.adam(prm, m, v, g, 1e-2, 0.9, 0.999, 1e-8, step)
    assert loss < 0.5 * first
    assert p.left.shape == (16, 24)


@pytest.mark.parametrize("round_bf16", [False, True])
def test_backward_from_given_output_gradient(orc, round_bf16):
    """The backward from a given dL/dz4 equals the loss gradient when dL/dz4 is
    the BCE gradient (sigmoid(z4) - y) / N of the loss's own logits, and it is
    linear in dL/dz4 (scaling by a power of two scales every gradient exactly,
    and a sum of two output gradients gives the sum of the two gradients when
    nothing is rounded)."""
    rng = np.random.default_rng(21)
    B, H, W = 2, 9, 13
    feat = rng.uniform(0, 1.5, (B, H, W, 4)).astype(np.float32)
    label = (rng.uniform(size=(B, H, W)) < 0.6).astype(np.uint8)
    prm = rand_params(rng)
    _, z, g_loss = orc.lrnet(feat, prm, label, round_bf16=round_bf16, want_grad=True)
    s = 1.0 / (1.0 + np.exp(-z.astype(np.float64)))
    dz4 = ((s - label) / (B * H * W)).astype(np.float32)
    g = orc.lrnet_backward(feat, dz4, prm, round_bf16=round_bf16)
    assert np.array_equal(g, g_loss)
    assert np.array_equal(orc.lrnet_backward(feat, 4 * dz4, prm, round_bf16=round_bf16), 4 * g)
    if not round_bf16:
        e = rng.standard_normal((B, H, W)).astype(np.float32) * 1e-3
        ge = orc.lrnet_backward(feat, e, prm, round_bf16=False)
        gs = orc.lrnet_backward(feat, dz4 + e, prm, round_bf16=False)
        err = np.abs(gs.astype(np.float64) - g - ge)
        assert err.max() <= 1e-5 * np.abs(g).max(), err.max()
