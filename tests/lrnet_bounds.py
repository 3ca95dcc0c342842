"""Error analysis of the learned stand-in's GPU arithmetic against the oracle.

Test infrastructure: nothing here produces an expected value (those come from
the oracle).  This module gives (i) the condition under which every FP32 sum
of the network is exact, so that the GPU's summation order cannot matter and
its results must equal the oracle's bit for bit, and (ii) per-element bounds
on |GPU - oracle| for arbitrary inputs, propagated layer by layer from the two
sides' only legitimate differences:
  * the GPU forms each sum in FP32 in its own order (the oracle sums exactly
    and rounds once): at most gamma(n) times the sum of the absolute terms,
    plus the oracle's own final rounding;
  * a changed FP32 sum can round to a different BF16 value (one BF16 unit,
    2^-7 relative) and can change the sign test of a ReLU where the
    pre-activation is within its bound of zero;
  * the GPU's sigmoid is FP32 (expf), the oracle's FP64.
The magnitudes come from a float64 evaluation of the network's definition
(the same layer formulas the oracle's header states), which is used only for
these bounds and conditions.  Layouts: feat [B][H][W][4], params flat as in
the oracle.
"""
import numpy as np

U = 2.0 ** -24
BF16_REL = 2.0 ** -7


def gamma(n):
    return n * U / (1.0 - n * U)


def bf16(x):
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def unpack(params):
    p = np.asarray(params, np.float32)
    W1 = p[0:576].reshape(16, 4, 3, 3)
    b1 = p[576:592]
    W2 = p[592:2896].reshape(16, 16, 3, 3)
    b2 = p[2896:2912]
    W3 = p[2912:5216].reshape(16, 16, 3, 3)
    b3 = p[5216:5232]
    W4 = p[5232:5376].reshape(1, 16, 3, 3)
    b4 = p[5376:5377]
    return [(W1, b1), (W2, b2), (W3, b3), (W4, b4)]


def conv(a, w):
    """z[b,o,y,x] = sum_{c,ky,kx} w[o,c,ky,kx] a[b,c,y+ky-1,x+kx-1] (zero padding)."""
    B, C, H, W = a.shape
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    z = np.zeros((B, w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            z += np.einsum("oc,bchw->bohw", w[:, :, ky, kx].astype(np.float64), ap[:, :, ky:ky + H, kx:kx + W],
                           optimize=True)
    return z


def conv_t(g, w):
    """ga[b,c,y,x] = sum_{o,ky,kx} w[o,c,ky,kx] g[b,o,y-ky+1,x-kx+1]."""
    B, O, H, W = g.shape
    gp = np.pad(g, ((0, 0), (0, 0), (1, 1), (1, 1)))
    ga = np.zeros((B, w.shape[1], H, W))
    for ky in range(3):
        for kx in range(3):
            ga += np.einsum("oc,bohw->bchw", w[:, :, ky, kx].astype(np.float64),
                            gp[:, :, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W], optimize=True)
    return ga


def wgrad(g, a):
    """dW[o,c,ky,kx] = sum_{b,y,x} g[b,o,y,x] a[b,c,y+ky-1,x+kx-1]."""
    B, C, H, W = a.shape
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dw = np.zeros((g.shape[1], C, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", g, ap[:, :, ky:ky + H, kx:kx + W], optimize=True)
    return dw


def evaluate(feat, params, dz4=None):
    """Float64 evaluation of the network's definition with its BF16 roundings:
    activations a0..a3, pre-activations z1..z4 and, for a given dL/dz4, the
    backward signals gz1..gz3 (layer inputs' gradients, BF16) and ga1..ga3."""
    f = np.asarray(feat, np.float32)
    if f.ndim == 3:
        f = f[None]
    layers = [(bf16(w).astype(np.float64), b.astype(np.float64)) for w, b in unpack(params)]
    a = [bf16(np.transpose(f, (0, 3, 1, 2))).astype(np.float64)]
    z = []
    for l, (w, b) in enumerate(layers):
        zl = (conv(a[-1], w) + b[None, :, None, None]).astype(np.float32).astype(np.float64)
        z.append(zl)
        if l < 3:
            a.append(bf16(np.maximum(zl, 0.0)).astype(np.float64))
    out = {"a": a, "z": z, "layers": layers}
    if dz4 is not None:
        g = np.asarray(dz4, np.float32).reshape(z[3].shape).astype(np.float64)
        gz = [None, None, None, g]  # gz[l] = dL/dz_{l+1}
        ga = [None, None, None]
        for l in (3, 2, 1):
            gal = conv_t(gz[l], layers[l][0])
            ga[l - 1] = gal
            gz[l - 1] = bf16(np.where(z[l - 1] > 0, gal.astype(np.float32), 0.0)).astype(np.float64)
        out.update(gz=gz, ga=ga)
    return out


def _v2(x):
    """2-adic valuation of each nonzero float64 (exponent of its lowest set bit);
    +inf for zeros."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)
    M = np.abs(m * 2.0 ** 53).astype(np.int64)
    tz = np.zeros(M.shape, np.int64)
    mm = M.copy()
    nz = mm != 0
    for s in (32, 16, 8, 4, 2, 1):
        low = nz & ((mm & ((1 << s) - 1)) == 0)
        tz[low] += s
        mm[low] >>= s
    v = (e - 53 + tz).astype(np.float64)
    v[~nz] = np.inf
    return v


def _fits(abs_sum, *vals):
    """Sums whose terms are products of the given factor arrays are exact in
    FP32, in any order, when every term is a multiple of q = 2^(sum of the
    factors' smallest valuations) and the absolute sum stays below 2^24 q."""
    if any(np.size(v) == 0 for v in vals):
        return True
    q = sum(float(np.min(_v2(v))) for v in vals)
    if not np.isfinite(q):
        return True
    return float(np.max(abs_sum)) < 2.0 ** (24 + q)


def sums_exact(feat, params, dz4=None):
    """True when every FP32 sum of the forward (and, with dz4, of the backward
    and the weight gradients) is exact whatever its order."""
    ev = evaluate(feat, params, dz4)
    a, layers = ev["a"], ev["layers"]
    for l, (w, b) in enumerate(layers):
        s = conv(np.abs(a[l]), np.abs(w)) + np.abs(b)[None, :, None, None]
        bv = b[b != 0]
        if not _fits(s, w[w != 0], a[l][a[l] != 0]):
            return False
        if bv.size and not _fits(s, bv):
            return False
    if dz4 is None:
        return True
    gz = ev["gz"]
    for l in (3, 2, 1):
        w = layers[l][0]
        g = gz[l]
        if not _fits(conv_t(np.abs(g), np.abs(w)), w[w != 0], g[g != 0]):
            return False
    for l in range(4):
        g, al = gz[l], a[l]
        if not _fits(wgrad(np.abs(g), np.abs(al)), g[g != 0], al[al != 0]):
            return False
        if not _fits(np.abs(g).sum(axis=(0, 2, 3)), g[g != 0]):
            return False
    return True


def boundary_distance(v):
    """Distance of each value (float64 array, taken as FP32) to the nearest
    rounding boundary of BF16 round-to-nearest-even: the midpoints between its
    BF16 value and the two neighbouring BF16 values (0 on a boundary)."""
    v = np.asarray(v, np.float64)
    r = bf16(v.astype(np.float32))
    bits = r.view(np.uint32).astype(np.int64)
    up = (bits + 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    dn_bits = np.where((bits & 0x7FFFFFFF) == 0, bits ^ 0x80000000 | 0x10000, bits - 0x10000)
    dn = dn_bits.astype(np.uint32).view(np.float32).astype(np.float64)
    rr = r.astype(np.float64)
    lo, hi = (rr + dn) / 2.0, (rr + up) / 2.0
    lo, hi = np.minimum(lo, hi), np.maximum(lo, hi)
    return np.minimum(np.abs(v - lo), np.abs(hi - v))


def _rounding_change(v, d):
    """Bound on |bf16(x) - bf16(v)| for |x - v| <= d: zero when no rounding
    boundary lies within d of v (both round to the same BF16 value), else d
    plus one BF16 unit."""
    amb = boundary_distance(v) <= d
    return np.where(amb, d + BF16_REL * (np.abs(v) + d), 0.0)


def forward_bounds(ev):
    """Per-element bounds dz[l] on |z_gpu - z_oracle| and da[l] on the layer
    inputs' differences.  An activation can differ only where its
    pre-activation lies within its bound of zero (the ReLU) or of a BF16
    rounding boundary; everywhere else both sides hold the same BF16 value.
    The float64 evaluation may itself differ from the oracle's FP32 values by
    one FP32 unit, which the 2u|z| terms cover."""
    a, z, layers = ev["a"], ev["z"], ev["layers"]
    n_terms = [36, 144, 144, 144]
    da = [np.zeros_like(a[0])]
    dz = []
    for l, (w, b) in enumerate(layers):
        aw = np.abs(w)
        S = conv(np.abs(a[l]) + da[l], aw) + np.abs(b)[None, :, None, None]
        d = conv(da[l], aw) + gamma(n_terms[l] + 1) * S + 2 * U * np.abs(z[l])
        dz.append(d)
        if l < 3:
            relu_amb = np.abs(z[l]) <= d
            dal = np.where(z[l] > 0, _rounding_change(z[l], d), 0.0)
            da.append(np.where(relu_amb, d + BF16_REL * (np.abs(z[l]) + d), dal))
    return dz, da


def gradient_bounds(ev, dz, da, ddz4):
    """Per-parameter bound on |grad_gpu - grad_oracle| (flat, 5377) for the
    backward from dL/dz4 whose two sides differ by at most ddz4 per pixel."""
    a, z, layers, gz, ga = ev["a"], ev["z"], ev["layers"], ev["gz"], ev["ga"]
    N = gz[3].size
    dgz = [None, None, None, np.broadcast_to(np.asarray(ddz4, np.float64).reshape(
        (-1,) + gz[3].shape[2:])[:, None] if np.ndim(ddz4) else np.asarray(ddz4, np.float64), gz[3].shape)]
    for l in (3, 2, 1):
        aw = np.abs(layers[l][0])
        n = 16 * 9 if l < 3 else 9
        dga = conv_t(dgz[l], aw) + gamma(n + 1) * conv_t(np.abs(gz[l]) + dgz[l], aw) + 2 * U * np.abs(ga[l - 1])
        gate_amb = (np.abs(z[l - 1]) <= dz[l - 1]) | (np.abs(z[l - 1]) < 1e-37)
        full = np.abs(ga[l - 1]) + dga
        opened = np.where(z[l - 1] > 0, _rounding_change(ga[l - 1], dga), 0.0)
        dgz[l - 1] = np.where(gate_amb, full + BF16_REL * full, opened)
    out = []
    for l in range(4):
        g, dg, al, dal = np.abs(gz[l]), dgz[l], np.abs(a[l]), da[l]
        dW = (wgrad(dg, al + dal) + wgrad(g, dal) + gamma(N) * wgrad(g + dg, al + dal)
              + 2 * U * np.abs(wgrad(gz[l], a[l])))
        db = dg.sum(axis=(0, 2, 3)) + gamma(N) * (g + dg).sum(axis=(0, 2, 3)) + 2 * U * np.abs(gz[l].sum(axis=(0, 2, 3)))
        out += [dW.reshape(-1), db]
    return np.concatenate(out)


def loss_gradient_bound(ev, dz4_bound):
    """Bound on |dL/dz4_gpu - dL/dz4_oracle| for the mean BCE loss: the GPU's
    FP32 sigmoid (expf, one division, one subtraction, one product) against
    the oracle's FP64 one rounded to FP32, plus the logits' own difference
    (the sigmoid's slope is at most 1/4)."""
    z4 = ev["z"][3]
    N = z4.size
    return (dz4_bound / 4.0 + 2.0 ** -20) / N


def dyadic_case(seed, B, H, W, with_dz4=True):
    """A seeded dyadic input (features k/16, weights k/16 with |k| <= 4 in the
    first and last layers and <= 2 in the middle ones, biases k/256, a sparse
    dL/dz4 of multiples of 1/1024) whose every sum is exact, trying seeds from
    `seed` on."""
    NP = 5377
    for s in range(seed, seed + 100):
        rng = np.random.default_rng(s)
        feat = (rng.integers(0, 17, (B, H, W, 4)) / 16.0).astype(np.float32)
        prm = (rng.integers(-4, 5, NP) / 16.0).astype(np.float32)
        prm[592:2896] = rng.integers(-2, 3, 2304) / 16.0
        prm[2912:5216] = rng.integers(-2, 3, 2304) / 16.0
        for off in (576, 2896, 5216):
            prm[off:off + 16] = rng.integers(-64, 257, 16) / 256.0
        prm[5376] = rng.integers(-256, 257) / 256.0
        dz4 = np.zeros((B, H, W), np.float32)
        n = max(1, (H * W) // 150)
        for b in range(B):
            idx = rng.choice(H * W, n, replace=False)
            dz4[b].reshape(-1)[idx] = rng.integers(-8, 9, n) / 1024.0
        if sums_exact(feat, prm, dz4 if with_dz4 else None):
            return feat, prm, dz4
    raise AssertionError("no exact dyadic case")
