"""Seeded synthetic inputs for the stereo / scene-flow hot path.

This module draws images, ground-truth disparity and optical flow.  It holds
none of the method's arithmetic (no census, no matching cost, no path
aggregation, no combination): it only renders scenes whose geometry is known,
so that both the HIP path and the CPU oracle consume identical bytes.

Workloads (the paper measures on KITTI Scene Flow frames, which are not
available here; these stand in for their shape, 1242x375, and nothing more):

* ``pair_rectangles``: 320x96 random-texture pair, piecewise-constant disparity
  (background 4 plus three rectangles with integer disparities in [0, D)),
  right view formed by shifting left pixels, occlusions filled with noise.
* ``frame_planar``: a full scene-flow frame (stereo pairs at t0 and t1 plus a
  noisy FP32 flow field) from a seeded piecewise-planar scene; used at
  1242x375 / D=128 (the headline workload), 640x480 / D=64,
  1920x1080 / D=256 and 2048x1024 / D=256.

Random numbers come from ``numpy.random.Generator(PCG64(seed))`` with
``seed = 1801047200 + 1000 * stream + index``, where ``stream`` is a small
integer that keeps the inputs of different uses (parity pairs, frames, batch
pairs, training pairs, sequences) apart.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 1801047200


def rng_for(stream: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * int(stream) + int(index)))


def blurred_texture(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """Uniform 0..255 noise, 3x3 box blur with clamp-to-edge, (sum + 4) // 9."""
    T = rng.integers(0, 256, size=(H, W), dtype=np.int32)
    P = np.pad(T, 1, mode="edge")
    s = np.zeros((H, W), np.int32)
    for dy in range(3):
        for dx in range(3):
            s += P[dy:dy + H, dx:dx + W]
    return ((s + 4) // 9).astype(np.uint8)


@dataclass
class StereoPair:
    left: np.ndarray        # uint8 [H][W]
    right: np.ndarray       # uint8 [H][W]
    gt_disp: np.ndarray     # float32 [H][W], left-view disparity
    occluded: np.ndarray    # bool [H][W], left pixels with no visible match
    disc: np.ndarray        # bool [H][W], pixels on a ground-truth discontinuity
    D: int


@dataclass
class Frame:
    t0: StereoPair
    t1: StereoPair
    flow: np.ndarray        # float32 [H][W][2] (u, v), the given (noisy) flow
    gt_flow: np.ndarray     # float32 [H][W][2]
    gt_disp1_at_t0: np.ndarray  # float32 [H][W]: t1 disparity of each t0 pixel
    D: int


def _last_wins(target: np.ndarray, key: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """For each distinct target index, the position (into the inputs) whose key
    is largest (ties: the later input).  Returns (unique targets, positions)."""
    order = np.lexsort((np.arange(target.size), key, target))
    t_sorted = target[order]
    rev = t_sorted[::-1]
    uniq, first_rev = np.unique(rev, return_index=True)
    pos = order[::-1][first_rev]
    return uniq, pos


def pair_rectangles(index: int = 0, H: int = 96, W: int = 320, D: int = 32, stream: int = 1) -> StereoPair:
    """Piecewise-constant disparity pair (the 320x96, D=32 parity workload)."""
    rng = rng_for(stream, index)
    L = blurred_texture(rng, H, W)
    gt = np.full((H, W), 4, np.int32)
    for _ in range(3):
        w = int(rng.integers(20, min(100, W) + 1)) if W >= 20 else W
        h = int(rng.integers(16, min(60, H) + 1)) if H >= 16 else H
        x0 = int(rng.integers(0, W - w + 1))
        y0 = int(rng.integers(0, H - h + 1))
        gt[y0:y0 + h, x0:x0 + w] = int(rng.integers(0, D))
    R = rng.integers(0, 256, size=(H, W), dtype=np.int32).astype(np.uint8)
    owner = np.full((H, W), -1, np.int64)
    ys, xs = np.mgrid[0:H, 0:W]
    # Visit pixels in increasing disparity so that the nearer surface wins.
    for d in np.unique(gt):
        sel = gt == d
        y = ys[sel]
        x = xs[sel]
        xr = x - d
        keep = xr >= 0
        R[y[keep], xr[keep]] = L[y[keep], x[keep]]
        owner[y[keep], xr[keep]] = y[keep] * W + x[keep]
    xr_all = xs - gt
    inb = xr_all >= 0
    own = np.full((H, W), -2, np.int64)
    own[inb] = owner[ys[inb], xr_all[inb]]
    occluded = own != (ys * W + xs)
    disc = np.zeros((H, W), bool)
    disc[:, 1:] |= gt[:, 1:] != gt[:, :-1]
    disc[:, :-1] |= gt[:, 1:] != gt[:, :-1]
    disc[1:, :] |= gt[1:, :] != gt[:-1, :]
    disc[:-1, :] |= gt[1:, :] != gt[:-1, :]
    return StereoPair(L, R, gt.astype(np.float32), occluded, disc, D)


def constant_pair(d: int, H: int, W: int, seed: int = 7) -> StereoPair:
    """Fronto-parallel scene at one integer disparity: R[x - d] = L[x]."""
    rng = rng_for(9, seed)
    L = blurred_texture(rng, H, W)
    R = rng.integers(0, 256, size=(H, W), dtype=np.int32).astype(np.uint8)
    if d < W:
        R[:, : W - d] = L[:, d:]
    gt = np.full((H, W), float(d), np.float32)
    xs = np.arange(W)[None, :].repeat(H, 0)
    return StereoPair(L, R, gt, xs - d < 0, np.zeros((H, W), bool), 0)


def _planes(rng, H, W, D, K):
    """Region labels and per-region disparity planes d = a + b x + c y."""
    lab = np.zeros((H, W), np.int32)
    hi = 0.85 * (D - 1)
    # Background: slanted plane, disparity growing towards the bottom rows.
    c0 = float(rng.uniform(0.3, 0.7)) * hi / max(H, 1)
    a0 = float(rng.uniform(0.05, 0.15)) * (D - 1)
    planes = [(a0, 0.0, c0)]
    for k in range(K):
        w = int(rng.integers(max(W // 16, 2), max(W // 3, 3)))
        h = int(rng.integers(max(H // 10, 2), max(H // 2, 3)))
        x0 = int(rng.integers(0, max(W - w, 1)))
        y0 = int(rng.integers(0, max(H - h, 1)))
        lab[y0:y0 + h, x0:x0 + w] = k + 1
        xc = x0 + 0.5 * w
        yc = y0 + 0.5 * h
        b = float(rng.uniform(-0.1, 0.1))
        c = float(rng.uniform(-0.1, 0.1))
        # Keep the plane inside [0, D-1] over its rectangle.
        span = abs(b) * 0.5 * w + abs(c) * 0.5 * h
        lo_c = min(span + 1.0, hi)
        dc = float(rng.uniform(lo_c, max(hi - span, lo_c)))
        planes.append((dc - b * xc - c * yc, b, c))
    return lab, planes


def _render_right(L, lab, planes, D, rng):
    """Right view by backward mapping each right pixel through every plane;
    the visible (largest disparity) plane whose support holds the pre-image
    wins.  Left intensities are sampled linearly along the row and rounded
    half-to-even; right pixels no plane reaches get fresh noise."""
    H, W = L.shape
    yr, xr = np.mgrid[0:H, 0:W].astype(np.float64)
    best_d = np.full((H, W), -1.0)
    best_x = np.zeros((H, W))
    best_k = np.full((H, W), -1, np.int32)
    for k, (a, b, c) in enumerate(planes):
        x = (xr + a + c * yr) / (1.0 - b)
        xi = np.rint(x).astype(np.int64)
        ok = (xi >= 0) & (xi < W)
        xi_c = np.clip(xi, 0, W - 1)
        ok &= lab[yr.astype(np.int64), xi_c] == k
        d = a + b * x + c * yr
        ok &= (d >= 0) & (d <= D - 1) & (x >= 0) & (x <= W - 1)
        better = ok & (d > best_d)
        best_d = np.where(better, d, best_d)
        best_x = np.where(better, x, best_x)
        best_k = np.where(better, k, best_k)
    x0 = np.floor(best_x).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    f = best_x - x0
    yi = yr.astype(np.int64)
    val = L[yi, np.clip(x0, 0, W - 1)] * (1.0 - f) + L[yi, x1] * f
    R = rng.integers(0, 256, size=(H, W), dtype=np.int32).astype(np.uint8)
    hit = best_k >= 0
    R[hit] = np.clip(np.rint(val[hit]), 0, 255).astype(np.uint8)
    return R, best_k, best_x


def _gt_disp(lab, planes, H, W, D):
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    P = np.array(planes)
    a = P[lab, 0]
    b = P[lab, 1]
    c = P[lab, 2]
    return np.clip(a + b * xs + c * ys, 0, D - 1)


def _occlusion(gt, lab, best_k, best_x):
    H, W = gt.shape
    ys, xs = np.mgrid[0:H, 0:W]
    xr = np.rint(xs - gt).astype(np.int64)
    inb = xr >= 0
    xr_c = np.clip(xr, 0, W - 1)
    vis = inb & (best_k[ys, xr_c] == lab) & (np.abs(best_x[ys, xr_c] - xs) < 1.0)
    return ~vis


def _disc(lab):
    disc = np.zeros(lab.shape, bool)
    dx = lab[:, 1:] != lab[:, :-1]
    dy = lab[1:, :] != lab[:-1, :]
    disc[:, 1:] |= dx
    disc[:, :-1] |= dx
    disc[1:, :] |= dy
    disc[:-1, :] |= dy
    return disc


def _pair_planar_labels(rng: np.random.Generator, H: int, W: int, D: int, K: int):
    L = blurred_texture(rng, H, W)
    lab, planes = _planes(rng, H, W, D, K)
    gt = _gt_disp(lab, planes, H, W, D)
    R, best_k, best_x = _render_right(L, lab, planes, D, rng)
    occ = _occlusion(gt, lab, best_k, best_x)
    return StereoPair(L, R, gt.astype(np.float32), occ, _disc(lab), D), lab


def pair_planar(rng: np.random.Generator, H: int, W: int, D: int, K: int = 6) -> StereoPair:
    """Random-texture pair over a seeded piecewise-planar disparity field."""
    return _pair_planar_labels(rng, H, W, D, K)[0]


def _splat(src_vals, depth_key, xt, yt, H, W, fill):
    """Forward splat to rounded targets, nearest (largest key) wins."""
    xi = np.rint(xt).astype(np.int64)
    yi = np.rint(yt).astype(np.int64)
    ok = (xi >= 0) & (xi < W) & (yi >= 0) & (yi < H)
    tgt = (yi * W + xi)[ok]
    uniq, pos = _last_wins(tgt, depth_key[ok])
    out = fill.copy().reshape(-1)
    out[uniq] = src_vals[ok][pos]
    hit = np.zeros(H * W, bool)
    hit[uniq] = True
    return out.reshape(H, W), hit.reshape(H, W)


def frame_planar(rng: np.random.Generator, H: int, W: int, D: int, flow_max: float,
                 K: int = 6) -> Frame:
    """Full scene-flow frame: stereo pairs at t0 and t1 and a noisy flow field.

    t0 is a piecewise-planar pair (``pair_planar``).  Each region moves with an
    affine 2-D flow (clipped to +-flow_max) and changes disparity by an affine
    offset within +-5 px.  The t1 left image is the t0 left image forward
    splatted along the ground-truth flow (nearer surface wins, holes get
    noise); the t1 right image is rendered from it the same way along the t1
    disparity.  The flow handed to the method is ground truth plus N(0, 0.5^2)
    per component, in FP32."""
    t0, lab = _pair_planar_labels(rng, H, W, D, K)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    nlab = K + 1
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    u0 = rng.uniform(-0.6, 0.6, nlab) * flow_max
    v0 = rng.uniform(-0.2, 0.2, nlab) * flow_max
    ux = rng.uniform(-0.05, 0.05, nlab)
    uy = rng.uniform(-0.05, 0.05, nlab)
    vx = rng.uniform(-0.05, 0.05, nlab)
    vy = rng.uniform(-0.05, 0.05, nlab)
    e0 = rng.uniform(-3.0, 3.0, nlab)
    ex = rng.uniform(-0.004, 0.004, nlab)
    ey = rng.uniform(-0.004, 0.004, nlab)
    # Background (label 0): forward ego-motion, radial expansion.
    u0[0], v0[0] = 0.0, 0.0
    ux[0], uy[0], vx[0], vy[0] = 0.04, 0.0, 0.0, 0.04
    gu = np.clip(u0[lab] + ux[lab] * (xs - cx) + uy[lab] * (ys - cy), -flow_max, flow_max)
    gv = np.clip(v0[lab] + vx[lab] * (xs - cx) + vy[lab] * (ys - cy), -flow_max, flow_max)
    dd = np.clip(e0[lab] + ex[lab] * (xs - cx) + ey[lab] * (ys - cy), -5.0, 5.0)
    d1 = np.clip(t0.gt_disp + dd, 0, D - 1)
    gt_flow = np.stack([gu, gv], -1).astype(np.float32)
    noise = rng.normal(0.0, 0.5, size=(H, W, 2))
    flow = (gt_flow + noise).astype(np.float32)
    # t1 left image and disparity grid.
    noise_img = rng.integers(0, 256, size=(H, W), dtype=np.int32).astype(np.uint8)
    L1, hit = _splat(t0.left.reshape(-1), d1.reshape(-1), (xs + gu).reshape(-1),
                     (ys + gv).reshape(-1), H, W, noise_img)
    bg = t0.gt_disp.copy()
    D1grid, _ = _splat(d1.reshape(-1), d1.reshape(-1), (xs + gu).reshape(-1),
                       (ys + gv).reshape(-1), H, W, bg)
    # t1 right image: splat L1 along the t1 disparity.
    noise_r = rng.integers(0, 256, size=(H, W), dtype=np.int32).astype(np.uint8)
    R1, hit_r = _splat(L1.reshape(-1), D1grid.reshape(-1), (xs - D1grid).reshape(-1),
                       ys.reshape(-1), H, W, noise_r)
    occ1 = ~hit
    t1 = StereoPair(L1.astype(np.uint8), R1.astype(np.uint8), D1grid.astype(np.float32),
                    occ1, _disc_real(D1grid), D)
    return Frame(t0, t1, flow, gt_flow, d1.astype(np.float32), D)


@dataclass
class Sequence:
    pairs: list          # StereoPair per time step t_0 .. t_{T-1}
    flows: list          # float32 [H][W][2]: the given (noisy) flow t_k -> t_{k+1}
    gt_flows: list       # float32 [H][W][2]
    gt_d1: list          # float32 [H][W]: disparity at t_{k+1} of each t_k pixel
    D: int


def sequence_planar(rng: np.random.Generator, T: int, H: int, W: int, D: int, flow_max: float,
                    K: int = 6) -> Sequence:
    """T stereo pairs of one scene: the t_0 pair is piecewise planar
    (``pair_planar``); every region keeps one affine 2-D velocity (small
    gradients, so motion is nearly constant from step to step) and one
    disparity change per step within +-2 px.  Each step forward-splats the left
    image, its disparities and region labels along the ground-truth flow
    (nearer surface wins; holes get noise and keep their previous disparity
    and label) and renders the right image along the new disparities.  The
    flow handed to the method is ground truth plus N(0, 0.5^2) per component."""
    t0, lab = _pair_planar_labels(rng, H, W, D, K)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    nlab = K + 1
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    u0 = rng.uniform(-0.6, 0.6, nlab) * flow_max
    v0 = rng.uniform(-0.2, 0.2, nlab) * flow_max
    ux = rng.uniform(-0.01, 0.01, nlab)
    uy = rng.uniform(-0.01, 0.01, nlab)
    vx = rng.uniform(-0.01, 0.01, nlab)
    vy = rng.uniform(-0.01, 0.01, nlab)
    e0 = rng.uniform(-2.0, 2.0, nlab)
    u0[0], v0[0] = 0.0, 0.0
    ux[0], uy[0], vx[0], vy[0] = 0.01, 0.0, 0.0, 0.01
    pairs, flows, gt_flows, gt_d1 = [t0], [], [], []
    L, d, lb = t0.left, t0.gt_disp.astype(np.float64), lab
    for _ in range(T - 1):
        gu = np.clip(u0[lb] + ux[lb] * (xs - cx) + uy[lb] * (ys - cy), -flow_max, flow_max)
        gv = np.clip(v0[lb] + vx[lb] * (xs - cx) + vy[lb] * (ys - cy), -flow_max, flow_max)
        d1 = np.clip(d + e0[lb], 0, D - 1)
        gt = np.stack([gu, gv], -1).astype(np.float32)
        gt_flows.append(gt)
        flows.append((gt + rng.normal(0.0, 0.5, size=(H, W, 2))).astype(np.float32))
        gt_d1.append(d1.astype(np.float32))
        tx, ty = (xs + gu).reshape(-1), (ys + gv).reshape(-1)
        noise_img = rng.integers(0, 256, size=(H, W), dtype=np.int32).astype(np.uint8)
        L1, hit = _splat(L.reshape(-1), d1.reshape(-1), tx, ty, H, W, noise_img)
        D1grid, _ = _splat(d1.reshape(-1), d1.reshape(-1), tx, ty, H, W, d)
        lab1, _ = _splat(lb.reshape(-1), d1.reshape(-1), tx, ty, H, W, lb)
        noise_r = rng.integers(0, 256, size=(H, W), dtype=np.int32).astype(np.uint8)
        R1, _ = _splat(L1.reshape(-1), D1grid.reshape(-1), (xs - D1grid).reshape(-1),
                       ys.reshape(-1), H, W, noise_r)
        pairs.append(StereoPair(L1.astype(np.uint8), R1.astype(np.uint8), D1grid.astype(np.float32),
                                ~hit, _disc_real(D1grid), D))
        L, d, lb = L1.astype(np.uint8), D1grid, lab1.astype(lab.dtype)
    return Sequence(pairs, flows, gt_flows, gt_d1, D)


def _disc_real(d: np.ndarray) -> np.ndarray:
    """Pixels next to a jump of more than half a pixel in a disparity map."""
    disc = np.zeros(d.shape, bool)
    dx = np.abs(d[:, 1:] - d[:, :-1]) > 0.5
    dy = np.abs(d[1:, :] - d[:-1, :]) > 0.5
    disc[:, 1:] |= dx
    disc[:, :-1] |= dx
    disc[1:, :] |= dy
    disc[:-1, :] |= dy
    return disc


# Named workloads ---------------------------------------------------------------

WORKLOADS = {
    "pair_320x96": dict(H=96, W=320, D=32),
    "frame_1242x375": dict(H=375, W=1242, D=128, flow_max=100.0),
    "vga": dict(H=480, W=640, D=64, flow_max=100.0),
    "fhd": dict(H=1080, W=1920, D=256, flow_max=100.0),
    "frame_2048x1024": dict(H=1024, W=2048, D=256, flow_max=200.0),
}


def frame_1242x375(index: int = 0) -> Frame:
    """1242x375, D=128 scene-flow frame (flow within +-100 px)."""
    return frame_planar(rng_for(2, index), 375, 1242, 128, 100.0)


def batch_sizes(n_pairs: int = 64):
    """Size classes of the uneven batch: pair i has class i mod 3."""
    classes = [(480, 640, 64), (375, 1242, 128), (1080, 1920, 256)]
    return [classes[i % 3] for i in range(n_pairs)]


def pair_batch(index: int, H: int, W: int, D: int) -> StereoPair:
    return pair_planar(rng_for(3, index), H, W, D)
