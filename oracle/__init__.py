"""CPU oracle for the stereo / scene-flow hot path (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  The
C sources (sgm_oracle.c, lrnet_oracle.c, flow_oracle.c) are plain single-threaded loops that
follow the definitions one by one; this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = ["sgm_oracle.c", "lrnet_oracle.c", "flow_oracle.c"]
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, one thread."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp] + [os.path.join(_HERE, s) for s in _SRCS] + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ct.CDLL(_SO)
        _declare(_lib)
    return _lib


P = ct.c_void_p
I = ct.c_int
F = ct.c_float


def _declare(L):
    L.oracle_census.argtypes = [P, I, I, I, P]
    L.oracle_cost.argtypes = [P, P, I, I, I, I, P]
    L.oracle_path_cost.argtypes = [P, I, I, I, I, I, I, P]
    L.oracle_aggregate.argtypes = [P, I, I, I, I, I, ct.c_uint, P]
    L.oracle_wta.argtypes = [P, I, I, I, P, P]
    L.oracle_lr_check.argtypes = [P, P, P, I, I, I, P, P]
    L.oracle_no_check.argtypes = [P, I, I, P, P]
    L.oracle_combine.argtypes = [P, P, P, P, P, I, I, I, F, F, F, F, P, P, P, P]
    L.oracle_disparity.argtypes = [P, P, I, I, I, I, I, I, ct.c_uint, I, P, P, P]
    L.oracle_path_cost_adaptive.argtypes = [P, P, I, I, I, I, I, I, I, P]
    L.oracle_aggregate_adaptive.argtypes = [P, P, I, I, I, I, I, I, ct.c_uint, P]
    L.oracle_wta_right_diag.argtypes = [P, I, I, I, P]
    L.oracle_median3x3.argtypes = [P, I, I, P]
    L.oracle_disparity_ex.argtypes = [P, P, I, I, I, I, I, I, ct.c_uint, I, I, P, P, P]
    L.oracle_densify.argtypes = [P, P, I, I, P, P]
    L.oracle_temporal_check.argtypes = [P, P, P, P, I, I, F, F, P]
    L.oracle_aggregate_at.argtypes = [P, P, I, I, I, I, I, I, ct.c_uint, I, I, P]
    L.oracle_disparity_at.argtypes = [P, P, I, I, I, I, I, I, I, P, P, I, P, P, P]
    L.oracle_splitmix64.argtypes = [ct.c_uint64, ct.c_uint64]
    L.oracle_splitmix64.restype = ct.c_uint64
    L.oracle_pyr_down.argtypes = [P, I, I, P]
    L.oracle_pm_offset.argtypes = [ct.c_uint64, I, I, I, I, I, I, P, P]
    L.oracle_pm_pixel.argtypes = [P, P, I, I, I, I, I, ct.c_uint64, P, I, I, P, P, P, I]
    L.oracle_pm_pixel.restype = I
    L.oracle_flow_cost.argtypes = [P, P, I, I, I, I, I, I]
    L.oracle_pm_flow.argtypes = [P, P, I, I, I, I, I, I, ct.c_uint64, P]
    L.oracle_fb_check.argtypes = [P, P, I, I, I, P]
    L.oracle_flow.argtypes = [P, P, I, I, I, I, I, I, ct.c_uint64, I, P, P, P]
    L.oracle_features.argtypes = [P, I, P, P, I, I, I, I, P]
    L.oracle_lrnet.argtypes = [P, P, I, I, I, P, I, P, P]
    L.oracle_lrnet.restype = ct.c_double
    L.oracle_lrnet_nparams.restype = I
    L.oracle_lrnet_backward.argtypes = [P, P, I, I, I, P, I, P]
    L.oracle_bf16.argtypes = [F]
    L.oracle_bf16.restype = F
    L.oracle_adam.argtypes = [P, P, P, P, I, F, F, F, F, F, F]


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ct.c_void_p)


def census(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    H, W = img.shape
    out = np.zeros((H, W), np.uint64)
    lib().oracle_census(_p(img), H, W, W, _p(out))
    return out


def cost(cen_base, cen_match, D: int, base_is_right: bool) -> np.ndarray:
    cb = np.ascontiguousarray(cen_base, np.uint64)
    cm = np.ascontiguousarray(cen_match, np.uint64)
    H, W = cb.shape
    out = np.zeros((H, W, D), np.uint8)
    lib().oracle_cost(_p(cb), _p(cm), H, W, D, int(base_is_right), _p(out))
    return out


def path_cost(cost_vol: np.ndarray, P1: int, P2: int, direction: int) -> np.ndarray:
    c = np.ascontiguousarray(cost_vol, np.uint8)
    H, W, D = c.shape
    out = np.zeros((H, W, D), np.int32)
    lib().oracle_path_cost(_p(c), H, W, D, P1, P2, direction, _p(out))
    return out


def aggregate(cost_vol: np.ndarray, P1: int, P2: int, path_mask: int = 0xFF) -> np.ndarray:
    c = np.ascontiguousarray(cost_vol, np.uint8)
    H, W, D = c.shape
    out = np.zeros((H, W, D), np.uint16)
    lib().oracle_aggregate(_p(c), H, W, D, P1, P2, path_mask, _p(out))
    return out


def path_cost_adaptive(cost_vol: np.ndarray, img: np.ndarray, P1: int, P2: int,
                       direction: int) -> np.ndarray:
    """Path cost with the intensity-adaptive large-jump penalty (img = base image)."""
    c = np.ascontiguousarray(cost_vol, np.uint8)
    im = np.ascontiguousarray(img, np.uint8)
    H, W, D = c.shape
    out = np.zeros((H, W, D), np.int32)
    lib().oracle_path_cost_adaptive(_p(c), _p(im), W, H, W, D, P1, P2, direction, _p(out))
    return out


def aggregate_adaptive(cost_vol: np.ndarray, img: np.ndarray, P1: int, P2: int,
                       path_mask: int = 0xFF) -> np.ndarray:
    c = np.ascontiguousarray(cost_vol, np.uint8)
    im = np.ascontiguousarray(img, np.uint8)
    H, W, D = c.shape
    out = np.zeros((H, W, D), np.uint16)
    lib().oracle_aggregate_adaptive(_p(c), _p(im), W, H, W, D, P1, P2, path_mask, _p(out))
    return out


def wta_right_diag(S: np.ndarray) -> np.ndarray:
    """Right-view WTA by the diagonal search in the left volume S_L."""
    S = np.ascontiguousarray(S, np.uint16)
    H, W, D = S.shape
    w = np.zeros((H, W), np.int16)
    lib().oracle_wta_right_diag(_p(S), H, W, D, _p(w))
    return w


def median3x3(m: np.ndarray) -> np.ndarray:
    m = np.ascontiguousarray(m, np.float32)
    H, W = m.shape
    out = np.zeros((H, W), np.float32)
    lib().oracle_median3x3(_p(m), H, W, _p(out))
    return out


def wta(S: np.ndarray):
    S = np.ascontiguousarray(S, np.uint16)
    H, W, D = S.shape
    w = np.zeros((H, W), np.int16)
    ds = np.zeros((H, W), np.float32)
    lib().oracle_wta(_p(S), H, W, D, _p(w), _p(ds))
    return w, ds


def lr_check(wta_l, wta_r, dsub_l, tol: int = 1):
    wl = np.ascontiguousarray(wta_l, np.int16)
    wr = np.ascontiguousarray(wta_r, np.int16)
    ds = np.ascontiguousarray(dsub_l, np.float32)
    H, W = wl.shape
    valid = np.zeros((H, W), np.uint8)
    disp = np.zeros((H, W), np.float32)
    lib().oracle_lr_check(_p(wl), _p(wr), _p(ds), H, W, tol, _p(valid), _p(disp))
    return valid, disp


def no_check(dsub_l):
    ds = np.ascontiguousarray(dsub_l, np.float32)
    H, W = ds.shape
    valid = np.zeros((H, W), np.uint8)
    disp = np.zeros((H, W), np.float32)
    lib().oracle_no_check(_p(ds), H, W, _p(valid), _p(disp))
    return valid, disp


def combine(disp0, valid0, disp1, valid1, flow, cam=None):
    d0 = np.ascontiguousarray(disp0, np.float32)
    v0 = np.ascontiguousarray(valid0, np.uint8)
    d1 = np.ascontiguousarray(disp1, np.float32)
    v1 = np.ascontiguousarray(valid1, np.uint8)
    fl = np.ascontiguousarray(flow, np.float32)
    H, W = d0.shape
    sf4 = np.zeros((H, W, 4), np.float32)
    valid = np.zeros((H, W), np.uint8)
    xyz0 = np.zeros((H, W, 3), np.float32)
    motion = np.zeros((H, W, 3), np.float32)
    if cam is None:
        has, f, B, cx, cy = 0, 0.0, 0.0, 0.0, 0.0
    else:
        has = 1
        f, B, cx, cy = cam
    lib().oracle_combine(_p(d0), _p(v0), _p(d1), _p(v1), _p(fl), H, W, has, f, B, cx, cy,
                         _p(sf4), _p(valid), _p(xyz0), _p(motion))
    if cam is None:
        return sf4, valid
    return sf4, valid, xyz0, motion


def disparity(left, right, D, P1=10, P2=120, path_mask=0xFF, tol=1):
    """Full plain disparity map of one pair (census, both views, LR check)."""
    L = np.ascontiguousarray(left, np.uint8)
    R = np.ascontiguousarray(right, np.uint8)
    H, W = L.shape
    w = np.zeros((H, W), np.int16)
    disp = np.zeros((H, W), np.float32)
    valid = np.zeros((H, W), np.uint8)
    lib().oracle_disparity(_p(L), _p(R), H, W, W, D, P1, P2, path_mask, tol, _p(w), _p(disp),
                           _p(valid))
    return w, disp, valid


def densify(sf4, valid):
    """Dense scene-flow map and fill code (1 defined, 2 row fill, 3 copied row, 0 none)."""
    s = np.ascontiguousarray(sf4, np.float32)
    v = np.ascontiguousarray(valid, np.uint8)
    H, W = v.shape
    out = np.zeros((H, W, 4), np.float32)
    fill = np.zeros((H, W), np.uint8)
    lib().oracle_densify(_p(s), _p(v), H, W, _p(out), _p(fill))
    return out, fill


def aggregate_at(cen_base, cen_match, D, base_is_right, P1, P2, x, y, path_mask=0xFF):
    """S(x, y, .) [D] uint16 from the path recurrences along the lines into (x, y)."""
    cb = np.ascontiguousarray(cen_base, np.uint64)
    cm = np.ascontiguousarray(cen_match, np.uint64)
    H, W = cb.shape
    out = np.zeros(D, np.uint16)
    lib().oracle_aggregate_at(_p(cb), _p(cm), H, W, D, int(base_is_right), P1, P2, path_mask, x, y,
                              _p(out))
    return out


def disparity_at(left, right, D, xs, ys, P1=10, P2=120, tol=1):
    """Plain disparity map (with LR check) at sampled pixels: (wta, disp, valid) per sample."""
    L = np.ascontiguousarray(left, np.uint8)
    R = np.ascontiguousarray(right, np.uint8)
    H, W = L.shape
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    n = len(xs)
    w = np.zeros(n, np.int16)
    disp = np.zeros(n, np.float32)
    valid = np.zeros(n, np.uint8)
    lib().oracle_disparity_at(_p(L), _p(R), H, W, W, D, P1, P2, tol, _p(xs), _p(ys), n, _p(w),
                              _p(disp), _p(valid))
    return w, disp, valid


def temporal_check(sf4a, va, sf4b, vb, tau_f=2.0, tau_d=1.0):
    """1 where S_k is kept by the check against S_{k+1} along its own flow."""
    a = np.ascontiguousarray(sf4a, np.float32)
    b = np.ascontiguousarray(sf4b, np.float32)
    pa = np.ascontiguousarray(va, np.uint8)
    pb = np.ascontiguousarray(vb, np.uint8)
    H, W = pa.shape
    out = np.zeros((H, W), np.uint8)
    lib().oracle_temporal_check(_p(a), _p(pa), _p(b), _p(pb), H, W, tau_f, tau_d, _p(out))
    return out


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().oracle_splitmix64(seed, counter))


def pyr_down(img):
    a = np.ascontiguousarray(img, np.uint8)
    H, W = a.shape
    out = np.zeros(((H + 1) // 2, (W + 1) // 2), np.uint8)
    lib().oracle_pyr_down(_p(a), H, W, _p(out))
    return out


def pm_offset(seed, level, it, k, x, y, r):
    """Random-search offset (u, v) of candidate k with radius r at pixel (x, y)."""
    ou, ov = ct.c_int(0), ct.c_int(0)
    lib().oracle_pm_offset(seed, level, it, k, x, y, r, ct.byref(ou), ct.byref(ov))
    return ou.value, ov.value


def pm_pixel(c0, c1, level, it, Rl, seed, fin, x, y, max_trace=64):
    """One pixel of one search iteration: the winner (u, v) and the evaluated
    candidates as rows (u, v, cost), in evaluation order."""
    a = np.ascontiguousarray(c0, np.uint64)
    b = np.ascontiguousarray(c1, np.uint64)
    f = np.ascontiguousarray(fin, np.int16)
    H, W = a.shape
    tr = np.zeros((max_trace, 3), np.int32)
    bu, bv = ct.c_int(0), ct.c_int(0)
    n = lib().oracle_pm_pixel(_p(a), _p(b), H, W, level, it, Rl, seed, _p(f), x, y, ct.byref(bu),
                              ct.byref(bv), _p(tr), max_trace)
    assert n <= max_trace
    return (bu.value, bv.value), tr[:n]


def flow_cost(c0, c1, x, y, fu, fv):
    a = np.ascontiguousarray(c0, np.uint64)
    b = np.ascontiguousarray(c1, np.uint64)
    H, W = a.shape
    return int(lib().oracle_flow_cost(_p(a), _p(b), H, W, x, y, fu, fv))


def pm_flow(A, B, levels=5, iters=4, R=128, seed=1801, fine_radius=0):
    """Integer flow [H][W][2] int16 from A to B (the stand-in without the check)."""
    a = np.ascontiguousarray(A, np.uint8)
    b = np.ascontiguousarray(B, np.uint8)
    H, W = a.shape
    assert 1 <= levels <= 16
    out = np.zeros((H, W, 2), np.int16)
    lib().oracle_pm_flow(_p(a), _p(b), H, W, levels, iters, R, fine_radius, seed, _p(out))
    return out


def fb_check(F, B, tol=1):
    f = np.ascontiguousarray(F, np.int16)
    b = np.ascontiguousarray(B, np.int16)
    H, W = f.shape[:2]
    out = np.zeros((H, W, 2), np.float32)
    lib().oracle_fb_check(_p(f), _p(b), H, W, tol, _p(out))
    return out


def flow(L0, L1, levels=5, iters=4, R=128, seed=1801, tol=1, fine_radius=0):
    """Forward, backward integer flows and the checked float flow (NaN where dropped)."""
    a = np.ascontiguousarray(L0, np.uint8)
    b = np.ascontiguousarray(L1, np.uint8)
    H, W = a.shape
    assert 1 <= levels <= 16
    F = np.zeros((H, W, 2), np.int16)
    B = np.zeros((H, W, 2), np.int16)
    out = np.zeros((H, W, 2), np.float32)
    lib().oracle_flow(_p(a), _p(b), H, W, levels, iters, R, fine_radius, seed, tol, _p(F), _p(B),
                      _p(out))
    return F, B, out


DIAG, MEDIAN, ADAPTIVE = 1, 2, 4


def disparity_ex(left, right, D, flags, P1=10, P2=120, path_mask=0xFF, tol=1):
    """Disparity map of one pair with the SGM variants (DIAG | MEDIAN | ADAPTIVE)."""
    L = np.ascontiguousarray(left, np.uint8)
    R = np.ascontiguousarray(right, np.uint8)
    H, W = L.shape
    w = np.zeros((H, W), np.int16)
    disp = np.zeros((H, W), np.float32)
    valid = np.zeros((H, W), np.uint8)
    lib().oracle_disparity_ex(_p(L), _p(R), H, W, W, D, P1, P2, path_mask, tol, flags, _p(w),
                              _p(disp), _p(valid))
    return w, disp, valid


def features(img, S, wta_map, P2: int = 120):
    img = np.ascontiguousarray(img, np.uint8)
    S = np.ascontiguousarray(S, np.uint16)
    w = np.ascontiguousarray(wta_map, np.int16)
    H, W, D = S.shape
    feat = np.zeros((H, W, 4), np.float32)
    lib().oracle_features(_p(img), W, _p(S), _p(w), H, W, D, P2, _p(feat))
    return feat


NPARAM = 5377


def lrnet(feat, params, label=None, round_bf16=True, want_grad=False):
    """Forward (and backward) of the 4-layer network over a batch.

    feat: float32 [B][H][W][4]; params: float32 [5377]; label: uint8 [B][H][W].
    Returns (loss, logits[B][H][W], grad[5377] or None)."""
    f = np.ascontiguousarray(feat, np.float32)
    if f.ndim == 3:
        f = f[None]
    B, H, W, _ = f.shape
    prm = np.ascontiguousarray(params, np.float32)
    assert prm.size == NPARAM
    logits = np.zeros((B, H, W), np.float32)
    grad = np.zeros(NPARAM, np.float32) if want_grad else None
    lb = None
    if label is not None:
        lb = np.ascontiguousarray(label, np.uint8).reshape(B, H, W)
    loss = lib().oracle_lrnet(_p(f), _p(lb) if lb is not None else None, B, H, W, _p(prm),
                              int(round_bf16), _p(grad) if grad is not None else None,
                              _p(logits))
    return loss, logits, grad


def lrnet_backward(feat, dz4, params, round_bf16=True):
    """Parameter gradient [5377] of the network for a given dL/dz4 [B][H][W]."""
    f = np.ascontiguousarray(feat, np.float32)
    if f.ndim == 3:
        f = f[None]
    B, H, W, _ = f.shape
    g = np.ascontiguousarray(dz4, np.float32).reshape(B, H, W)
    prm = np.ascontiguousarray(params, np.float32)
    grad = np.zeros(NPARAM, np.float32)
    lib().oracle_lrnet_backward(_p(f), _p(g), B, H, W, _p(prm), int(round_bf16), _p(grad))
    return grad


def bf16(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, np.float32)
    f = lib().oracle_bf16
    return np.array([f(float(v)) for v in x.reshape(-1)], np.float32).reshape(x.shape)


def adam(w, m, v, g, lr, b1, b2, eps, step):
    """One Adam step in place (FP32); b1^step and b2^step formed in FP32 by
    repeated multiplication."""
    b1t = np.float32(1.0)
    b2t = np.float32(1.0)
    for _ in range(step):
        b1t = np.float32(b1t * np.float32(b1))
        b2t = np.float32(b2t * np.float32(b2))
    lib().oracle_adam(_p(w), _p(m), _p(v), _p(np.ascontiguousarray(g, np.float32)), w.size, lr,
                      b1, b2, eps, float(b1t), float(b2t))
