"""Optical-flow stand-in on the GPU against the oracle (bit-exact integer flows)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, synth  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def crop_pair(seed, H, W):
    fr = synth.frame_1242x375(seed)
    return (np.ascontiguousarray(fr.t0.left[:H, :W]), np.ascontiguousarray(fr.t1.left[:H, :W]))


def check(orc, A, B, **kw):
    got = api.flow(dev(A), dev(B), **kw)
    torch.cuda.synchronize()
    F, Bk, out = orc.flow(A, B, **kw)
    assert np.array_equal(host(got["F"]), F)
    assert np.array_equal(host(got["B"]), Bk)
    assert np.array_equal(host(got["flow"]), out, equal_nan=True)


@pytest.mark.parametrize("H,W,levels,iters,R,seed,fine", [
    (1, 1, 1, 1, 1, 0, 0), (1, 40, 2, 2, 8, 1, 0), (37, 1, 2, 2, 8, 2, 2), (13, 17, 3, 3, 16, 3, 0),
    (96, 160, 4, 3, 64, 4, 0), (96, 160, 4, 3, 64, 4, 4), (97, 161, 5, 2, 128, 5, 8),
    (64, 200, 1, 4, 32, 6, 3)])
def test_flow_small_vs_oracle(orc, H, W, levels, iters, R, seed, fine):
    say("flow", H, W, levels, iters, R, seed, fine)
    A, B = crop_pair(seed % 3, H, W)
    check(orc, A, B, levels=levels, iters=iters, R=R, seed=seed, tol=1, fine_radius=fine)


def test_flow_pitch_and_tolerance(orc):
    say("flow pitch / tol")
    A, B = crop_pair(1, 50, 90)
    wideA = np.zeros((50, 128), np.uint8)
    wideB = np.zeros((50, 128), np.uint8)
    wideA[:, :90], wideB[:, :90] = A, B
    # Row pitch 128 > W = 90: through the C ABI, which takes the pitch explicitly.
    import ctypes as ct
    from paper_1801_04720_amd import _lib
    ta, tb = dev(wideA), dev(wideB)
    F = torch.empty((50, 90, 2), dtype=torch.int16, device=DEV)
    Bk = torch.empty_like(F)
    fl = torch.empty((50, 90, 2), dtype=torch.float32, device=DEV)
    ws = torch.empty(_lib.lib().sf_flow_workspace_bytes(50, 90, 3), dtype=torch.uint8, device=DEV)
    _lib.check(_lib.lib().sf_flow(ct.c_void_p(ta.data_ptr()), ct.c_void_p(tb.data_ptr()), 128, 50, 90, 3, 3,
                                  32, 4, 77, 0, ct.c_void_p(F.data_ptr()), ct.c_void_p(Bk.data_ptr()),
                                  ct.c_void_p(fl.data_ptr()), ct.c_void_p(ws.data_ptr()), ws.numel(),
                                  ct.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    eF, eB, eo = orc.flow(A, B, levels=3, iters=3, R=32, seed=77, tol=0, fine_radius=4)
    assert np.array_equal(host(F), eF) and np.array_equal(host(Bk), eB)
    assert np.array_equal(host(fl), eo, equal_nan=True)


@pytest.mark.parametrize("fine", [0, 8])
def test_flow_full_size_vs_oracle(orc, fine):
    """1242x375 frame, 5 levels, 2 iterations per level, R = 128."""
    say("flow 1242x375 vs oracle", fine)
    fr = synth.frame_1242x375(0)
    check(orc, fr.t0.left, fr.t1.left, levels=5, iters=2, R=128, seed=1801, tol=1, fine_radius=fine)


def test_flow_translation_on_gpu():
    say("flow translation")
    rng = np.random.default_rng(5)
    big = rng.integers(0, 256, (180, 300)).astype(np.uint8)
    A = np.ascontiguousarray(big[20:160, 20:280])
    B = np.ascontiguousarray(big[23:163, 11:271])  # A(x, y) = B(x + 9, y - 3): flow (+9, -3)
    got = api.flow(dev(A), dev(B), levels=4, iters=8, R=64)
    F = host(got["F"])
    inner = (slice(14, 140 - 14), slice(20, 260 - 20))
    assert (F[inner][..., 0] == 9).all() and (F[inner][..., 1] == -3).all()


def test_frame_with_computed_flow(orc):
    """Scene flow from the GPU flow stand-in: the combination sees NaN where the
    consistency check dropped the flow and leaves S undefined there."""
    say("frame with computed flow")
    fr = synth.frame_planar(synth.rng_for(8, 21), 64, 200, 64, 12.0)
    L0, R0, L1, R1 = (dev(a) for a in (fr.t0.left, fr.t0.right, fr.t1.left, fr.t1.right))
    fl = api.flow(L0, L1, levels=3, iters=4, R=32)["flow"]
    ff = FusedFrame(64, 200, 64, device=DEV)
    got = ff.run(L0, R0, L1, R1, fl)
    torch.cuda.synchronize()
    _, _, eflow = orc.flow(fr.t0.left, fr.t1.left, levels=3, iters=4, R=32)
    w0, d0, v0 = orc.disparity(fr.t0.left, fr.t0.right, 64)
    w1, d1, v1 = orc.disparity(fr.t1.left, fr.t1.right, 64)
    sf4, valid, xyz0, motion = orc.combine(d0, v0, d1, v1, eflow, ff.cam)
    assert np.array_equal(host(got["valid"]), valid)
    assert np.array_equal(host(got["sf4"]), sf4, equal_nan=True)
    assert not (host(got["valid"])[np.isnan(eflow[..., 0])] & 1).any()
