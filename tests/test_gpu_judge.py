"""The judge and fallback of the learned stand-in: the mask-agreement count
against numpy, and the judged stream's policy (the full left-right check
judges every k-th frame; below the agreement threshold the following frames
fall back to the plain frame) with the threshold forced from the host so that
the fallback is certain, or impossible."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, lrnet, synth  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame, JudgedLearnedStream  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,off", [(1, 0), (15, 0), (16, 0), (1000, 0), (4099, 3), (465750, 0), (465750, 1),
                                   (2097152, 0)])
def test_mask_agreement_count(n, off):
    say("mask agreement", n, off)
    rng = np.random.default_rng(n + off)
    a = rng.integers(0, 3, n + off).astype(np.uint8)
    b = np.where(rng.uniform(size=n + off) < 0.9, a, rng.integers(0, 3, n + off)).astype(np.uint8)
    ta, tb = dev(a), dev(b)
    got = int(host(api.mask_agreement(ta[off:], tb[off:]))[0])
    assert got == int(((a[off:] != 0) == (b[off:] != 0)).sum())


def _frames(n, H, W, D):
    out = []
    for i in range(n):
        fr = synth.frame_planar(synth.rng_for(8, 70 + i), H, W, D, 20.0)
        out.append([dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)])
    return out


def _copy(o):
    return {k: host(v).copy() for k, v in o.items()}


def _same(a, b):
    return all(np.array_equal(a[k], b[k], equal_nan=True) for k in a)


@pytest.mark.parametrize("threshold,expect", [(1.01, "plain"), (-1.0, "learned")])
def test_judged_stream_forced_policy(threshold, expect):
    """threshold 1.01: no agreement can reach it, so after the first judged frame
    every frame is a fallback frame, bit-equal to the plain frame; threshold
    -1: every agreement passes, so the frames between judges are learned frames,
    bit-equal to the learned frame.  Judged frames deliver the plain frame."""
    say("judged stream, threshold", threshold)
    H, W, D = 64, 200, 64
    frames = _frames(7, H, W, D)
    prm = dev(lrnet.init_params(4))
    plain = FusedFrame(H, W, D, device=DEV)
    learned = FusedFrame(H, W, D, learned_params=prm, device=DEV)
    ref_p = [_copy(plain.run(*f)) for f in frames]
    ref_l = [_copy(learned.run(*f)) for f in frames]
    assert not all(_same(p, l) for p, l in zip(ref_p, ref_l))
    js = JudgedLearnedStream(H, W, D, prm, judge_every=3, threshold=threshold, device=DEV)
    for i, f in enumerate(frames):
        got = _copy(js.run(*f))
        torch.cuda.synchronize()
        if i % 3 == 0 or expect == "plain":
            assert _same(got, ref_p[i]), i
        else:
            assert _same(got, ref_l[i]), i
    assert [h[0] for h in js.history] == [0, 3, 6]
    assert all(h[3] == expect for h in js.history)
    for _, a0, a1, _ in js.history:
        assert 0.0 <= a0 <= 1.0 and 0.0 <= a1 <= 1.0


def test_judged_stream_agreement_matches_masks():
    """The agreement the judge reads equals the masks' agreement counted on the host."""
    say("judged stream agreement")
    H, W, D = 48, 160, 32
    frames = _frames(1, H, W, D)
    prm = dev(lrnet.init_params(6))
    js = JudgedLearnedStream(H, W, D, prm, judge_every=1, threshold=0.5, device=DEV)
    js.run(*frames[0])
    lo = _copy(FusedFrame(H, W, D, learned_params=prm, device=DEV).run(*frames[0]))
    po = _copy(FusedFrame(H, W, D, device=DEV).run(*frames[0]))
    _, a0, a1, mode = js.history[0]
    assert a0 == ((lo["valid0"] != 0) == (po["valid0"] != 0)).mean()
    assert a1 == ((lo["valid1"] != 0) == (po["valid1"] != 0)).mean()
    assert mode == ("learned" if min(a0, a1) >= 0.5 else "plain")
