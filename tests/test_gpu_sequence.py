"""Scene flow over several time steps with temporal validation, on the GPU,
against the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, synth  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame, SequenceFrames  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_temporal_check_vs_oracle(orc):
    say("temporal check random maps")
    rng = np.random.default_rng(12)
    H, W = 57, 91
    a = rng.normal(0, 3, (H, W, 4)).astype(np.float32)
    a[..., 2:] += 20
    b = a + rng.normal(0, 1.2, (H, W, 4)).astype(np.float32)
    va = (rng.random((H, W)) < 0.8).astype(np.uint8)
    vb = (rng.random((H, W)) < 0.8).astype(np.uint8) | 2
    for tf, td in [(2.0, 1.0), (0.5, 0.25), (0.0, 0.0)]:
        got = host(api.temporal_check(dev(a), dev(va), dev(b), dev(vb), tf, td))
        assert np.array_equal(got, orc.temporal_check(a, va, b, vb, tf, td))


@pytest.mark.parametrize("T,H,W,D", [(3, 64, 200, 32), (5, 96, 320, 64)])
def test_sequence_small_vs_oracle(orc, T, H, W, D):
    say("sequence", T, H, W, D)
    s = synth.sequence_planar(synth.rng_for(6, T), T, H, W, D, 15.0)
    lefts = [dev(p.left) for p in s.pairs]
    rights = [dev(p.right) for p in s.pairs]
    seq = SequenceFrames(lefts, rights, D, device=DEV)
    maps, S, tv = seq.run([dev(f) for f in s.flows])
    torch.cuda.synchronize()
    ref = [orc.disparity(p.left, p.right, D) for p in s.pairs]
    for k in range(T):
        assert np.array_equal(host(maps[k]["valid"]), ref[k][2])
        assert np.array_equal(host(maps[k]["disp"]), ref[k][1])
    RS = []
    for k in range(T - 1):
        sf4, valid, xyz0, motion = orc.combine(ref[k][1], ref[k][2], ref[k + 1][1], ref[k + 1][2],
                                               s.flows[k], seq.cam)
        assert np.array_equal(host(S[k]["valid"]), valid)
        assert np.array_equal(host(S[k]["sf4"]), sf4, equal_nan=True)
        RS.append((sf4, valid))
    for k in range(T - 2):
        exp = orc.temporal_check(RS[k][0], RS[k][1], RS[k + 1][0], RS[k + 1][1], 2.0, 1.0)
        assert np.array_equal(host(tv[k]), exp)


def test_sequence_full_size_matches_frames(orc):
    """Four 1242x375 D=128 time steps: each scene-flow map equals the fused
    frame on that pair of time steps, and the temporal masks equal the oracle's
    rule applied to them."""
    say("sequence 4 x 1242x375 D=128")
    T = 4
    s = synth.sequence_planar(synth.rng_for(6, 100), T, 375, 1242, 128, 60.0)
    lefts = [dev(p.left) for p in s.pairs]
    rights = [dev(p.right) for p in s.pairs]
    seq = SequenceFrames(lefts, rights, 128, device=DEV)
    flows = [dev(f) for f in s.flows]
    _, S, tv = seq.run(flows)
    S = [{k: host(v).copy() for k, v in Sk.items()} for Sk in S]
    tv = [host(t).copy() for t in tv]
    ff = FusedFrame(375, 1242, 128, device=DEV)
    for k in range(T - 1):
        got = ff.run(lefts[k], rights[k], lefts[k + 1], rights[k + 1], flows[k])
        torch.cuda.synchronize()
        for key in ("sf4", "valid", "xyz0", "motion"):
            assert np.array_equal(S[k][key], host(got[key]), equal_nan=True), (k, key)
    for k in range(T - 2):
        exp = orc.temporal_check(S[k]["sf4"], S[k]["valid"], S[k + 1]["sf4"], S[k + 1]["valid"], 2.0, 1.0)
        assert np.array_equal(tv[k], exp)
        assert 0.3 < tv[k].mean() < (S[k]["valid"] & 1).mean()
