"""Densification of the sparse scene-flow map on the GPU against the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, synth  # noqa: E402
from paper_1801_04720_amd.evaluate import sf_outliers  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402
from test_gpu_variants import oracle_frame_ex  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("H,W,density", [(1, 1, 1.0), (1, 1, 0.0), (1, 300, 0.05), (40, 1, 0.3),
                                         (37, 203, 0.0), (37, 203, 0.02), (37, 203, 0.5),
                                         (37, 203, 1.0), (3, 8192, 0.01), (375, 1242, 0.8)])
def test_densify_random(orc, H, W, density):
    say("densify", H, W, density)
    rng = np.random.default_rng(H * 13 + W + int(100 * density))
    valid = (rng.random((H, W)) < density).astype(np.uint8)
    if H > 4:
        valid[rng.integers(0, H, H // 4)] = 0  # empty rows
    sf4 = rng.normal(0, 30, (H, W, 4)).astype(np.float32)
    sf4[..., 2] = np.round(sf4[..., 2])  # ties in d0
    sf4[valid == 0] = np.nan
    got = api.densify(dev(sf4), dev(valid))
    out, fill = orc.densify(sf4, valid)
    assert np.array_equal(host(got["fill"]), fill)
    assert np.array_equal(host(got["sf4"]), out, equal_nan=True)


def test_densify_frame_1242x375(orc):
    say("densify a 1242x375 D=128 frame")
    fr = synth.frame_1242x375(7)
    ff = FusedFrame(375, 1242, 128, device=DEV)
    got = ff.run(dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow))
    dense = api.densify(got["sf4"], got["valid"])
    torch.cuda.synchronize()
    ref = oracle_frame_ex(orc, fr, 128, ff.cam, 0)
    out, fill = orc.densify(ref["sf4"], ref["valid"])
    assert np.array_equal(host(dense["fill"]), fill)
    assert np.array_equal(host(dense["sf4"]), out, equal_nan=True)
    est = sf_outliers(got["sf4"], got["valid"] & 1, fr.gt_flow, fr.t0.gt_disp, fr.gt_disp1_at_t0)
    full = sf_outliers(dense["sf4"], dense["fill"] > 0, fr.gt_flow, fr.t0.gt_disp, fr.gt_disp1_at_t0)
    say("Est", est, "All", full)
    assert full["density"] == 1.0 and 0.5 < est["density"] < 1.0
