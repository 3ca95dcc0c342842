"""bench.py's scene-flow diagnostics (density over non-occluded pixels and the
causes of undefined pixels) on the oracle's own frame outputs: the three
causes are disjoint, they and the defined pixels cover the frame, and the
combination rule they restate gives the oracle's validity mask."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1801_04720_amd import synth  # noqa: E402


@pytest.mark.parametrize("seed", [3, 4])
def test_diagnostics_cover_the_frame(orc, seed):
    fr = synth.frame_planar(synth.rng_for(8, seed), 60, 200, 32, 20.0)
    _, d0, v0 = orc.disparity(fr.t0.left, fr.t0.right, 32)
    _, d1, v1 = orc.disparity(fr.t1.left, fr.t1.right, 32)
    _, valid = orc.combine(d0, v0, d1, v1, fr.flow)
    dg = bench.sceneflow_diagnostics(fr, v0, v1, valid)
    assert dg["rule_matches_kernel"]
    undefined = (dg["undefined_flow_leaves_image"] + dg["undefined_t0_disparity_rejected"]
                 + dg["undefined_t1_disparity_rejected"])
    assert abs((1.0 - undefined) - (valid & 1).mean()) < 1e-12
    assert dg["undefined_flow_leaves_image"] > 0  # flows up to 20 px leave a 200 px wide frame
    assert 0.5 < dg["noc_fraction"] < 1.0
    assert dg["sceneflow_density_noc"] >= (valid & 1).mean()
