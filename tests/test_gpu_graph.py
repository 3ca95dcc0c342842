"""Frame runs captured in a HIP graph (through torch.cuda.CUDAGraph): a run
only launches kernels (plans allocate and upload at creation, the persistent
aggregation returns its task counter to zero itself), so a captured frame
replays.  Each case replays three times, with eager work and synchronisations
between the replays, and every replay equals the eager run bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import lrnet, synth  # noqa: E402
from paper_1801_04720_amd._lib import SfAggTuning  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402

KEYS = ("disp0", "valid0", "disp1", "valid1", "sf4", "valid", "xyz0", "motion")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", ["plain", "persistent_packed", "learned"])
def test_frame_graph_replays_equal_eager(case):
    say("frame graph", case)
    H, W, D = 375, 1242, 128
    fr = synth.frame_1242x375(1)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    kw = {}
    if case == "persistent_packed":
        kw["tuning"] = SfAggTuning(4, 8, 0, 8, 1)
    if case == "learned":
        kw["learned_params"] = dev(lrnet.init_params(0))
    ff = FusedFrame(H, W, D, device=DEV, **kw)
    out = ff.run(*args)
    torch.cuda.synchronize()
    eager = {k: host(out[k]).copy() for k in KEYS}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ff.run(*args)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ff.run(*args)
    for rep in range(3):
        for v in ff.out.values():
            v.fill_(7)
        other = ff.run(*args) if rep == 1 else None  # eager work between replays
        torch.cuda.synchronize()
        if other is not None:
            for v in ff.out.values():
                v.fill_(3)
        g.replay()
        torch.cuda.synchronize()
        for k in KEYS:
            assert np.array_equal(host(ff.out[k]), eager[k], equal_nan=True), (case, rep, k)
