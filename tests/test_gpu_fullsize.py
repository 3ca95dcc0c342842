"""The largest workloads against the oracle, whole arrays: the plain frame at
2048x1024 D=256 (the stream's frame size) under the packed-cost tunings the
stream runs, a 400x600 D=256 frame with packed costs (the smallest width at which
the packed cost writer's interior tiles run for both bases), and a batch
holding the three pair sizes of the uneven batch, 1920x1080 D=256 included, in
the graph-captured launch the batch bench times, with packed costs for the
D = 128 and 256 classes.  The oracle computes each view in its own thread."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import synth  # noqa: E402
from paper_1801_04720_amd._lib import SfAggTuning  # noqa: E402
from paper_1801_04720_amd.batch import Batch  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame  # noqa: E402

import oracle_maps  # noqa: E402
from gpu_util import DEV, assert_close_rel, dev, host  # noqa: E402
from test_gpu_frame import check_frame, oracle_frame_par  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("H,W,tunings", [
    (400, 600, [(16, 8, 0, 0, 1), (4, 8, 1, 8, 1)]),
    (1024, 2048, [(8, 4, 1, 4, 1), (16, 8, 0, 0, 1)]),
])
def test_frame_d256_packed_vs_oracle(orc, H, W, tunings):
    fr = synth.frame_planar(synth.rng_for(5, 3 if W == 2048 else 7), H, W, 256, 200.0 if W == 2048 else 60.0)
    args = [dev(fr.t0.left), dev(fr.t0.right), dev(fr.t1.left), dev(fr.t1.right), dev(fr.flow)]
    ref = None
    for t in tunings:
        ff = FusedFrame(H, W, 256, tuning=SfAggTuning(*t), device=DEV)
        if ref is None:
            say(f"oracle for the {W}x{H} D=256 frame (four views in parallel)")
            ref = oracle_frame_par(orc, fr, 256, ff.cam)
        for rep in range(2 if t[3] else 1):
            say(f"frame {W}x{H} D=256, tuning {t}, run {rep}")
            for v in ff.out.values():
                v.fill_(7)
            got = ff.run(*args)
            torch.cuda.synchronize()
            check_frame(got, ref)


def test_uneven_batch_graph_vs_oracle(orc):
    say("uneven batch (640x480/64, 1242x375/128, 1920x1080/256) in one graph vs oracle")
    sizes = [(480, 640, 64), (375, 1242, 128), (1080, 1920, 256)]
    pairs = [synth.pair_batch(i, *s) for i, s in enumerate(sizes)]
    ts = [{"left": dev(p.left), "right": dev(p.right), "D": s[2]} for p, s in zip(pairs, sizes)]
    say("  oracle, 6 views in parallel")
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=3) as ex:
        refs = list(ex.map(lambda ps: oracle_maps.maps(orc, [(ps[0].left, ps[0].right)], ps[1][2], threads=2)[0],
                           zip(pairs, sizes)))
    tuning_sets = [
        {sizes[0][:2] + (64,): SfAggTuning(8, 4, 0, 0, 0), (375, 1242, 128): SfAggTuning(16, 8, 0, 0, 1),
         (1080, 1920, 256): SfAggTuning(4, 8, 1, 8, 1)},
        {sizes[0][:2] + (64,): SfAggTuning(8, 4, 0, 0, 0), (375, 1242, 128): SfAggTuning(4, 8, 0, 4, 0),
         (1080, 1920, 256): SfAggTuning(16, 8, 0, 0, 1)},
    ]
    for tun in tuning_sets:
        b = Batch(ts, tunings=tun, device=DEV)
        st = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            b.capture(st)
            for rep in range(2):
                say("  graph launch", rep, "tunings", {k: (t.chains_per_block, t.persistent_per_cu, t.packed)
                                                       for k, t in tun.items()})
                for o in b.out:
                    for v in o.values():
                        v.fill_(7)
                out = b.launch(st)
                torch.cuda.synchronize()
                for s, o, r in zip(sizes, out, refs):
                    assert np.array_equal(host(o["wta"]), r["wta_left"]), s
                    assert np.array_equal(host(o["valid"]), r["valid"]), s
                    assert_close_rel(host(o["disp"]), r["disp"], 1.0, what=f"disp {s}")
