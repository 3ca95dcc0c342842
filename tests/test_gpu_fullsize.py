"""The largest workloads against the oracle.  Whole arrays: the plain frame at
2048x1024 D=256 (the stream's frame size) under the packed-cost tunings the
stream runs, a 400x600 D=256 frame with packed costs (the smallest width at which
the packed cost writer's interior tiles run for both bases), and a batch
holding the three pair sizes of the uneven batch, 1920x1080 D=256 included, in
the graph-captured launch the batch bench times, with packed costs for the
D = 128 and 256 classes.  The oracle computes each view in its own thread.
Sampled pixels: the largest volume the entry points accept (2047 x 4096 x 256,
just under 2^31 cells per view), for the aggregation calls and the fused frame."""
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


@pytest.mark.parametrize("right", [0, 1])
def test_largest_volume_sampled(orc, right):
    """The largest volume the aggregation entry points accept (2047 x 4096 x 256,
    just under 2^31 cells, so S takes 4.3 GB): cost volume + aggregation with
    both output stages and the census mode give the same S, and S and the WTA
    disparity at sampled pixels (corners, every edge, the last row, the
    interior) equal the oracle's path recurrences into those pixels."""
    from paper_1801_04720_amd import api

    H, W, D = 2047, 4096, 256
    assert H * W * D < 2 ** 31 <= (H + 1) * W * D  # one more row would pass the limit
    say("largest volume", H, W, D, "right base", right)
    rng = np.random.default_rng(2047 + right)
    L = rng.integers(0, 256, (H, W), dtype=np.uint8)
    R = np.roll(L, -17, axis=1) // 2 + rng.integers(0, 128, (H, W), dtype=np.uint8)
    cl, cr = api.census(dev(L)), api.census(dev(R))
    cb, cm = (cr, cl) if right else (cl, cr)
    C = api.cost(cb, cm, D, bool(right))
    ws = torch.empty(api.sgm_workspace_bytes(H, W, D), dtype=torch.uint8, device=DEV)
    S = api.sgm_aggregate(C, 10, 120, workspace=ws)
    S2 = api.sgm_aggregate_census(cb, cm, D, right, 10, 120, workspace=ws)
    assert torch.equal(S, S2)
    del S2
    api.sgm_set_epilogue(2)
    try:
        S3 = api.sgm_aggregate(C, 10, 120, workspace=ws)
    finally:
        api.sgm_set_epilogue(0)
    assert torch.equal(S, S3)
    del S3, C, ws
    out = api.wta_lr(S, None, None, 120, 1)
    wta = host(out["wta_left"])
    cbh, cmh = host(cb, np.uint64), host(cm, np.uint64)
    pts = [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1), (2048, 0), (2048, H - 1), (0, 1023), (W - 1, 1023),
           (255, 1), (W - 256, H - 2), (3001, 1500), (17, 2000)]
    for x, y in pts:
        ref = orc.aggregate_at(cbh, cmh, D, right, 10, 120, x, y)
        got = host(S[y, x], np.uint16)
        assert np.array_equal(got, ref), (x, y)
        assert int(wta[y, x]) == int(np.argmin(ref)), (x, y)


def test_largest_frame_sampled(orc):
    """The fused frame at the largest size its plan accepts (2047 x 4096, D = 256;
    each view's volume just under 2^31 cells, 4 views in one aggregation
    launch), with byte costs and with the packed persistent tuning: the LR-checked
    maps of both time steps at sampled pixels (corners, every edge, the
    interior) equal the oracle's."""
    H, W, D = 2047, 4096, 256
    rng = np.random.default_rng(4096)

    def pair(shift):
        L = rng.integers(0, 256, (H, W), dtype=np.uint8)
        R = (np.roll(L, -shift, axis=1) // 4 * 3 + rng.integers(0, 64, (H, W), dtype=np.uint8)).astype(np.uint8)
        return L, R

    (L0, R0), (L1, R1) = pair(17), pair(40)
    flow = np.zeros((H, W, 2), np.float32)
    args = [dev(L0), dev(R0), dev(L1), dev(R1), dev(flow)]
    xs = np.array([0, W - 1, 0, W - 1, 2048, 2048, 0, W - 1, 255, W - 256, 3001, 17, 600], np.int32)
    ys = np.array([0, 0, H - 1, H - 1, 0, H - 1, 1023, 1023, 1, H - 2, 1500, 2000, 777], np.int32)
    say("largest frame: oracle samples")
    refs = [orc.disparity_at(L0, R0, D, xs, ys), orc.disparity_at(L1, R1, D, xs, ys)]
    for t in [None, (4, 8, 1, 8, 1)]:
        say("largest frame", H, W, D, "tuning", t)
        ff = FusedFrame(H, W, D, tuning=SfAggTuning(*t) if t else None, device=DEV)
        got = ff.run(*args)
        torch.cuda.synchronize()
        for k, (_, rdisp, rvalid) in zip((0, 1), refs):
            v = host(got[f"valid{k}"])[ys, xs]
            d = host(got[f"disp{k}"])[ys, xs]
            assert np.array_equal(v, rvalid), (k, v, rvalid)
            assert_close_rel(d, rdisp, 1.0, what=f"disp{k}")
        assert host(got["valid0"]).mean() > 0.05  # not a degenerate all-invalid case
        del ff, got
        torch.cuda.empty_cache()
