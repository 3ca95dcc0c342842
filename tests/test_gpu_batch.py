"""Batched plain SGM over uneven pairs: every pair equals the oracle (small
sizes) or the per-pair C-ABI path (larger ones) bit for bit, whatever the
waves, tunings and schedule; the captured graph replays identically; the
autotuner returns a valid choice."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import api, batch, synth  # noqa: E402
from paper_1801_04720_amd._lib import SfAggTuning  # noqa: E402

from gpu_util import DEV, assert_close_rel, dev, host  # noqa: E402

SIZES = [(48, 160, 32), (61, 203, 64), (40, 97, 96), (33, 300, 256), (48, 160, 32), (61, 203, 64)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_pairs(sizes, cfg=7):
    pairs, host_pairs = [], []
    for i, (H, W, D) in enumerate(sizes):
        p = synth.pair_planar(synth.rng_for(cfg, i), H, W, D)
        host_pairs.append(p)
        pairs.append({"left": dev(p.left), "right": dev(p.right), "D": D})
    return pairs, host_pairs


def per_pair_gpu(p):
    L, R, D = p["left"], p["right"], p["D"]
    cl, cr = api.census(L), api.census(R)
    Sr = api.sgm_aggregate(api.cost(cr, cl, D, True), 10, 120)
    Sl = api.sgm_aggregate(api.cost(cl, cr, D, False), 10, 120)
    return api.wta_lr(Sl, Sr, None, 120, 1)


def test_batch_vs_oracle(orc):
    say("batch vs oracle")
    pairs, hp = make_pairs(SIZES)
    b = batch.Batch(pairs)
    out = b.run()
    torch.cuda.synchronize()
    for o, p in zip(out, hp):
        w, d, v = orc.disparity(p.left, p.right, p.D)
        assert np.array_equal(host(o["wta"]), w)
        assert np.array_equal(host(o["valid"]), v)
        assert_close_rel(host(o["disp"]), d, 1.0)


@pytest.mark.parametrize("cpb,pf,order,pers,packed", [(4, 4, 0, 0, 0), (8, 8, 1, 0, 1), (16, 4, 1, 4, 0),
                                                      (4, 8, 0, 8, 1), (16, 8, 0, 2, 1)])
def test_batch_tunings_and_waves_identical(cpb, pf, order, pers, packed):
    """Every tuning, 6-bit packed costs included (used by the D = 256 pairs),
    gives the default plan's maps bit for bit."""
    say("batch tuning", cpb, pf, order, pers, packed)
    pairs, _ = make_pairs(SIZES)
    ref = [{k: host(v).copy() for k, v in o.items()} for o in batch.Batch(pairs).run()]
    t = SfAggTuning(cpb, pf, order, pers, packed)
    b = batch.Batch(pairs, tunings=[t] * 4, mem_budget=8 << 20)  # tiny budget: several waves
    assert b.nwaves > 1
    for rep in range(2):  # twice: a persistent launch leaves its task counter at zero
        for o in b.out:
            for v in o.values():
                v.fill_(7)
        out = b.run()
        torch.cuda.synchronize()
        for o, r in zip(out, ref):
            for k in r:
                assert np.array_equal(host(o[k]), r[k]), (rep, k)


@pytest.mark.parametrize("tuning", [None, (8, 8, 0, 4, 1)])
def test_graph_replays_match_eager(tuning):
    """Replays of the captured batch equal the eager run, also with a persistent
    aggregation, whose task counter is reset by the launch itself (the graph
    holds no clearing node)."""
    say("batch graph", tuning)
    pairs, _ = make_pairs(SIZES[:4], cfg=8)
    b = batch.Batch(pairs, tunings=None if tuning is None else [SfAggTuning(*tuning)] * 4)
    eager = [{k: host(v).copy() for k, v in o.items()} for o in b.run()]
    s = torch.cuda.Stream()
    b.capture(s)
    for rep in range(3):
        for o in b.out:  # scribble over the outputs between replays
            for v in o.values():
                v.fill_(7)
        torch.cuda.synchronize()
        b.launch(s)
        s.synchronize()
        x = torch.ones(1000, device=DEV).sum()  # unrelated eager work in between
        torch.cuda.synchronize()
        assert float(x) == 1000.0
        for o, r in zip(b.out, eager):
            for k in r:
                assert np.array_equal(host(o[k]), r[k]), (rep, k)


def test_batch_uneven_classes_vs_per_pair_path():
    """The three size classes of the uneven batch (640x480/64, 1242x375/128,
    1920x1080/256), two pairs each, against the per-pair C-ABI path."""
    say("uneven batch size classes")
    sizes = [(480, 640, 64), (375, 1242, 128), (1080, 1920, 256)] * 2
    pairs, _ = make_pairs(sizes, cfg=3)
    b = batch.Batch(pairs, mem_budget=16 << 30)
    out = b.run()
    torch.cuda.synchronize()
    for o, p in zip(out, pairs):
        r = per_pair_gpu(p)
        torch.cuda.synchronize()
        assert np.array_equal(host(o["wta"]), host(r["wta_left"]))
        assert np.array_equal(host(o["valid"]), host(r["valid"]))
        assert np.array_equal(host(o["disp"]), host(r["disp"]))


def test_autotune_returns_valid_choice(tmp_path):
    say("autotune")
    t, ms = batch.autotune(96, 320, 32, cache=str(tmp_path / "at.json"))
    assert t.chains_per_block in (4, 8, 16) and t.prefetch in (4, 8)
    assert t.order in (0, 1) and 0 <= t.persistent_per_cu <= 8 and t.packed == 0  # D = 32: bytes
    assert ms > 0
    t2, ms2 = batch.autotune(96, 320, 32, cache=str(tmp_path / "at.json"))
    assert batch.tuning_dict(t2) == batch.tuning_dict(t)


def test_frame_autotune_returns_valid_choice(tmp_path):
    """Whole-frame tuner: a valid candidate, cached, and a frame with it equals the default plan's."""
    from paper_1801_04720_amd.pipeline import FusedFrame

    say("frame autotune")
    H, W, D = 48, 160, 128
    t, ms = batch.frame_autotune(H, W, D, cache=str(tmp_path / "ft.json"))
    assert t.chains_per_block in (4, 8, 16) and t.prefetch in (4, 8)
    assert t.order in (0, 1) and t.persistent_per_cu in (0, 4, 8) and t.packed in (0, 1)
    assert ms > 0
    t2, _ = batch.frame_autotune(H, W, D, cache=str(tmp_path / "ft.json"))
    assert batch.tuning_dict(t2) == batch.tuning_dict(t)
    fr = synth.frame_planar(synth.rng_for(8, 31), H, W, D, 10.0)
    args = [dev(a) for a in (fr.t0.left, fr.t0.right, fr.t1.left, fr.t1.right, fr.flow)]
    a = FusedFrame(H, W, D, device=DEV).run(*args)
    b = FusedFrame(H, W, D, tuning=t, device=DEV).run(*args)
    torch.cuda.synchronize()
    for k in ("disp0", "valid0", "disp1", "valid1", "valid"):
        assert np.array_equal(host(a[k]), host(b[k])), k
    assert np.array_equal(host(a["sf4"]), host(b["sf4"]), equal_nan=True)
