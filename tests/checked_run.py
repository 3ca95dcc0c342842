"""Runs the library's data-dependent paths on the GPU and saves their outputs
(npz at argv[1]), then prints one JSON line with sf_debug_check's bits and the
self-test's.  tests/test_gpu_checked.py runs it once with the checked library
(SF_LIB_PATH) and compares the outputs with those of the normal library."""
import ctypes as ct
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1801_04720_amd import _lib, api, lrnet, synth  # noqa: E402
from paper_1801_04720_amd._lib import SfAggTuning  # noqa: E402
from paper_1801_04720_amd.pipeline import FusedFrame, PlainFrame, SequenceFrames  # noqa: E402

DEV = "cuda:0"


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def bits(lib, clear=1):
    b = ct.c_uint32(0)
    _lib.check(lib.sf_debug_check(ct.byref(b), clear))
    return int(b.value)


def run(out_path):
    lib = _lib.lib()
    res = {"checked": int(lib.sf_debug_checked()), "before": bits(lib)}
    _lib.check(lib.sf_debug_selftest(1000, None))
    res["selftest"] = bits(lib)
    res["after_clear"] = bits(lib)
    out = {}
    # Plain frame at 1242x375 D=128 (flow within +-100 px: taps at every border),
    # byte and packed costs, persistent; learned and diagonal frames.
    fr = synth.frame_1242x375(0)
    args = [t(fr.t0.left), t(fr.t0.right), t(fr.t1.left), t(fr.t1.right), t(fr.flow)]
    for name, ff in (("plain", FusedFrame(375, 1242, 128, device=DEV)),
                     ("packed", FusedFrame(375, 1242, 128, tuning=SfAggTuning(4, 8, 0, 8, 1), device=DEV)),
                     ("learned", FusedFrame(375, 1242, 128, learned_params=t(lrnet.init_params(0)), device=DEV)),
                     ("diag", FusedFrame(375, 1242, 128, diag=True, device=DEV))):
        o = ff.run(*args)
        for k in ("valid0", "disp0", "valid1", "sf4", "valid"):
            out[f"{name}_{k}"] = o[k].cpu().numpy()
    # Per-stage path (S materialised, both epilogues, census mode, adaptive P2).
    pf = PlainFrame(375, 1242, 128, device=DEV)
    m0, m1, o = pf.run(*args)
    out["stages_valid"] = o["valid"].cpu().numpy()
    cl, cr = api.census(args[0]), api.census(args[1])
    for right, (cb, cm) in ((0, (cl, cr)), (1, (cr, cl))):
        out[f"census_agg_{right}"] = api.sgm_aggregate_census(cb, cm, 128, right, 10, 120)[::37, ::41].cpu().numpy()
    api.sgm_set_epilogue(2)
    out["atomic_S"] = api.sgm_aggregate(api.cost(cl, cr, 128, False), 10, 300)[::37, ::41].cpu().numpy()
    api.sgm_set_epilogue(0)
    out["adaptive_S"] = api.sgm_aggregate_adaptive(api.cost(cl, cr, 128, False), args[0], 10, 120)[::37, ::41].cpu().numpy()
    # Densification, flow stand-in, a short sequence with the temporal check.
    d = api.densify(o["sf4"], o["valid"])
    out["dense"] = d["sf4"].cpu().numpy()
    f = api.flow(args[0], args[2], levels=5, iters=2, fine_radius=8)
    out["flow"] = f["flow"].cpu().numpy()
    sq = synth.sequence_planar(synth.rng_for(6, 0), 4, 96, 320, 32, 20.0)
    seq = SequenceFrames([t(p.left) for p in sq.pairs], [t(p.right) for p in sq.pairs], 32, device=DEV)
    _, sfs, tm = seq.run([t(x) for x in sq.flows])
    out["temporal"] = np.stack([m.cpu().numpy() for m in tm])
    # Degenerate shapes.
    for H, W in ((1, 1), (7, 9), (3, 200)):
        rng = np.random.default_rng(H * 100 + W)
        L = rng.integers(0, 256, (H, W), dtype=np.uint8)
        R = rng.integers(0, 256, (H, W), dtype=np.uint8)
        flw = rng.uniform(-3 * W, 3 * W, (H, W, 2)).astype(np.float32)
        p = PlainFrame(H, W, 32, device=DEV)
        _, _, od = p.run(t(L), t(R), t(R), t(L), t(flw))
        out[f"tiny_{H}x{W}"] = od["valid"].cpu().numpy()
    torch.cuda.synchronize()
    res["workloads"] = bits(lib)
    np.savez(out_path, **out)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    run(sys.argv[1])
