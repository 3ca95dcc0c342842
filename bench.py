"""Benchmark of the scene-flow hot path on one MI355X.

A step is one plain scene-flow frame at 1242x375, D = 128 (the KITTI frame
shape): census of the four images, left- and right-base cost volumes and
8-path aggregations for t0 and t1, WTA + sub-pixel + LR check for both time
steps, then the combination with the flow and triangulation.  Inputs are
seeded synthetic frames already resident in HBM when the timed region starts.

Prints one JSON line.  `value` is GCUPS per delivered disparity map
(2 maps x W*H*D*8 cell updates per frame / frame time).
"""
from __future__ import annotations

import argparse
import ctypes as ct
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS (W·H·D·8 paths/s) + scene-flow fps @1242×375 D=128, plain vs learned"
PEAK_U16_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # packed-u16 VALU element ops/s, 78.6 T
PEAK_HBM_GBS = 8000.0


def kernel_ms(lib, name):
    import ctypes as ct

    tot = ct.c_double(0.0)
    n = ct.c_int(0)
    rc = lib.sf_prof_query(name.encode(), ct.byref(tot), ct.byref(n))
    if rc != 0:
        raise RuntimeError(lib.sf_last_error().decode())
    return tot.value, n.value


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "sgm_tasks_frame_1242x375_traffic.json")
# The aggregation kernel and the frame plan that builds its task table.
TRAFFIC_SOURCES = ["paper_1801_04720_amd/csrc/sgm.hip", "paper_1801_04720_amd/csrc/sgm_tasks.hpp",
                   "paper_1801_04720_amd/csrc/sf_internal.hpp", "paper_1801_04720_amd/csrc/frame.hip"]
SWEEP_FRAMES = 2   # frames per tuning in --tuning-sweep; the counters of the last one are kept
# Where the bench legs cache the autotuners' choices (machine-specific, not part of the
# repository); later runs on the same machine reuse them.
TUNE_CACHE = os.environ.get("SF_TUNE_CACHE", os.path.join(ROOT, ".tune_cache", "autotune_cache.json"))


def tuning_candidates():
    """The 72 aggregation tunings (chains_per_block, prefetch, order,
    persistent_per_cu, packed) in the order sf_frame_autotune tries them at
    D = 128 (packed costs are a candidate where D is 128 or 256)."""
    return [(cpb, pf, order, pp, pk) for pk in (0, 1) for cpb in (4, 8, 16) for order in (0, 1)
            for pf in (4, 8) for pp in (0, 4, 8)]


def _sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, tuning):
    """HBM-side bytes per launch of the aggregation kernel under this tuning
    (a (chains_per_block, prefetch, order, persistent_per_cu, packed) tuple) from the
    committed counter table, only if the kernel sources are unchanged since the
    counters were taken; None otherwise."""
    if not kernel.startswith("sgm_tasks") or not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        rec = json.load(f)
    if rec.get("sources") != TRAFFIC_SOURCES or rec.get("sources_sha256") != _sources_sha256():
        return None
    e = rec.get("by_tuning", {}).get(",".join(str(v) for v in tuning))
    return e["traffic_bytes_per_launch"] if e else None


def _pmc_per_dispatch(db, counter):
    """(dispatch id, kernel name, value) of one counter from a rocprofv3 results
    database, in dispatch order."""
    import sqlite3

    con = sqlite3.connect(db)
    try:
        return con.execute("select dispatch_id, name, counter_value from pmc_events "
                           "where counter_name = ? order by dispatch_id", (counter,)).fetchall()
    finally:
        con.close()


def write_traffic_table(fetch_db, write_db, out=TRAFFIC_JSON):
    """Turn the FETCH_SIZE and WRITE_SIZE passes over `bench.py --tuning-sweep`
    into the per-tuning traffic table: each counter is scaled by what it reads
    for the sweep's own 1 GiB copies (known to move 1 GiB each way)."""
    f, w = _pmc_per_dispatch(fetch_db, "FETCH_SIZE"), _pmc_per_dispatch(write_db, "WRITE_SIZE")
    kib = 1 << 20  # KiB in 1 GiB

    def copies(rows):
        v = sorted((x for _, n, x in rows if "copyBuffer" in n), reverse=True)[:3]
        if len(v) < 3:
            raise SystemExit("bench.py: fewer than three 1 GiB copies in the counter pass")
        return sum(v) / len(v)

    cf, cw = copies(f), copies(w)
    ff, fw = kib / cf, kib / cw
    ag_f = [x for _, n, x in f if "sgm_tasks_kernel" in n]
    ag_w = [x for _, n, x in w if "sgm_tasks_kernel" in n]
    names = sorted({n.split("(")[0] for _, n, _x in f if "sgm_tasks_kernel" in n})
    cand = tuning_candidates()
    if len(ag_f) != SWEEP_FRAMES * len(cand) or len(ag_w) != len(ag_f):
        raise SystemExit(f"bench.py: expected {SWEEP_FRAMES * len(cand)} aggregation dispatches, "
                         f"found {len(ag_f)} / {len(ag_w)}")
    table = {}
    for i, c in enumerate(cand):
        k = SWEEP_FRAMES * i + SWEEP_FRAMES - 1
        table[",".join(str(v) for v in c)] = {
            "fetch_size_kib": ag_f[k], "write_size_kib": ag_w[k],
            "traffic_bytes_per_launch": (ag_f[k] * ff + ag_w[k] * fw) * 1024}
    sweep = "python3 bench.py --tuning-sweep"
    rec = {"kernels": names,
           "workload": "plain scene-flow frame 1242x375 D=128, all 4 views in one aggregation launch; "
                       f"{SWEEP_FRAMES} frames per tuning, counters of the last one",
           "keys": "chains_per_block,prefetch,order,persistent_per_cu,packed",
           "sources": TRAFFIC_SOURCES, "sources_sha256": _sources_sha256(),
           "copy_calibration": {"bytes": 1 << 30, "fetch_size_kib": cf, "write_size_kib": cw,
                                "fetch_factor": ff, "write_factor": fw},
           "by_tuning": table,
           "commands": [f"rocprofv3 --pmc FETCH_SIZE -d {os.path.dirname(fetch_db) or '.'} -o fetch -- {sweep}",
                        f"rocprofv3 --pmc WRITE_SIZE -d {os.path.dirname(write_db) or '.'} -o write -- {sweep}",
                        f"python3 bench.py --traffic-from {fetch_db} {write_db}"]}
    with open(out, "w") as fo:
        json.dump(rec, fo, indent=1)
    tb = [e["traffic_bytes_per_launch"] / 1e9 for e in table.values()]
    print(json.dumps({"traffic_table": out, "tunings": len(table), "GB_min": min(tb),
                      "GB_max": max(tb)}), flush=True)


def bench_tuning_sweep(args, dev):
    """Three 1 GiB device copies (the calibration kernel), then SWEEP_FRAMES plain
    1242x375/128 frames for every aggregation tuning: the program the FETCH_SIZE
    and WRITE_SIZE passes of the traffic table run."""
    import numpy as np
    import torch

    from paper_1801_04720_amd import synth
    from paper_1801_04720_amd._lib import SfAggTuning
    from paper_1801_04720_amd.pipeline import FusedFrame

    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device=dev)
    b = torch.empty(n, dtype=torch.uint8, device=dev)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    H, W, D = 375, 1242, 128
    fr = synth.frame_1242x375(0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    inputs = [t(fr.t0.left), t(fr.t0.right), t(fr.t1.left), t(fr.t1.right), t(fr.flow)]
    torch.cuda.synchronize()
    cand = tuning_candidates()
    for i, c in enumerate(cand):
        pipe = FusedFrame(H, W, D, tuning=SfAggTuning(*c), device=dev)
        for _ in range(SWEEP_FRAMES):
            pipe.run(*inputs)
        torch.cuda.synchronize()
        del pipe
        if i % 6 == 5:
            print(f"tuning sweep: {i + 1}/{len(cand)} tunings", flush=True)
    print(json.dumps({"tuning_sweep": cand, "frames_per_tuning": SWEEP_FRAMES, "copy_bytes": n,
                      "copies": 3}), flush=True)


def sceneflow_diagnostics(fr, valid0, valid1, valid):
    """Density of the scene flow over all pixels and over non-occluded ones,
    and why the other pixels are undefined, in the order the combination rule
    tests them: the flow leaves the image, the t0 disparity was rejected, or a
    t1 disparity tap was rejected.  Non-occluded: visible in the t0 right view,
    moved (by the generator's flow) to a pixel inside the image that is visible
    in the t1 right view.  Host-side, from one frame's outputs."""
    import numpy as np

    H, W = valid0.shape
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float32)
    u, v = fr.flow[..., 0], fr.flow[..., 1]
    xp, yp = xs + u, ys + v
    inside = (xp >= 0) & (xp <= W - 1) & (yp >= 0) & (yp <= H - 1)
    x0 = np.clip(np.floor(np.where(inside, xp, 0)), 0, W - 1).astype(np.int64)
    y0 = np.clip(np.floor(np.where(inside, yp, 0)), 0, H - 1).astype(np.int64)
    x1, y1 = np.minimum(x0 + 1, W - 1), np.minimum(y0 + 1, H - 1)
    v1 = valid1.astype(bool)
    taps = v1[y0, x0] & v1[y0, x1] & v1[y1, x0] & v1[y1, x1]
    d0 = valid0.astype(bool)
    defined = (valid & 1).astype(bool)
    out_img = ~inside
    bad_d0 = inside & ~d0
    bad_d1 = inside & d0 & ~taps
    gu, gv = fr.gt_flow[..., 0], fr.gt_flow[..., 1]
    gx, gy = np.rint(xs + gu), np.rint(ys + gv)
    gin = (gx >= 0) & (gx <= W - 1) & (gy >= 0) & (gy <= H - 1)
    gxi = np.clip(gx, 0, W - 1).astype(np.int64)
    gyi = np.clip(gy, 0, H - 1).astype(np.int64)
    noc = ~fr.t0.occluded & gin & ~fr.t1.occluded[gyi, gxi]
    n = float(H * W)
    return {"sceneflow_density_noc": float(defined[noc].mean()), "noc_fraction": float(noc.mean()),
            "undefined_flow_leaves_image": float(out_img.sum() / n),
            "undefined_t0_disparity_rejected": float(bad_d0.sum() / n),
            "undefined_t1_disparity_rejected": float(bad_d1.sum() / n),
            "rule_matches_kernel": bool(np.array_equal(defined, inside & d0 & taps))}


def cpu_baseline(fr, D, runs=3):
    """The oracle on one stereo pair of the frame, timed `runs` times on one
    host thread; the median run gives the rate."""
    import oracle

    # Pinned to one core of those this process may use (the oracle is single-threaded).
    allowed = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    core = allowed[0] if allowed else None
    if core is not None:
        os.sched_setaffinity(0, {core})
    try:
        times = []
        for _ in range(runs):
            t = time.perf_counter()
            oracle.disparity(fr.t0.left, fr.t0.right, D)
            times.append(time.perf_counter() - t)
    finally:
        if core is not None:
            os.sched_setaffinity(0, set(allowed))
    dt = sorted(times)[len(times) // 2]
    H, W = fr.t0.left.shape
    return {"value": H * W * D * 8 / dt / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
            "sample": f"one {W}x{H} D={D} stereo pair (t0 of frame 0): census of both views, both "
                      f"cost volumes, both 8-path aggregations, WTA, sub-pixel, LR check; "
                      f"single thread pinned to core {core}, median of {runs} runs "
                      f"({', '.join(f'{x:.2f}' for x in times)} s)",
            "seconds": dt, "runs_s": times, "pinned_core": core, "cpu": _cpu_model(),
            "host_threads": os.cpu_count(), "affinity_threads": len(allowed) or None}


def _cpu_model():
    """The host CPU as /proc/cpuinfo names it: model string, family / model /
    stepping numbers, clock, cache (a virtual machine may shorten the string)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if info:
                        break  # first processor only
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("vendor_id", "model name", "cpu family", "model", "stepping", "microcode", "cpu MHz",
                         "cache size") and k not in info:
                    info[k] = v
    except OSError:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "BIOS Model name", "Hypervisor vendor", "Virtualization type"):
                info["lscpu " + k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info or None


def _gen_pair(arg):
    from paper_1801_04720_amd import synth

    i, (H, W, D) = arg
    p = synth.pair_batch(i, H, W, D)
    return p.left, p.right


def bench_batch(args, dev):
    """Uneven batch: one captured graph for all pairs, per-class GCUPS, and the
    speed-up over running the same pairs one by one through the C-ABI stages."""
    import concurrent.futures as cf

    import torch

    from paper_1801_04720_amd import api, batch, synth

    sizes = synth.batch_sizes(args.pairs)
    with cf.ProcessPoolExecutor(max_workers=12) as ex:
        imgs = list(ex.map(_gen_pair, list(enumerate(sizes)), chunksize=2))
    pairs = [{"left": torch.from_numpy(L).to(dev), "right": torch.from_numpy(R).to(dev), "D": D}
             for (L, R), (_, _, D) in zip(imgs, sizes)]
    classes = []
    for s_ in sizes:
        if s_ not in classes:
            classes.append(s_)
    tunings, tune_info = {}, {}
    for (H, W, D) in classes:
        t, ms = batch.autotune(H, W, D, nviews=2,
                               cache=TUNE_CACHE)
        tunings[(H, W, D)] = t
        tune_info[f"{W}x{H}xD{D}"] = dict(batch.tuning_dict(t), aggregation_ms_per_pair=ms)
    budget = int(args.mem_budget_gb * (1 << 30))

    def time_graph(prs, steps, warmup):
        b = batch.Batch(prs, tunings=tunings, mem_budget=budget, device=dev)
        s = torch.cuda.Stream()
        b.capture(s)
        for _ in range(warmup):
            b.launch(s)
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            b.launch(s)
        e1.record(s)
        s.synchronize()
        return e0.elapsed_time(e1) / steps, b

    steps = max(1, min(args.steps, 10))
    ms_batch, b = time_graph(pairs, steps, max(1, args.warmup))
    nwaves = b.nwaves
    # Free the whole batch's workspace (up to the budget) before the per-class
    # batches take theirs; the parity spot check below builds it again.
    del b
    torch.cuda.empty_cache()
    cells = lambda prs: sum(p["left"].shape[0] * p["left"].shape[1] * p["D"] * 8 for p in prs)  # noqa: E731
    per_class = {}
    for (H, W, D) in classes:
        prs = [p for p in pairs if (p["left"].shape[0], p["left"].shape[1], p["D"]) == (H, W, D)]
        ms_c, bc = time_graph(prs, steps, 1)
        del bc
        torch.cuda.empty_cache()
        per_class[f"{W}x{H}xD{D}"] = {"pairs": len(prs), "ms": ms_c,
                                     "gcups_delivered": cells(prs) / (ms_c * 1e-3) / 1e9,
                                     "gcups_all_passes": 2 * cells(prs) / (ms_c * 1e-3) / 1e9}
    # Plain form: the same pairs one by one through the per-stage C-ABI calls.
    bufs = {}
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def plain_pair(p):
        H, W = p["left"].shape
        D = p["D"]
        k = (H, W, D)
        if k not in bufs:
            bufs[k] = {"cost": torch.empty((H, W, D), dtype=torch.uint8, device=dev),
                       "Sl": torch.empty((H, W, D), dtype=torch.int16, device=dev),
                       "Sr": torch.empty((H, W, D), dtype=torch.int16, device=dev),
                       "ws": torch.empty(api.sgm_workspace_bytes(H, W, D), dtype=torch.uint8, device=dev)}
        q = bufs[k]
        cl, cr = api.census(p["left"]), api.census(p["right"])
        api.sgm_aggregate(api.cost(cr, cl, D, True, out=q["cost"]), 10, 120, out=q["Sr"], workspace=q["ws"])
        api.sgm_aggregate(api.cost(cl, cr, D, False, out=q["cost"]), 10, 120, out=q["Sl"], workspace=q["ws"])
        return api.wta_lr(q["Sl"], q["Sr"], None, 120, 1)

    for p in pairs[:3]:
        plain_pair(p)
    torch.cuda.synchronize()
    e0.record()
    for p in pairs:
        r = plain_pair(p)
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    # Spot parity: the last pair of each class, batched vs one-by-one.
    bufs.clear()
    torch.cuda.empty_cache()
    b = batch.Batch(pairs, tunings=tunings, mem_budget=budget, device=dev)
    b.run()
    torch.cuda.synchronize()
    same = True
    for (H, W, D) in classes:
        i = max(j for j, s_ in enumerate(sizes) if s_ == (H, W, D))
        r = plain_pair(pairs[i])
        torch.cuda.synchronize()
        same &= bool(torch.equal(r["valid"], b.out[i]["valid"]) and torch.equal(r["wta_left"], b.out[i]["wta"]))
    tot = cells(pairs)
    res = {
        "metric": "batched plain SGM: whole-batch latency + per-size GCUPS (W·H·D·8 paths/s)",
        "value": tot / (ms_batch * 1e-3) / 1e9, "unit": "GCUPS", "n_gpus": 1, "steps": steps,
        "warmup": max(1, args.warmup), "ms_per_step": ms_batch, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic (seeded piecewise-planar pairs)",
        "config": {"workload": f"{args.pairs} uneven stereo pairs: 640x480 D=64, 1242x375 D=128, "
                               "1920x1080 D=256 (pair i has class i mod 3), one HIP graph",
                   "mem_budget_gb": args.mem_budget_gb, "waves": nwaves},
        "batch_latency_ms": ms_batch, "per_class": per_class, "autotune": tune_info,
        "plain_one_by_one_ms": ms_plain, "speedup_batched_vs_plain": ms_plain / ms_batch,
        "spot_parity_batched_equals_one_by_one": same,
    }
    print(json.dumps(res), flush=True)


def _gen_frame(i):
    from paper_1801_04720_amd import synth

    fr = synth.frame_planar(synth.rng_for(5, i), 1024, 2048, 256, 200.0)
    return fr.t0.left, fr.t0.right, fr.t1.left, fr.t1.right, fr.flow


def bench_stream(args, dev):
    """Stream of 2048x1024 D=256 frames resident in HBM: the learned frame on every
    frame (t0 and t1 aggregated in one launch), the plain frame as judge on every
    16th; per-frame latency from events on the stream; compared with the all-plain
    stream on the same frames."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    from paper_1801_04720_amd import api, batch
    from paper_1801_04720_amd.pipeline import FusedFrame, JudgedLearnedStream

    H, W, D = 1024, 2048, 256
    n = args.frames
    with cf.ProcessPoolExecutor(max_workers=14) as ex:
        host = [tuple(torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in f)
                for f in ex.map(_gen_frame, range(n), chunksize=2)]
    frames = [tuple(a.to(dev) for a in f) for f in host]
    with np.load(args.lrnet, allow_pickle=False) as z:
        prm = torch.from_numpy(z["params"].astype(np.float32)).to(dev)
    cache = TUNE_CACHE
    t2, _ = batch.frame_autotune(H, W, D, flags=api.FRAME_LEARNED, cache=cache)
    t4, _ = batch.frame_autotune(H, W, D, cache=cache)
    learned = FusedFrame(H, W, D, learned_params=prm, tuning=t2, device=dev)
    plain = FusedFrame(H, W, D, tuning=t4, device=dev)
    s = torch.cuda.current_stream()

    def run_stream(judge_every):
        """judge_every > 0: the judged learned stream (JudgedLearnedStream: the plain
        frame judges every judge_every-th frame and is delivered there; below the
        agreement threshold the frames up to the next judge are plain frames);
        0: the all-plain stream."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        js = None
        if judge_every:
            js = JudgedLearnedStream(H, W, D, prm, judge_every=judge_every, threshold=args.fallback_threshold,
                                     device=dev, learned=learned, plain=plain)
        for f in frames[:2]:  # warm-up, a judged frame included
            (js if judge_every else plain).run(*f)
        if js is not None:
            js.k, js.mode, js.history = 0, "learned", []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        modes = []
        for i, f in enumerate(frames):
            ev[i][0].record(s)
            if judge_every:
                judged = js.k % judge_every == 0
                js.run(*f)
                modes.append("judged" if judged else js.mode)
            else:
                plain.run(*f)
            ev[i][1].record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        agree = [[h[1], h[2]] for h in js.history] if js else []
        return wall, lat, agree, modes

    def run_stream_from_host(judge_every):
        """Inputs start in pinned host memory and the scene flow (sf4 + valid) goes
        back to pinned host memory: two frame slots, uploads on one stream and
        downloads on another, both overlapped with the compute of the other slot."""
        h2d, d2h = torch.cuda.Stream(), torch.cuda.Stream()
        slots = []
        for _ in range(2):
            ff = FusedFrame(H, W, D, learned_params=prm, tuning=t2, device=dev)
            slots.append({"ff": ff, "inp": [torch.empty_like(a) for a in frames[0]],
                          "sf4": torch.empty((H, W, 4), dtype=torch.float32).pin_memory(),
                          "valid": torch.empty((H, W), dtype=torch.uint8).pin_memory(),
                          "copied": torch.cuda.Event(), "computed": torch.cuda.Event(),
                          "freed": torch.cuda.Event()})
        t_in = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
        t_out = [torch.cuda.Event(enable_timing=True) for _ in range(n)]

        def upload(i):
            sl = slots[i % 2]
            with torch.cuda.stream(h2d):
                if i >= 2:
                    h2d.wait_event(sl["freed"])
                t_in[i].record(h2d)
                for dst, src in zip(sl["inp"], host[i]):
                    dst.copy_(src, non_blocking=True)
                sl["copied"].record(h2d)

        agree = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        upload(0)
        for i in range(n):
            if i + 1 < n:
                upload(i + 1)
            sl = slots[i % 2]
            s.wait_event(sl["copied"])
            out = sl["ff"].run(*sl["inp"])
            if judge_every and i % judge_every == 0:
                ref = plain.run(*sl["inp"])
                agree.append((out["valid0"] == ref["valid0"]).float().mean())
            sl["computed"].record(s)
            with torch.cuda.stream(d2h):
                d2h.wait_event(sl["computed"])
                sl["sf4"].copy_(out["sf4"], non_blocking=True)
                sl["valid"].copy_(out["valid"], non_blocking=True)
                t_out[i].record(d2h)
                sl["freed"].record(d2h)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(b) for a, b in zip(t_in, t_out)])
        return wall, lat, [float(a.item()) for a in agree]

    wl, ll, agree, modes = run_stream(16)
    wp, lp, _, _ = run_stream(0)
    we, le, agree_e = run_stream_from_host(16)

    # Per-kernel times of the plain frame at this size, where the per-pixel
    # stages are not launch-bound: bytes moved per launch over the time.
    from paper_1801_04720_amd import _lib

    lib = _lib.lib()
    nk = 10
    torch.cuda.synchronize()
    _lib.check(lib.sf_prof_enable(64 * nk))
    for f in frames[:nk]:
        plain.run(*f)
    torch.cuda.synchronize()
    lib.sf_prof_disable()
    npx = H * W
    # Bytes each launch moves by design; a cost byte is 6 bits when the tuning packs costs.
    cb = 0.75 * D if t4.packed and D in (128, 256) else D
    moved = {"census": 4 * npx * (1 + 8), "cost": 4 * npx * (16 + cb),
             "sgm_tasks": 4 * npx * (8 * cb + 8 * D), "wta_slab_right": 2 * npx * D * 8,
             "wta_slab_left": 2 * npx * D * 8, "combine": npx * 59}
    kern = {}
    for name, nbytes in moved.items():
        tot, nl = kernel_ms(lib, name)
        if nl:
            kern[name] = {"avg_ms": tot / nl, "bytes_per_launch": nbytes,
                          "TBps": nbytes / (tot / nl * 1e-3) / 1e12}
    res = {
        "metric": "scene-flow stream: sustained fps + p50/p99 per-frame latency @2048x1024 D=256",
        "value": n / wl, "unit": "frames/s", "n_gpus": 1, "steps": n, "warmup": 2,
        "ms_per_step": 1e3 * wl / n, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u16", "data": "synthetic (seeded piecewise-planar 2048x1024 frames, flow within 200 px)",
        "config": {"workload": f"{n} frames 2048x1024 D=256: learned frame (t0+t1 in one aggregation "
                               "launch, network mask) with the plain frame as judge on every 16th and "
                               "as fallback below the agreement threshold"},
        "learned_stream": {"fps": n / wl, "p50_ms": float(np.percentile(ll, 50)),
                           "p99_ms": float(np.percentile(ll, 99))},
        "plain_stream": {"fps": n / wp, "p50_ms": float(np.percentile(lp, 50)),
                         "p99_ms": float(np.percentile(lp, 99))},
        "speedup_learned_vs_plain": wp / wl,
        "learned_stream_end_to_end": {
            "fps": n / we, "p50_ms": float(np.percentile(le, 50)), "p99_ms": float(np.percentile(le, 99)),
            "note": "inputs (4 images + flow, 24 MiB) from pinned host memory, scene flow sf4 + valid "
                    "(34 MiB) back to pinned host memory; latency = upload start to download end"},
        "judge_mask_agreement_mean": [float(np.mean([a[0] for a in agree])), float(np.mean([a[1] for a in agree]))],
        "judge_mask_agreement_min": [float(np.min([a[0] for a in agree])), float(np.min([a[1] for a in agree]))],
        "judged_frames": len(agree),
        "fallback": {"threshold": args.fallback_threshold,
                     "frames_judged": modes.count("judged"), "frames_learned": modes.count("learned"),
                     "frames_plain_fallback": modes.count("plain"),
                     "policy": "the plain frame judges every 16th frame and is delivered there; when the "
                               "lower of its t0 / t1 mask agreements with the learned frame falls below the "
                               "threshold, the frames up to the next judge are plain frames"},
        "plain_frame_kernels_2048x1024": kern,
        "tuning": {"learned_2views": batch.tuning_dict(t2), "plain_4views": batch.tuning_dict(t4)},
    }
    print(json.dumps(res), flush=True)


def bench_lrnet(args, dev):
    """The fused network inference alone (lrnet_fused_kernel, weights packed by
    their own launch) on the two left maps of the 1242x375 D=128 frame: kernel
    time from HIP events on the launch stream, useful FLOP rate (10,656 FLOP per
    pixel) against the dense BF16 MFMA peak."""
    import numpy as np
    import torch

    from paper_1801_04720_amd import _lib, api, lrnet, synth

    H, W, D = 375, 1242, 128
    fr = synth.frame_1242x375(0)
    feats = []
    for L, R in ((fr.t0.left, fr.t0.right), (fr.t1.left, fr.t1.right)):
        Lt, Rt = torch.from_numpy(L).to(dev), torch.from_numpy(R).to(dev)
        cl, cr = api.census(Lt), api.census(Rt)
        S = api.sgm_aggregate(api.cost(cl, cr, D, False), 10, 120)
        feats.append(api.wta_lr(S, None, Lt, 120, 1, want_feat=True)["feat"])
    feat = torch.stack(feats).contiguous()
    with np.load(args.lrnet, allow_pickle=False) as z:
        prm = torch.from_numpy(z["params"].astype(np.float32)).to(dev)
    logits = torch.empty((2, H, W), dtype=torch.float32, device=dev)
    ws = torch.empty(lrnet.workspace_bytes(2, H, W, False), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        lrnet.forward(prm, feat, logits, ws)
    lib = _lib.lib()
    torch.cuda.synchronize()
    _lib.check(lib.sf_prof_enable(4 * max(args.steps, 1)))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lrnet.forward(prm, feat, logits, ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lib.sf_prof_disable()
    tot, n = kernel_ms(lib, "lrnet_fused")
    ms = tot / max(n, 1)
    flop = 2 * H * W * 10656.0
    peak = 2.5e15
    res = {"metric": "learned LR stand-in inference: fused 4-layer network, two 1242x375 maps",
           "value": flop / (ms * 1e-3) / 1e12, "unit": "TFLOP/s (useful)", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * wall / max(args.steps, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic (features of the seeded frame)",
           "config": {"workload": "fused network inference on 2 maps of 1242x375 (features of frame 0)"},
           "kernel_ms": ms, "timed_launches": n, "flop_per_launch": flop,
           "roofline": {"bound": "mfma", "achieved": flop / (ms * 1e-3) / 1e12, "peak": peak / 1e12,
                        "unit": "TFLOP/s", "frac": flop / (ms * 1e-3) / peak}}
    print(json.dumps(res), flush=True)


def bench_agg(args, dev):
    """One left-base view of the 1242x375 D=128 frame: cost volume + eight-path
    aggregation (sf_cost, sf_sgm_aggregate) against the aggregation that computes
    the Hamming costs from the census images inside the path walk
    (sf_sgm_aggregate_census).  Per-launch times from HIP events on the launch
    stream; value = cell updates per second of the census-mode aggregation."""
    import numpy as np
    import torch

    from paper_1801_04720_amd import _lib, api, synth

    H, W, D = 375, 1242, 128
    fr = synth.frame_1242x375(0)
    L = torch.from_numpy(np.ascontiguousarray(fr.t0.left)).to(dev)
    R = torch.from_numpy(np.ascontiguousarray(fr.t0.right)).to(dev)
    cl, cr = api.census(L), api.census(R)
    C = api.cost(cl, cr, D, False)
    S1 = torch.empty((H, W, D), dtype=torch.int16, device=dev)
    S2 = torch.empty_like(S1)
    ws = torch.empty(api.sgm_workspace_bytes(H, W, D), dtype=torch.uint8, device=dev)
    lib = _lib.lib()
    res = {}
    for name, fn in (("volume", lambda: (api.cost(cl, cr, D, False, out=C),
                                         api.sgm_aggregate(C, 10, 120, out=S1, workspace=ws))),
                     ("census", lambda: api.sgm_aggregate_census(cl, cr, D, False, 10, 120, out=S2,
                                                                 workspace=ws))):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        _lib.check(lib.sf_prof_enable(8 * max(args.steps, 1)))
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        lib.sf_prof_disable()
        r = {}
        for k in ("cost", "sgm_paths", "slab_sum"):
            tot, n = kernel_ms(lib, k)
            if n:
                r[k + "_ms"] = tot / n
        r["total_ms"] = sum(r.values())
        res[name] = r
    if not torch.equal(S1, S2):
        raise SystemExit("census-mode aggregation differs from the cost-volume path")
    cells = H * W * D * 8
    ms = res["census"]["sgm_paths_ms"]
    out = {"metric": "eight-path aggregation of one 1242x375 D=128 view with costs from the census images",
           "value": cells / (ms * 1e-3) / 1e9, "unit": "G cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u16", "data": "synthetic (left view of the seeded frame)",
           "config": {"workload": "one view 1242x375 D=128, P1=10, P2=120, 8 paths"},
           "legs": res}
    print(json.dumps(out), flush=True)


def learned_leg(args, plain_pipe, inputs, H, W, D, ms_plain, dev):
    """Learned frame (right views skipped, network mask): fps, speed-up over the
    plain frame, and agreement of its masks with the plain LR check on this frame."""
    import numpy as np
    import torch

    from paper_1801_04720_amd import api, lrnet
    from paper_1801_04720_amd.pipeline import FusedFrame

    trained = os.path.exists(args.lrnet)
    if trained:
        with np.load(args.lrnet, allow_pickle=False) as z:
            prm = z["params"].astype(np.float32)
    else:
        prm = lrnet.init_params(0)
    prm_t = torch.from_numpy(prm).to(dev)
    tuning = None
    if not args.no_autotune:
        from paper_1801_04720_amd import batch

        tuning, _ = batch.frame_autotune(H, W, D, flags=api.FRAME_LEARNED,
                                         cache=TUNE_CACHE)
    lp = FusedFrame(H, W, D, learned_params=prm_t, tuning=tuning, device=dev)
    for _ in range(args.warmup):
        lp.run(*inputs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = lp.run(*inputs)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / max(args.steps, 1)
    plain = plain_pipe.run(*inputs)
    torch.cuda.synchronize()
    agree = [float((out[k] == plain[k]).float().mean().item()) for k in ("valid0", "valid1")]
    both = lambda m: float((m & 1).float().mean().item())  # noqa: E731
    return {"fps_learned": 1e3 / ms, "ms_learned": ms, "speedup_learned_vs_plain": ms_plain / ms,
            "gcups_learned_delivered": 2 * H * W * D * 8 / (ms * 1e-3) / 1e9,
            "learned_weights": os.path.relpath(args.lrnet, ROOT) if trained else "untrained init",
            "lr_mask_agreement_t0_t1": agree,
            "sceneflow_density_learned": both(out["valid"])}


def variants_leg(args, plain_pipe, inputs, fr, H, W, D, ms_plain, dev):
    """Frames with the cited SGM method's variants: right maps by the diagonal
    search in the left volumes (right-view aggregations skipped), 3x3 median of
    the sub-pixel maps, intensity-adaptive P2, and all three.  Per variant: ms
    per frame, speed-up over the full plain frame, agreement of the t0/t1 masks
    with the plain LR check, the t0 map's density and end-point error against
    the generator's ground-truth disparity, and the scene-flow outlier rates
    (the paper's Table 1 metric) of the sparse map ("Est") and of its
    densified version ("All")."""
    import torch

    from paper_1801_04720_amd import _lib, api
    from paper_1801_04720_amd.evaluate import sf_outliers
    from paper_1801_04720_amd.pipeline import FusedFrame

    lib = _lib.lib()
    tuned = not args.no_autotune
    if tuned:
        from paper_1801_04720_amd import batch

        cache = TUNE_CACHE
    gt = torch.from_numpy(fr.t0.gt_disp).to(dev)
    plain = plain_pipe.run(*inputs)
    plain = {k: plain[k].clone() for k in ("valid0", "valid1", "disp0", "sf4", "valid")}

    def quality(o):
        v = o["valid0"].bool()
        dense = api.densify(o["sf4"], o["valid"])
        gts = (fr.gt_flow, fr.t0.gt_disp, fr.gt_disp1_at_t0)
        return {"density_t0": float(v.float().mean().item()),
                "epe_t0": float((o["disp0"][v] - gt[v]).abs().mean().item()),
                "sf_outliers_est": sf_outliers(o["sf4"], o["valid"] & 1, *gts),
                "sf_outliers_all": sf_outliers(dense["sf4"], dense["fill"] > 0, *gts)}

    res = {"plain": quality(plain)}
    # Densification of the plain frame's map, timed on its own.
    dn = api.densify(plain["sf4"], plain["valid"])
    torch.cuda.synchronize()
    _lib.check(lib.sf_prof_enable(64 * max(args.steps, 1)))
    for _ in range(args.steps):
        api.densify(plain["sf4"], plain["valid"], out=dn)
    torch.cuda.synchronize()
    lib.sf_prof_disable()
    tot, n = kernel_ms(lib, "densify")
    res["plain"]["densify_ms"] = tot / max(n, 1)
    for name, kw in (("diag", dict(diag=True)), ("median", dict(median=True)),
                     ("adaptive_p2", dict(adaptive_p2=True)),
                     ("diag_median_adaptive", dict(diag=True, median=True, adaptive_p2=True))):
        flags = ((api.FRAME_DIAG if kw.get("diag") else 0) | (api.FRAME_MEDIAN if kw.get("median") else 0) |
                 (api.FRAME_ADAPTIVE_P2 if kw.get("adaptive_p2") else 0))
        tun = batch.frame_autotune(H, W, D, flags=flags, cache=cache)[0] if tuned else None
        fp = FusedFrame(H, W, D, tuning=tun, device=dev, **kw)
        for _ in range(args.warmup):
            fp.run(*inputs)
        torch.cuda.synchronize()
        _lib.check(lib.sf_prof_enable(64 * max(args.steps, 1)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = fp.run(*inputs)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / max(args.steps, 1)
        lib.sf_prof_disable()
        kern = {}
        for kname in ["cost", "sgm_tasks", "wta_slab_right", "wta_slab_left", "wta_diag", "median3x3"]:
            tot, n = kernel_ms(lib, kname)
            if n:
                kern[kname] = tot / n
        r = {"ms": ms, "fps": 1e3 / ms, "speedup_vs_plain": ms_plain / ms,
             "mask_agreement_t0_t1": [float((out[k] == plain[k]).float().mean().item())
                                      for k in ("valid0", "valid1")],
             "kernels_avg_ms": kern}
        r.update(quality(out))
        res[name] = r
        del fp
    return {"variants": res, "fps_diag": res["diag"]["fps"], "ms_diag": res["diag"]["ms"],
            "speedup_diag_vs_plain": res["diag"]["speedup_vs_plain"]}


def flow_leg(args, plain_pipe, inputs, fr, H, W, D, dev):
    """Optical-flow stand-in on the frame's two left images: GPU ms per flow field
    (forward + backward + consistency check) for a few iteration counts, its
    quality against the generator's flow (end-point error on the kept pixels,
    Fl outliers, density), and the whole scene flow computed from the four
    images alone (flow + plain frame): ms and Table-1 outliers Est / All."""
    import torch

    from paper_1801_04720_amd import _lib, api
    from paper_1801_04720_amd.evaluate import sf_outliers

    lib = _lib.lib()
    L0, R0, L1, R1, _ = inputs
    gt = torch.from_numpy(fr.gt_flow).to(dev)
    res = {}
    buf = api.flow(L0, L1, levels=5, iters=2, R=128)
    for iters, fine in ((2, 0), (4, 0), (6, 0), (8, 0), (4, 8), (6, 8)):
        api.flow(L0, L1, levels=5, iters=iters, R=128, fine_radius=fine, out=buf)
        torch.cuda.synchronize()
        _lib.check(lib.sf_prof_enable(64 * max(args.steps, 1)))
        for _ in range(max(1, args.steps // 3)):
            api.flow(L0, L1, levels=5, iters=iters, R=128, fine_radius=fine, out=buf)
        torch.cuda.synchronize()
        lib.sf_prof_disable()
        tot, n = kernel_ms(lib, "flow")
        fl = buf["flow"]
        kept = ~torch.isnan(fl[..., 0])
        err = torch.linalg.norm(fl - gt, dim=-1)
        gtn = torch.linalg.norm(gt, dim=-1)
        res[f"levels5_iters{iters}_R128" + (f"_fine{fine}" if fine else "")] = {
            "ms": tot / max(n, 1), "density": float(kept.float().mean().item()),
            "epe_kept": float(err[kept].mean().item()),
            "fl_outliers_kept_pct": float(100.0 * ((err > 3) & (err > 0.05 * gtn))[kept].float().mean().item())}
    # Scene flow from images alone with 4 iterations per level, fine-level radius 8.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 3)):
        api.flow(L0, L1, levels=5, iters=4, R=128, fine_radius=8, out=buf)
        out = plain_pipe.run(L0, R0, L1, R1, buf["flow"])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / max(1, args.steps // 3)
    dense = api.densify(out["sf4"], out["valid"])
    gts = (fr.gt_flow, fr.t0.gt_disp, fr.gt_disp1_at_t0)
    res["scene_flow_from_images"] = {
        "ms": ms, "fps": 1e3 / ms, "flow": "levels 5, iters 4, R 128, fine radius 8",
        "sf_outliers_est": sf_outliers(out["sf4"], out["valid"] & 1, *gts),
        "sf_outliers_all": sf_outliers(dense["sf4"], dense["fill"] > 0, *gts)}
    return {"flow_standin": res}


def sequence_leg(args, dev, T=8):
    """Scene flow over T = 8 time steps of one 1242x375 D=128 rig (flow within
    60 px): the T disparity maps in one batch plan (a HIP graph), the T-1
    combinations and the T-2 temporal checks.  Reports ms per time step and
    the Table-1 outlier rates of the scene-flow maps before and after the
    temporal validation, with their densities."""
    import numpy as np
    import torch

    from paper_1801_04720_amd import synth
    from paper_1801_04720_amd.evaluate import sf_outliers
    from paper_1801_04720_amd.pipeline import SequenceFrames

    s = synth.sequence_planar(synth.rng_for(6, 0), T, 375, 1242, 128, 60.0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    lefts, rights = [t(p.left) for p in s.pairs], [t(p.right) for p in s.pairs]
    flows = [t(f) for f in s.flows]
    seq = SequenceFrames(lefts, rights, 128, device=dev)
    st = torch.cuda.Stream()  # graph capture needs a stream of its own
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        seq.batch.capture(st)
        for _ in range(2):
            seq.run(flows)
        torch.cuda.synchronize()
        reps = max(1, args.steps // 3)
        t0 = time.perf_counter()
        for _ in range(reps):
            _, S, tv = seq.run(flows)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
    before, after = [], []
    for k in range(T - 2):
        gts = (s.gt_flows[k], s.pairs[k].gt_disp, s.gt_d1[k])
        before.append(sf_outliers(S[k]["sf4"], S[k]["valid"] & 1, *gts))
        after.append(sf_outliers(S[k]["sf4"], tv[k], *gts))
    mean = lambda rs, key: float(np.mean([r[key] for r in rs]))  # noqa: E731
    return {"sequence": {
        "workload": f"{T} time steps 1242x375 D=128, flow within 60 px",
        "ms_per_sequence": ms, "ms_per_time_step": ms / T,
        "sf_outliers_before": {k: mean(before, k) for k in ("density", "D1", "D2", "Fl", "SF")},
        "sf_outliers_temporally_validated": {k: mean(after, k) for k in ("density", "D1", "D2", "Fl", "SF")},
        "tau_f_px": seq.tau_f, "tau_d_px": seq.tau_d}}


def bench_peaks(args, dev):
    """Measured ceilings: HBM stream rates (2 GiB buffers, far above the 256 MB
    last-level cache), the same copy on a 64 MiB buffer that the last-level cache
    holds, and the packed 16-bit VALU rate."""
    import torch
    from paper_1801_04720_amd import _lib

    lib = _lib.lib()
    st = torch.cuda.current_stream()
    sp = ct.c_void_p(st.cuda_stream)
    reps = max(args.steps, 3)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"metric": "measured ceilings", "reps": reps}
    for label, nbytes in (("hbm", 2 << 30), ("llc", 64 << 20)):
        a = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        pa, pb = ct.c_void_p(a.data_ptr()), ct.c_void_p(b.data_ptr())
        for mode, name, moved in ((0, "copy", 2 * nbytes), (1, "read", nbytes), (2, "write", nbytes)):
            ms = timed(lambda: _lib.check(lib.sf_probe_stream(pa, pb, nbytes, mode, sp)))
            out[f"{label}_{name}_GBps"] = moved / (ms * 1e-3) / 1e9
        del a, b
    props = torch.cuda.get_device_properties(0)
    blocks, iters = props.multi_processor_count * 32, 8192
    o = torch.empty(blocks * 256, dtype=torch.int32, device=dev)
    ms = timed(lambda: _lib.check(lib.sf_probe_pk_u16(ct.c_void_p(o.data_ptr()), blocks, iters, sp)))
    out["valu_pk_u16_Tops"] = blocks * 256 * iters * 32 / (ms * 1e-3) / 1e12
    out["cu"] = props.multi_processor_count
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--epilogue", type=int, default=0, help="0 auto, 1 u8 slabs, 2 atomics")
    ap.add_argument("--pipeline", default="fused", choices=["fused", "persistent", "stages"],
                    help="fused: sf_frame_run; persistent: same with persistent aggregation "
                         "blocks; stages: one C-ABI call per stage")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-frame leg")
    ap.add_argument("--no-flow", action="store_true", help="skip the optical-flow stand-in leg")
    ap.add_argument("--no-sequence", action="store_true",
                    help="skip the multi-time-step leg with temporal validation")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the SGM-variant legs (diagonal search, median, adaptive P2)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default aggregation tuning instead of the autotuner's choice")
    ap.add_argument("--lrnet", default=os.path.join(ROOT, "paper_1801_04720_amd", "data",
                                                    "lrnet_1242x375.npz"),
                    help="trained parameters of the learned LR stand-in (.npz)")
    ap.add_argument("--workload", default="frame", choices=["frame", "batch", "stream", "lrnet", "agg"],
                    help="frame: the 1242x375 D=128 scene-flow frame (default); batch: the "
                         "uneven batch of 64 pairs (640x480/64, 1242x375/128, 1920x1080/256); "
                         "stream: 2048x1024 D=256 frames, learned with a plain judge every 16th; "
                         "lrnet: the fused network inference alone on two 1242x375 maps")
    ap.add_argument("--frames", type=int, default=240, help="frames in the 2048x1024 stream")
    ap.add_argument("--fallback-threshold", type=float, default=0.99,
                    help="stream: mask agreement below which the judged stream falls back to plain frames")
    ap.add_argument("--pairs", type=int, default=64, help="pairs in the uneven batch")
    ap.add_argument("--mem-budget-gb", type=float, default=128.0,
                    help="workspace per wave of the uneven batch")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the HBM / last-level-cache stream rates and the packed "
                         "16-bit VALU rate, and exit")
    ap.add_argument("--tuning-sweep", action="store_true",
                    help="only run three 1 GiB copies and two plain frames per aggregation tuning "
                         "(the program of the FETCH_SIZE / WRITE_SIZE passes), and exit")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the per-tuning traffic table from the rocprofv3 databases of the "
                         "two counter passes over --tuning-sweep, and exit (no GPU needed)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (the reference kernel "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the path shards per stereo pair / frame, see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.traffic_from:
        return write_traffic_table(*args.traffic_from)

    import numpy as np
    import torch

    from paper_1801_04720_amd import _lib, api, synth
    from paper_1801_04720_amd.pipeline import FusedFrame, PlainFrame

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    if args.peaks:
        return bench_peaks(args, dev)
    if args.tuning_sweep:
        return bench_tuning_sweep(args, dev)
    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device=dev)
        b = torch.empty(n, dtype=torch.uint8, device=dev)
        a.fill_(1)
        for _ in range(max(args.steps, 1)):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": max(args.steps, 1)}), flush=True)
        return
    lib = _lib.lib()
    if args.workload == "batch":
        return bench_batch(args, dev)
    if args.workload == "stream":
        return bench_stream(args, dev)
    if args.workload == "lrnet":
        return bench_lrnet(args, dev)
    if args.workload == "agg":
        return bench_agg(args, dev)
    H, W, D = 375, 1242, 128
    fr = synth.frame_1242x375(0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    L0, R0, L1, R1, flow = t(fr.t0.left), t(fr.t0.right), t(fr.t1.left), t(fr.t1.right), t(fr.flow)
    api.sgm_set_epilogue(args.epilogue)
    tuning, tuning_info = None, None
    if args.pipeline != "stages" and not args.no_autotune:
        from paper_1801_04720_amd import batch

        tuning, t_ms = batch.frame_autotune(H, W, D,
                                            cache=TUNE_CACHE)
        tuning_info = dict(batch.tuning_dict(tuning), tuner_ms=t_ms)
    if args.pipeline == "stages":
        pipe = PlainFrame(H, W, D, device=dev)
    else:
        pipe = FusedFrame(H, W, D, persistent=args.pipeline == "persistent", tuning=tuning, device=dev)
    for _ in range(args.warmup):
        pipe.run(L0, R0, L1, R1, flow)
    torch.cuda.synchronize()
    # The tuning the fused plan runs (the plan's default when none is given).
    if tuning is not None:
        tuning_key = (tuning.chains_per_block, tuning.prefetch, tuning.order, tuning.persistent_per_cu,
                      tuning.packed)
    else:
        tuning_key = (16, 8, 0, 8 if args.pipeline == "persistent" else 0, 0)

    # Dominant kernel: the path aggregation (one launch for all 4 views, or one per view).
    kname, views_per_launch = ("sgm_paths", 1) if args.pipeline == "stages" else ("sgm_tasks", 4)
    # Timed region: HIP events on the launch stream around the dominant kernel only.
    _lib.check(lib.sf_prof_enable(64 * max(args.steps, 1)))
    _lib.check(lib.sf_prof_only(kname.encode()))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res_run = pipe.run(L0, R0, L1, R1, flow)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lib.sf_prof_disable()
    dom_tot, dom_n = kernel_ms(lib, kname)
    lib.sf_prof_only(None)

    ms = 1e3 * elapsed / max(args.steps, 1)
    cells = H * W * D * 8
    gcups_delivered = 2 * cells / (ms * 1e-3) / 1e9
    gcups_passes = 4 * cells / (ms * 1e-3) / 1e9
    # Per-kernel breakdown from a separate pass with every launch timed (outside the timed region).
    nb = max(min(args.steps, 20), 1)
    _lib.check(lib.sf_prof_enable(64 * nb))
    for _ in range(nb):
        pipe.run(L0, R0, L1, R1, flow)
    torch.cuda.synchronize()
    lib.sf_prof_disable()
    breakdown = {}
    for name in ["census", "cost", "sgm_paths", "sgm_tasks", "slab_sum", "wta_right", "wta_left",
                 "wta_slab_right", "wta_slab_left", "combine"]:
        tot, n = kernel_ms(lib, name)
        if n:
            breakdown[name] = {"avg_ms": tot / n, "launches": n, "ms_per_frame": tot / nb}
    sg = {"avg_ms": dom_tot / max(dom_n, 1), "launches": dom_n}
    avg_s = sg["avg_ms"] * 1e-3
    ops = 8 * cells * views_per_launch  # u16 element ops: 8 per cell update
    achieved = ops / avg_s / 1e12
    roofline = {"bound": "alu", "kernel": kname, "achieved": achieved,
                "peak": PEAK_U16_TOPS, "unit": "TOP/s (packed u16)",
                "frac": achieved / PEAK_U16_TOPS,
                "traffic": measured_traffic(kname, tuning_key),
                "ops_per_launch": ops, "avg_launch_ms": sg["avg_ms"], "timed_launches": sg["launches"],
                "gcups_per_launch": cells * views_per_launch / avg_s / 1e9}
    if roofline["traffic"]:
        # The launch's HBM-side bytes per second against the 8 TB/s HBM peak: the
        # aggregation is bound by this traffic, not by its packed 16-bit ALU work.
        roofline["traffic_TBps"] = roofline["traffic"] / avg_s / 1e12
        roofline["traffic_frac_of_hbm_peak"] = roofline["traffic_TBps"] / 8.0
    if args.pipeline == "stages":
        m0, m1, out = res_run
        v0t, vt = m0["valid"], out["valid"]
    else:
        v0t, vt = res_run["valid0"], res_run["valid"]
    valid0 = float(v0t.float().mean().item())
    dens = float((vt & 1).float().mean().item())
    v1t = res_run[1]["valid"] if args.pipeline == "stages" else res_run["valid1"]
    diag = sceneflow_diagnostics(fr, v0t.cpu().numpy(), v1t.cpu().numpy(), vt.cpu().numpy())
    res = {
        "metric": METRIC,
        "value": gcups_delivered,
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic (seeded piecewise-planar 1242x375 frame, noisy FP32 flow)",
        "config": {"workload": "plain scene-flow frame 1242x375 D=128 (SGM t0+t1 incl. right "
                               "views and LR check, combination, triangulation)",
                   "H": H, "W": W, "D": D, "paths": 8, "P1": 10, "P2": 120, "lr_tol": 1,
                   "epilogue": args.epilogue, "pipeline": args.pipeline,
                   "aggregation_tuning": tuning_info},
        "fps_plain": 1e3 / ms,
        "gcups_all_passes": gcups_passes,
        "lr_valid_frac_t0": valid0,
        "sceneflow_density": dens,
        "sceneflow_diagnostics": diag,
        "kernels": breakdown,
        "roofline": roofline,
    }
    if not args.no_learned and args.pipeline != "stages":
        res.update(learned_leg(args, pipe, (L0, R0, L1, R1, flow), H, W, D, ms, dev))
    if not args.no_variants and args.pipeline != "stages":
        res.update(variants_leg(args, pipe, (L0, R0, L1, R1, flow), fr, H, W, D, ms, dev))
    if not args.no_flow and args.pipeline != "stages":
        res.update(flow_leg(args, pipe, (L0, R0, L1, R1, flow), fr, H, W, D, dev))
    if not args.no_sequence and args.pipeline != "stages":
        res.update(sequence_leg(args, dev))
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(fr, D)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
