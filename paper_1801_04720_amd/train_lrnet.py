"""Train the learned stand-in for the LR check on seeded synthetic maps.

Three kinds of disparity maps, each labelled by the plain LR check (Sec. 3.1)
of the plain GPU path:
  * t0: piecewise-planar stereo pairs, 1242x375, D = 128 (KITTI's shape);
  * t1: the second time step of 1242x375 scene-flow frames: the left image is
    the first one forward-splatted along the flow with its holes filled by
    fresh noise, the right image rendered from it (synth.frame_planar);
  * big: both time steps of 2048x1024, D = 256 frames (the stream's size).
Each map goes through the plain GPU path once; its features and labels stay
resident in HBM.  Training samples random crops of random maps and runs the
HIP forward / backward / Adam kernels; validation runs the full network on
held-out maps of every kind and reports agreement with the LR check, end-point
error against ground truth on the learned and on the LR mask, and density,
per kind.

Checkpoints (--ckpt, every --ckpt-every steps and at the end) hold the weights,
Adam's moments and step, the seed, the crop sampler's generator state and the
data specification; --resume continues a run from one and gives the same
weights as the uninterrupted run.

    python -m paper_1801_04720_amd.train_lrnet --t0 6000 --t1 3000 --big 400 --steps 20000 --out lrnet.npz
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import time

import numpy as np
import torch

from . import api, lrnet, synth

# (stream, size, D, flow range) of each kind; training maps use indices from 0,
# validation maps from VAL0 on (disjoint seeds).
KINDS = {
    "t0": (4, 375, 1242, 128, None),
    "t1": (200, 375, 1242, 128, 100.0),
    "big": (300, 1024, 2048, 256, 200.0),
}
VAL0 = {"t0": 100000, "t1": 50000, "big": 50000}


def _gen(job):
    """One training unit: a list of (left, right, D, gt, occluded) maps."""
    kind, i, H, W = job
    stream, _, _, D, fmax = KINDS[kind]
    if kind == "t0":
        p = synth.pair_planar(synth.rng_for(stream, i), H, W, D)
        return [(p.left, p.right, D, p.gt_disp, p.occluded)]
    fr = synth.frame_planar(synth.rng_for(stream, i), H, W, D, fmax)
    maps = [(fr.t1.left, fr.t1.right, D, fr.t1.gt_disp, fr.t1.occluded)]
    if kind == "big":
        maps.insert(0, (fr.t0.left, fr.t0.right, D, fr.t0.gt_disp, fr.t0.occluded))
    return maps


class MapSet:
    """Features and labels (and, for validation, WTA, sub-pixel maps and ground
    truth) of many maps of mixed sizes, resident on the GPU."""

    def __init__(self):
        self.feats, self.labels, self.wtas, self.dsubs, self.gts, self.occs, self.kind = [], [], [], [], [], [], []

    def __len__(self):
        return len(self.feats)


def label_maps(jobs, workers, dev="cuda:0", keep_gt=False, log=None) -> MapSet:
    ms = MapSet()
    bufs = {}
    t0 = time.time()
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for n, (job, maps) in enumerate(zip(jobs, ex.map(_gen, jobs, chunksize=2))):
            if log and n and n % 500 == 0:
                log(f"  labelled {n} of {len(jobs)} units in {time.time() - t0:.0f} s")
            for L, R, D, gt, occ in maps:
                H, W = L.shape
                if (H, W, D) not in bufs:
                    bufs[(H, W, D)] = dict(
                        cost=torch.empty((H, W, D), dtype=torch.uint8, device=dev),
                        Sl=torch.empty((H, W, D), dtype=torch.int16, device=dev),
                        Sr=torch.empty((H, W, D), dtype=torch.int16, device=dev),
                        ws=torch.empty(api.sgm_workspace_bytes(H, W, D), dtype=torch.uint8, device=dev))
                b = bufs[(H, W, D)]
                Lt = torch.from_numpy(L).to(dev)
                Rt = torch.from_numpy(R).to(dev)
                cl, cr = api.census(Lt), api.census(Rt)
                api.cost(cr, cl, D, True, out=b["cost"])
                api.sgm_aggregate(b["cost"], 10, 120, out=b["Sr"], workspace=b["ws"])
                api.cost(cl, cr, D, False, out=b["cost"])
                api.sgm_aggregate(b["cost"], 10, 120, out=b["Sl"], workspace=b["ws"])
                o = {"feat": torch.empty((H, W, 4), dtype=torch.float32, device=dev),
                     "valid": torch.empty((H, W), dtype=torch.uint8, device=dev),
                     "wta_left": torch.empty((H, W), dtype=torch.int16, device=dev),
                     "disp": torch.empty((H, W), dtype=torch.float32, device=dev)}
                api.wta_lr(b["Sl"], b["Sr"], Lt, 120, 1, want_feat=True, out=o)
                ms.feats.append(o["feat"])
                ms.labels.append(o["valid"])
                ms.kind.append(job[0])
                if keep_gt:
                    ms.wtas.append(o["wta_left"])
                    ms.dsubs.append(o["disp"])
                    ms.gts.append(gt)
                    ms.occs.append(occ)
    torch.cuda.synchronize()
    return ms


def jobs_for(n_t0, n_t1, n_big, val=False):
    out = []
    for kind, n in (("t0", n_t0), ("t1", n_t1), ("big", n_big)):
        _, H, W, _, _ = KINDS[kind]
        base = VAL0[kind] if val else 0
        out += [(kind, base + i, H, W) for i in range(n)]
    return out


def evaluate(params, ms: MapSet, dev="cuda:0"):
    """Per kind: agreement with the LR check, EPE vs ground truth and density on
    the learned mask, the LR mask, no mask and the geometric rule x - d* >= 0."""
    res = {}
    for kind in sorted(set(ms.kind)):
        idx = [k for k in range(len(ms)) if ms.kind[k] == kind]
        agree = agree_g = 0.0
        tp = fp = fn = tn = 0
        e = {m: [] for m in ("learned", "lr", "none", "geom")}
        d = {m: [] for m in e}
        per_map = []
        for k in idx:
            H, W = ms.labels[k].shape
            xs = torch.arange(W, device=dev)[None, :]
            logits = lrnet.forward(params, ms.feats[k][None])
            geom = (xs - ms.wtas[k].long()) >= 0
            learned = (logits[0] > 0) & geom
            lab = ms.labels[k].bool()
            per_map.append(float((learned == lab).float().mean().item()))
            agree += per_map[-1]
            agree_g += float((geom == lab).float().mean().item())
            tp += int((learned & lab).sum())
            tn += int((~learned & ~lab).sum())
            fp += int((learned & ~lab).sum())
            fn += int((~learned & lab).sum())
            err = (ms.dsubs[k] - torch.from_numpy(ms.gts[k]).to(dev)).abs()
            for name, m in (("learned", learned), ("lr", lab), ("none", torch.ones_like(lab)), ("geom", geom)):
                e[name].append(float(err[m].mean().item()))
                d[name].append(float(m.float().mean().item()))
        n = len(idx)
        res[kind] = {"maps": n, "agreement": agree / n, "agreement_min": None, "tp": tp, "tn": tn, "fp": fp,
                     "fn": fn, "agreement_geometric": agree_g / n,
                     "agreement_no_check": float(np.mean([float(ms.labels[k].float().mean()) for k in idx]))}
        res[kind].update({f"epe_{m}_mask": float(np.mean(e[m])) for m in e})
        res[kind].update({f"density_{m}": float(np.mean(d[m])) for m in d})
        res[kind]["agreement_min"] = float(min(per_map))
    return res


def calibrate_bias(tr, ms: MapSet, n: int, dev="cuda:0") -> float:
    """Shift the output bias b4 by the logit threshold that maximises the lowest
    of the per-kind agreements (t0, t1, big) of the mask with the LR check, on
    the first n training maps of each kind; the mask rule itself stays
    logit > 0.  (The mask also needs x - d* >= 0, which every pixel of these
    maps meets: a match outside the image costs the maximum, so WTA never picks
    it.)  Thresholds are searched on a grid of 1/256 in [-4, 4].  Returns the
    threshold."""
    edges = torch.arange(-1024, 1025, device=dev, dtype=torch.float64) / 256.0
    per_kind = {}
    seen = {}
    for k in range(len(ms)):
        kd = ms.kind[k]
        if seen.get(kd, 0) >= n:
            continue
        seen[kd] = seen.get(kd, 0) + 1
        z = lrnet.forward(tr.params, ms.feats[k][None])[0].reshape(-1).double()
        y = ms.labels[k].reshape(-1).bool()
        # Errors at threshold e: valid pixels with z <= e plus invalid pixels with z > e.
        pos_le = torch.searchsorted(torch.sort(z[y]).values, edges, right=True).double()
        neg_sorted = torch.sort(z[~y]).values
        neg_gt = neg_sorted.numel() - torch.searchsorted(neg_sorted, edges, right=True).double()
        acc = per_kind.setdefault(kd, [torch.zeros_like(edges), 0])
        acc[0] += pos_le + neg_gt
        acc[1] += z.numel()
    agree = torch.stack([1.0 - e / cnt for e, cnt in per_kind.values()])
    worst = agree.min(dim=0).values
    best = float(worst.max())
    # The threshold closest to 0 among those reaching the best lowest agreement.
    cand = torch.nonzero(worst >= best).reshape(-1)
    i = int(cand[torch.argmin(edges[cand].abs())])
    thr = float(edges[i])
    tr.params[5376] -= thr
    return thr


def save_ckpt(path, tr, gen, cfg, step, extra=None):
    st = tr.state()
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=st["params"], m=st["m"], v=st["v"], step=st["step"], hyper=st["hyper"],
             next_step=step, seed=cfg["seed"], sampler_state=gen.get_state().numpy(),
             config=json.dumps(cfg), metrics=json.dumps(extra or {}))
    os.replace(tmp, path)


def train(cfg: dict, dev="cuda:0", log=print, resume: str | None = None, stop_after: int | None = None):
    """Runs (or resumes) one training; returns (trainer, metrics)."""
    t0 = time.time()
    train_set = label_maps(jobs_for(cfg["t0"], cfg["t1"], cfg["big"]), cfg["workers"], dev, log=log)
    val_set = label_maps(jobs_for(cfg["val_t0"], cfg["val_t1"], cfg["val_big"], val=True), cfg["workers"], dev,
                         keep_gt=True, log=log)
    t_data = time.time() - t0
    log(f"labelled {len(train_set)} training and {len(val_set)} validation maps in {t_data:.1f} s")
    init = lrnet.init_params(cfg["seed"])
    if cfg.get("init"):
        with np.load(cfg["init"], allow_pickle=False) as z:
            init = z["params"].astype(np.float32)
        log(f"initial weights from {cfg['init']}")
    tr = lrnet.Trainer(init, lr=cfg["lr"], device=dev)
    g = torch.Generator(device="cpu").manual_seed(cfg["seed"])
    start = 0
    if resume:
        with np.load(resume, allow_pickle=False) as z:
            saved = json.loads(str(z["config"]))
            for k in ("t0", "t1", "big", "steps", "batch", "crop", "lr", "seed"):
                if saved[k] != cfg[k]:
                    raise ValueError(f"--resume: checkpoint has {k} = {saved[k]}, this run {cfg[k]}")
            tr.load_state({"params": z["params"], "m": z["m"], "v": z["v"], "step": int(z["step"])})
            tr.lr = float(z["hyper"][0])
            g.set_state(torch.from_numpy(z["sampler_state"].copy()))
            start = int(z["next_step"])
        log(f"resumed at step {start}")
    ch, cw = cfg["crop"]
    B = cfg["batch"]
    bf = torch.empty((B, ch, cw, 4), dtype=torch.float32, device=dev)
    bl = torch.empty((B, ch, cw), dtype=torch.uint8, device=dev)
    nmaps = len(train_set)
    steps = cfg["steps"]
    hist = []
    t1 = time.time()
    kinds = sorted(set(train_set.kind))
    by_kind = [[k for k in range(nmaps) if train_set.kind[k] == kd] for kd in kinds]
    for step in range(start, steps):
        # Step decay of the learning rate: x0.3 at 60 % of the steps, x0.03 at 85 %.
        tr.lr = cfg["lr"] * (1.0 if step < int(0.6 * steps) else (0.3 if step < int(0.85 * steps) else 0.03))
        if cfg.get("balance"):
            # Each kind of map equally often, then a map of that kind.
            kk = torch.randint(0, len(kinds), (B,), generator=g)
            rr = torch.rand((B,), generator=g)
            idx = [by_kind[int(kk[b])][int(rr[b] * len(by_kind[int(kk[b])]))] for b in range(B)]
        else:
            idx = torch.randint(0, nmaps, (B,), generator=g)
        u = torch.rand((B, 2), generator=g)
        for b in range(B):
            i = int(idx[b])
            H, W = train_set.labels[i].shape
            y = int(u[b, 0] * (H - ch + 1))
            x = int(u[b, 1] * (W - cw + 1))
            bf[b].copy_(train_set.feats[i][y:y + ch, x:x + cw])
            bl[b].copy_(train_set.labels[i][y:y + ch, x:x + cw])
        loss = tr.step(bf, bl)
        if step % 500 == 0 or step == steps - 1:
            hist.append((step, float(loss.item())))
            log(f"step {step} loss {hist[-1][1]:.4f}")
        if cfg.get("ckpt") and cfg.get("ckpt_every") and (step + 1) % cfg["ckpt_every"] == 0:
            save_ckpt(cfg["ckpt"], tr, g, cfg, step + 1)
        if stop_after is not None and step + 1 >= stop_after:
            torch.cuda.synchronize()
            return tr, None
    torch.cuda.synchronize()
    t_train = time.time() - t1
    calib = None
    if cfg.get("calibrate", 0) > 0:
        calib = calibrate_bias(tr, train_set, cfg["calibrate"], dev)
        log(f"output bias shifted by {-calib:.4f} (agreement-maximising threshold on {cfg['calibrate']} training maps)")
    ev = {"val": evaluate(tr.params, val_set, dev), "train_maps": nmaps, "steps": steps, "batch": B,
          "bias_shift": None if calib is None else -calib,
          "crop": [ch, cw], "train_seconds": t_train, "data_seconds": t_data, "loss_history": hist,
          "config": {k: v for k, v in cfg.items() if k not in ("workers", "ckpt", "ckpt_every")}}
    if cfg.get("ckpt"):
        save_ckpt(cfg["ckpt"], tr, g, cfg, steps, ev)
    return tr, ev


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--t0", type=int, default=6000, help="training t0 pairs (1242x375)")
    ap.add_argument("--t1", type=int, default=3000, help="training t1 maps (1242x375 frames)")
    ap.add_argument("--big", type=int, default=400, help="training 2048x1024 frames (t0 and t1 maps)")
    ap.add_argument("--val-t0", type=int, default=32)
    ap.add_argument("--val-t1", type=int, default=32)
    ap.add_argument("--val-big", type=int, default=8)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, nargs=2, default=[128, 256])
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--workers", type=int, default=14)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="lrnet.npz")
    ap.add_argument("--ckpt", default=None, help="checkpoint file (written every --ckpt-every steps)")
    ap.add_argument("--ckpt-every", type=int, default=2000)
    ap.add_argument("--resume", default=None, help="continue the run saved in this checkpoint")
    ap.add_argument("--init", default=None, help="start from the weights of this .npz (fine-tuning)")
    ap.add_argument("--balance", action="store_true",
                    help="sample the kinds of maps (t0, t1, big) equally often instead of in proportion")
    ap.add_argument("--calibrate", type=int, default=0,
                    help="after training, shift the output bias to the agreement-maximising threshold "
                         "found on this many training maps of each kind (0: no shift)")
    ap.add_argument("--eval-only", default=None,
                    help="evaluate the parameters of this .npz on the validation maps and exit")
    ap.add_argument("--metrics-out", default=None, help="write the metrics to this JSON file")
    args = ap.parse_args()
    dev = "cuda:0"
    cfg = {"t0": args.t0, "t1": args.t1, "big": args.big, "val_t0": args.val_t0, "val_t1": args.val_t1,
           "val_big": args.val_big, "steps": args.steps, "batch": args.batch, "crop": list(args.crop),
           "lr": args.lr, "seed": args.seed, "workers": args.workers, "ckpt": args.ckpt,
           "ckpt_every": args.ckpt_every, "calibrate": args.calibrate, "balance": bool(args.balance),
           "init": args.init}
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.eval_only:
        with np.load(args.eval_only, allow_pickle=False) as z:
            params = torch.from_numpy(z["params"].astype(np.float32)).to(dev)
        vs = label_maps(jobs_for(args.val_t0, args.val_t1, args.val_big, val=True), args.workers, dev, keep_gt=True)
        ev = {"val": evaluate(params, vs, dev)}
    else:
        tr, ev = train(cfg, dev, log, resume=args.resume)
        st = tr.state()
        np.savez(args.out, params=st["params"], m=st["m"], v=st["v"], step=st["step"], metrics=json.dumps(ev))
    print(json.dumps(ev), flush=True)
    if args.metrics_out:
        with open(args.metrics_out, "w") as f:
            json.dump(ev, f, indent=1)


if __name__ == "__main__":
    main()
