"""Train the learned stand-in for the LR check on seeded synthetic pairs.

Pairs are 1242x375, D = 128, piecewise-planar scenes (the shape of the paper's
KITTI frames; KITTI itself is not used).  Each pair goes through the plain GPU
path once: its left-view features and its LR-check labels stay resident in
HBM.  Training samples random crops and runs the HIP forward / backward /
Adam kernels; validation runs the full network on held-out pairs and compares
the learned mask with the LR check.

    python -m paper_1801_04720_amd.train_lrnet --pairs 512 --steps 3000 --out lrnet.npz
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

H, W, D = 375, 1242, 128


def _gen(i):
    p = synth.pair_planar(synth.rng_for(4, i), H, W, D)
    return p.left, p.right, p.gt_disp, p.occluded


def label_pairs(indices, workers, dev="cuda:0", keep_gt=False):
    """Features [N][H][W][4], LR labels [N][H][W], WTA, sub-pixel disparity."""
    n = len(indices)
    feats = torch.empty((n, H, W, 4), dtype=torch.float32, device=dev)
    labels = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    wtas = torch.empty((n, H, W), dtype=torch.int16, device=dev) if keep_gt else None
    dsubs = torch.empty((n, H, W), dtype=torch.float32, device=dev) if keep_gt else None
    gts, occs = [], []
    cost = torch.empty((H, W, D), dtype=torch.uint8, device=dev)
    Sl = torch.empty((H, W, D), dtype=torch.int16, device=dev)
    Sr = torch.empty((H, W, D), dtype=torch.int16, device=dev)
    ws = torch.empty(api.sgm_workspace_bytes(H, W, D), dtype=torch.uint8, device=dev)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        for k, (L, R, gt, occ) in enumerate(ex.map(_gen, indices, chunksize=4)):
            Lt = torch.from_numpy(L).to(dev)
            Rt = torch.from_numpy(R).to(dev)
            cl, cr = api.census(Lt), api.census(Rt)
            api.cost(cr, cl, D, True, out=cost)
            api.sgm_aggregate(cost, 10, 120, out=Sr, workspace=ws)
            api.cost(cl, cr, D, False, out=cost)
            api.sgm_aggregate(cost, 10, 120, out=Sl, workspace=ws)
            o = {"feat": feats[k], "valid": labels[k]}
            if keep_gt:
                o["wta_left"] = wtas[k]
                o["disp"] = dsubs[k]
                gts.append(gt)
                occs.append(occ)
            api.wta_lr(Sl, Sr, Lt, 120, 1, want_feat=True, out=o)
    torch.cuda.synchronize()
    return feats, labels, wtas, dsubs, gts, occs


def evaluate(params, feats, labels, wtas, dsubs, gts, occs, dev="cuda:0"):
    """Agreement with the LR check, EPE vs ground truth and density on both masks."""
    n = feats.shape[0]
    xs = torch.arange(W, device=dev)[None, None, :]
    agree = 0.0
    tp = fp = fn = tn = 0
    epe_l, epe_p, den_l, den_p = [], [], [], []
    # Baselines without a learned or LR mask: keep every pixel ("no check"), or
    # drop only those whose match falls outside the right image (x - d* < 0).
    epe_n, den_n, epe_g, den_g, agree_g = [], [], [], [], 0.0
    for k in range(n):
        logits = lrnet.forward(params, feats[k:k + 1])
        learned = (logits[0] > 0) & ((xs[0] - wtas[k].long()) >= 0)
        lab = labels[k].bool()
        agree += float((learned == lab).float().mean().item())
        tp += int((learned & lab).sum())
        tn += int((~learned & ~lab).sum())
        fp += int((learned & ~lab).sum())
        fn += int((~learned & lab).sum())
        gt = torch.from_numpy(gts[k]).to(dev)
        err = (dsubs[k] - gt).abs()
        geom = (xs[0] - wtas[k].long()) >= 0
        nocheck = torch.ones_like(lab)
        agree_g += float((geom == lab).float().mean().item())
        for m, e, d in ((learned, epe_l, den_l), (lab, epe_p, den_p), (nocheck, epe_n, den_n),
                        (geom, epe_g, den_g)):
            e.append(float(err[m].mean().item()))
            d.append(float(m.float().mean().item()))
    return {"agreement": agree / n, "tp": tp, "tn": tn, "fp": fp, "fn": fn,
            "epe_learned_mask": float(np.mean(epe_l)), "epe_lr_mask": float(np.mean(epe_p)),
            "density_learned": float(np.mean(den_l)), "density_lr": float(np.mean(den_p)),
            "agreement_no_check": float(sum(float(labels[k].float().mean()) for k in range(n)) / n),
            "epe_no_check": float(np.mean(epe_n)), "density_no_check": float(np.mean(den_n)),
            "agreement_geometric": agree_g / n, "epe_geometric_mask": float(np.mean(epe_g)),
            "density_geometric": float(np.mean(den_g))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=512)
    ap.add_argument("--val", type=int, default=16)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, nargs=2, default=[128, 256])
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="lrnet.npz")
    ap.add_argument("--eval-only", default=None,
                    help="evaluate the parameters of this .npz on the validation pairs and exit")
    ap.add_argument("--metrics-out", default=None,
                    help="with --eval-only: merge the metrics into this JSON file")
    args = ap.parse_args()
    dev = "cuda:0"
    if args.eval_only:
        with np.load(args.eval_only, allow_pickle=False) as z:
            params = torch.from_numpy(z["params"].astype(np.float32)).to(dev)
        vf, vl, vw, vd, vg, vo = label_pairs(list(range(100000, 100000 + args.val)), args.workers,
                                              dev, keep_gt=True)
        ev = evaluate(params, vf, vl, vw, vd, vg, vo, dev)
        ev["val_pairs"] = args.val
        print(json.dumps(ev), flush=True)
        if args.metrics_out:
            old = {}
            if os.path.exists(args.metrics_out):
                with open(args.metrics_out) as f:
                    old = json.load(f)
            old.update(ev)
            with open(args.metrics_out, "w") as f:
                json.dump(old, f, indent=1)
        return
    t0 = time.time()
    feats, labels, _, _, _, _ = label_pairs(list(range(args.pairs)), args.workers, dev)
    vf, vl, vw, vd, vg, vo = label_pairs(list(range(100000, 100000 + args.val)), args.workers, dev,
                                          keep_gt=True)
    t_data = time.time() - t0
    print(f"labelled {args.pairs} + {args.val} pairs in {t_data:.1f} s", flush=True)
    tr = lrnet.Trainer(lrnet.init_params(args.seed), lr=args.lr, device=dev)
    g = torch.Generator(device="cpu").manual_seed(args.seed)
    ch, cw = args.crop
    bf = torch.empty((args.batch, ch, cw, 4), dtype=torch.float32, device=dev)
    bl = torch.empty((args.batch, ch, cw), dtype=torch.uint8, device=dev)
    t1 = time.time()
    hist = []
    for step in range(args.steps):
        idx = torch.randint(0, args.pairs, (args.batch,), generator=g)
        ys = torch.randint(0, H - ch + 1, (args.batch,), generator=g)
        xs = torch.randint(0, W - cw + 1, (args.batch,), generator=g)
        for b in range(args.batch):
            i, y, x = int(idx[b]), int(ys[b]), int(xs[b])
            bf[b].copy_(feats[i, y:y + ch, x:x + cw])
            bl[b].copy_(labels[i, y:y + ch, x:x + cw])
        loss = tr.step(bf, bl)
        if step % 250 == 0 or step == args.steps - 1:
            hist.append((step, float(loss.item())))
            print(f"step {step} loss {hist[-1][1]:.4f}", flush=True)
        if step == int(0.7 * args.steps):
            tr.lr *= 0.3
    torch.cuda.synchronize()
    t_train = time.time() - t1
    ev = evaluate(tr.params, vf, vl, vw, vd, vg, vo, dev)
    ev.update({"pairs": args.pairs, "val_pairs": args.val, "steps": args.steps, "batch": args.batch,
               "crop": [ch, cw], "train_seconds": t_train, "data_seconds": t_data,
               "loss_history": hist})
    print(json.dumps(ev), flush=True)
    st = tr.state()
    np.savez(args.out, params=st["params"], m=st["m"], v=st["v"], step=st["step"],
             metrics=json.dumps(ev))


if __name__ == "__main__":
    main()
