"""Scene-flow accuracy against the synthetic ground truth, in the outlier
convention the paper's Table 1 reports (the KITTI metric): an estimate is an
outlier when its error exceeds both 3 px and 5 % of the true value (disparity:
absolute difference; flow: end-point error of (u, v)); a scene-flow estimate is
an outlier when its d0, d1 or flow is.  Table 1 gives these rates for the
sparse estimate ("Est", over the pixels it defines, with its density) and for
a dense version ("All", over every pixel)."""
from __future__ import annotations

import torch


def _outlier(err, ref):
    return (err > 3.0) & (err > 0.05 * ref.abs())


def sf_outliers(sf4, defined, gt_flow, gt_d0, gt_d1, region=None) -> dict:
    """Outlier percentages D1 (d0), D2 (d1), Fl (flow), SF (any) over the pixels
    of `region` (default: all) that `defined` marks, and the density = defined
    share of the region.  sf4 [H][W][4] (u, v, d0, d1); gt_flow [H][W][2];
    gt_d0, gt_d1 [H][W] (d1 at the t0 pixel)."""
    dev = sf4.device
    gt_flow = torch.as_tensor(gt_flow, device=dev, dtype=torch.float32)
    gt_d0 = torch.as_tensor(gt_d0, device=dev, dtype=torch.float32)
    gt_d1 = torch.as_tensor(gt_d1, device=dev, dtype=torch.float32)
    reg = torch.ones_like(gt_d0, dtype=torch.bool) if region is None else torch.as_tensor(region, device=dev)
    m = reg & defined.bool()
    n = int(m.sum().item())
    out = {"density": float(n / max(1, int(reg.sum().item())))}
    if n == 0:
        return out | {"D1": None, "D2": None, "Fl": None, "SF": None}
    d1o = _outlier((sf4[..., 2] - gt_d0).abs(), gt_d0)
    d2o = _outlier((sf4[..., 3] - gt_d1).abs(), gt_d1)
    fe = torch.linalg.norm(sf4[..., :2] - gt_flow, dim=-1)
    flo = _outlier(fe, torch.linalg.norm(gt_flow, dim=-1))
    sfo = d1o | d2o | flo
    pct = lambda o: float(100.0 * (o & m).sum().item() / n)  # noqa: E731
    return out | {"D1": pct(d1o), "D2": pct(d2o), "Fl": pct(flo), "SF": pct(sfo)}
