"""Plain scene-flow frame on one GPU, composed from the C-ABI calls with all
buffers allocated once (Sec. 3: SGM on the t0 and t1 pairs, Sec. 3.3: the
combination with the given flow).

Per frame: census of the four images; for each time step the left-base and
right-base cost volumes and their 8-path aggregation, WTA + sub-pixel + LR
check; then the combination and triangulation.
"""
from __future__ import annotations

import torch

from . import api


class PlainFrame:
    """Per-stage frame: every stage is its own C-ABI call.  diag: right maps by
    the diagonal search in S_L; median: 3x3 median of the left sub-pixel maps
    before the LR mask."""

    def __init__(self, H: int, W: int, D: int, P1: int = 10, P2: int = 120, lr_tol: int = 1,
                 cam=(721.5, 0.54, None, None), path_mask: int = 0xFF, device="cuda:0",
                 diag: bool = False, median: bool = False, adaptive_p2: bool = False):
        self.H, self.W, self.D = H, W, D
        self.diag, self.median, self.adaptive = diag, median, adaptive_p2
        self.P1, self.P2, self.tol, self.mask = P1, P2, lr_tol, path_mask
        f, B, cx, cy = cam
        self.cam = (f, B, (W - 1) / 2.0 if cx is None else cx, (H - 1) / 2.0 if cy is None else cy)
        dev = torch.device(device)
        e = lambda *s, dt: torch.empty(s, dtype=dt, device=dev)  # noqa: E731
        self.cen = [e(H, W, dt=torch.int64) for _ in range(4)]
        self.cost = e(H, W, D, dt=torch.uint8)
        self.S_left = e(H, W, D, dt=torch.int16)
        self.S_right = e(H, W, D, dt=torch.int16)
        self.ws = e(api.sgm_workspace_bytes(H, W, D), dt=torch.uint8)
        self.maps = []
        for _ in range(2):
            self.maps.append({"wta_left": e(H, W, dt=torch.int16), "wta_right": e(H, W, dt=torch.int16),
                              "disp": e(H, W, dt=torch.float32), "valid": e(H, W, dt=torch.uint8),
                              "feat": None})
        self.out = {"sf4": e(H, W, 4, dt=torch.float32), "valid": e(H, W, dt=torch.uint8),
                    "xyz0": e(H, W, 3, dt=torch.float32), "motion": e(H, W, 3, dt=torch.float32)}
        self.dense = e(H, W, dt=torch.float32)
        self.ones = e(H, W, dt=torch.uint8)

    def _aggregate(self, base_img, out):
        if self.adaptive:
            api.sgm_aggregate_adaptive(self.cost, base_img, self.P1, self.P2, self.mask, out=out,
                                       workspace=self.ws)
        else:
            api.sgm_aggregate(self.cost, self.P1, self.P2, self.mask, out=out, workspace=self.ws)

    def disparity(self, t: int, left, right, cen_l, cen_r):
        api.census(left, out=cen_l)
        api.census(right, out=cen_r)
        m = self.maps[t]
        if not self.diag:
            api.cost(cen_r, cen_l, self.D, True, out=self.cost)
            self._aggregate(right, self.S_right)
        api.cost(cen_l, cen_r, self.D, False, out=self.cost)
        self._aggregate(left, self.S_left)
        if not self.diag and not self.median:
            return api.wta_lr(self.S_left, self.S_right, None, self.P2, self.tol, out=m)
        # Left WTA without a check (dense sub-pixel map), the right map, then the mask.
        api.wta_lr(self.S_left, None, None, self.P2, self.tol,
                   out={"wta_left": m["wta_left"], "disp": self.dense, "valid": self.ones,
                        "feat": None})
        if self.diag:
            api.wta_right_diag(self.S_left, out=m["wta_right"])
        else:
            api.wta_lr(self.S_right, None, None, self.P2, self.tol,
                       out={"wta_left": m["wta_right"], "disp": m["disp"], "valid": m["valid"],
                            "feat": None})
        api.lr_check(m["wta_left"], m["wta_right"], self.dense, self.tol, out=m)
        if self.median:
            api.median3x3(self.dense, m["valid"], out=m["disp"])
        return m

    def run(self, L0, R0, L1, R1, flow):
        m0 = self.disparity(0, L0, R0, self.cen[0], self.cen[1])
        m1 = self.disparity(1, L1, R1, self.cen[2], self.cen[3])
        out = api.combine(m0["disp"], m0["valid"], m1["disp"], m1["valid"], flow, self.cam,
                          out=self.out)
        return m0, m1, out


class FusedFrame:
    """The same frame through the fused sf_frame_run entry point: six launches,
    all four aggregations in one launch, S never materialised."""

    def __init__(self, H: int, W: int, D: int, P1: int = 10, P2: int = 120, lr_tol: int = 1,
                 cam=(721.5, 0.54, None, None), persistent: bool = False, learned_params=None,
                 tuning=None, device="cuda:0", diag: bool = False, median: bool = False,
                 adaptive_p2: bool = False):
        self.H, self.W, self.D = H, W, D
        f, B, cx, cy = cam
        self.cam = (f, B, (W - 1) / 2.0 if cx is None else cx, (H - 1) / 2.0 if cy is None else cy)
        self.params = learned_params
        self.plan = api.frame_plan(H, W, D, P1, P2, lr_tol, persistent,
                                   learned=learned_params is not None, tuning=tuning, diag=diag,
                                   median=median, adaptive_p2=adaptive_p2)
        dev = torch.device(device)
        e = lambda *s, dt: torch.empty(s, dtype=dt, device=dev)  # noqa: E731
        self.ws = e(self.plan.workspace_bytes(), dt=torch.uint8)
        self.out = {"disp0": e(H, W, dt=torch.float32), "valid0": e(H, W, dt=torch.uint8),
                    "disp1": e(H, W, dt=torch.float32), "valid1": e(H, W, dt=torch.uint8),
                    "sf4": e(H, W, 4, dt=torch.float32), "valid": e(H, W, dt=torch.uint8),
                    "xyz0": e(H, W, 3, dt=torch.float32), "motion": e(H, W, 3, dt=torch.float32)}

    def run(self, L0, R0, L1, R1, flow):
        if self.params is not None:
            return api.frame_run_learned(self.plan, L0, R0, L1, R1, flow, self.cam, self.params,
                                         self.out, self.ws)
        return api.frame_run(self.plan, L0, R0, L1, R1, flow, self.cam, self.out, self.ws)


class JudgedLearnedStream:
    """Learned frames with the full left-right check (Sec. 3.1) as judge and as
    fallback.

    Every `judge_every`-th frame (the first included) runs both the plain frame
    and the learned frame; the plain result is delivered, and the agreement of
    the two frames' masks (the lower of the t0 and t1 maps, counted by
    sf_mask_agreement and read back once per judged frame) sets the mode of
    the frames up to the next judge: learned frames while it is at least
    `threshold`, plain frames (the fallback) otherwise.  A fallback frame is
    the plain frame itself, so its outputs equal the plain frame's bit for bit.
    `history` holds (frame index, agreement t0, agreement t1, mode chosen)."""

    def __init__(self, H: int, W: int, D: int, params, judge_every: int = 16, threshold: float = 0.99,
                 tuning_learned=None, tuning_plain=None, device="cuda:0", learned=None, plain=None, **kw):
        """learned / plain: existing FusedFrame objects of this size to reuse (their
        plans and buffers); otherwise both are created here."""
        if judge_every < 1:
            raise ValueError("judge_every must be >= 1")
        self.learned = learned or FusedFrame(H, W, D, learned_params=params, tuning=tuning_learned, device=device,
                                             **kw)
        self.plain = plain or FusedFrame(H, W, D, tuning=tuning_plain, device=device, **kw)
        self.judge_every, self.threshold = judge_every, float(threshold)
        self.count = torch.zeros(2, dtype=torch.int32, device=device)
        self.count_host = torch.zeros(2, dtype=torch.int32).pin_memory()
        self.npx = H * W
        self.k = 0
        self.mode = "learned"
        self.history = []

    def run(self, L0, R0, L1, R1, flow):
        judged = self.k % self.judge_every == 0
        k = self.k
        self.k += 1
        if judged:
            lo = self.learned.run(L0, R0, L1, R1, flow)
            po = self.plain.run(L0, R0, L1, R1, flow)
            api.mask_agreement(lo["valid0"], po["valid0"], out=self.count[0:1])
            api.mask_agreement(lo["valid1"], po["valid1"], out=self.count[1:2])
            self.count_host.copy_(self.count, non_blocking=True)
            torch.cuda.current_stream().synchronize()
            a0, a1 = (int(v) / self.npx for v in self.count_host.tolist())
            self.mode = "learned" if min(a0, a1) >= self.threshold else "plain"
            self.history.append((k, a0, a1, self.mode))
            return po
        if self.mode == "plain":
            return self.plain.run(L0, R0, L1, R1, flow)
        return self.learned.run(L0, R0, L1, R1, flow)


class SequenceFrames:
    """Scene flow over T time steps of one stereo rig (the paper's future work:
    more than two frame pairs with an intermediate validation): every time
    step's disparity map is computed once (the T pairs in one batch plan), the
    combination runs for each consecutive pair, and each scene-flow map but the
    last is checked against the next one along its own flow.

    lefts, rights: T uint8 [H][W] tensors on the GPU (bound to the plan)."""

    def __init__(self, lefts, rights, D: int, P1: int = 10, P2: int = 120, lr_tol: int = 1,
                 cam=(721.5, 0.54, None, None), tau_f: float = 2.0, tau_d: float = 1.0,
                 tuning=None, device="cuda:0"):
        from . import batch as _batch

        self.T = len(lefts)
        H, W = lefts[0].shape
        self.H, self.W, self.D = H, W, D
        f, B, cx, cy = cam
        self.cam = (f, B, (W - 1) / 2.0 if cx is None else cx, (H - 1) / 2.0 if cy is None else cy)
        self.tau_f, self.tau_d = tau_f, tau_d
        pairs = [{"left": L, "right": R, "D": D} for L, R in zip(lefts, rights)]
        self.batch = _batch.Batch(pairs, P1, P2, lr_tol, tunings=[tuning] if tuning is not None else None,
                                  device=device)
        dev = torch.device(device)
        e = lambda *s, dt: torch.empty(s, dtype=dt, device=dev)  # noqa: E731
        self.S = [{"sf4": e(H, W, 4, dt=torch.float32), "valid": e(H, W, dt=torch.uint8),
                   "xyz0": e(H, W, 3, dt=torch.float32), "motion": e(H, W, 3, dt=torch.float32)}
                  for _ in range(self.T - 1)]
        self.temporal = [e(H, W, dt=torch.uint8) for _ in range(max(0, self.T - 2))]

    def run(self, flows):
        """flows: T-1 float [H][W][2] tensors (t_k -> t_k+1).  Returns (maps,
        scene flows, temporal masks)."""
        maps = self.batch.launch() if self.batch.captured else self.batch.run()
        for k in range(self.T - 1):
            api.combine(maps[k]["disp"], maps[k]["valid"], maps[k + 1]["disp"], maps[k + 1]["valid"],
                        flows[k], self.cam, out=self.S[k])
        for k in range(self.T - 2):
            api.temporal_check(self.S[k]["sf4"], self.S[k]["valid"], self.S[k + 1]["sf4"],
                               self.S[k + 1]["valid"], self.tau_f, self.tau_d, out=self.temporal[k])
        return maps, self.S, self.temporal
