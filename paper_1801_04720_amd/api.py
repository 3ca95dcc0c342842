"""Python binding of the C ABI: the same entry points, torch tensors in/out.

Argument marshalling only.  Every step of the path runs in the HIP kernels of
libsf.so on the caller's current torch stream; torch provides device memory
and streams.  Integer volumes use torch's signed dtypes as bit containers:
census descriptors live in int64 tensors (view them as uint64), aggregated
costs in int16 tensors (view them as uint16).
"""
from __future__ import annotations

import ctypes as ct

import torch

from . import _lib
from ._lib import SfCamera, check, lib

CMAX = 62


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("sf: tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("sf: tensors must be contiguous")
    return ct.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def abi_version() -> int:
    return lib().sf_abi_version()


def census(img: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """9x7 census of a uint8 [H][W] image -> int64 [H][W] (62-bit descriptors)."""
    H, W = img.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.int64, device=img.device)
    check(lib().sf_census(_ptr(img), H, W, img.stride(0), _ptr(out), _stream(stream)))
    return out


def cost(cen_base, cen_match, D: int, base_is_right: bool, out=None, stream=None):
    """Hamming cost volume uint8 [H][W][D]."""
    H, W = cen_base.shape
    if out is None:
        out = torch.empty((H, W, D), dtype=torch.uint8, device=cen_base.device)
    check(lib().sf_cost(_ptr(cen_base), _ptr(cen_match), H, W, D, int(base_is_right), _ptr(out),
                        _stream(stream)))
    return out


def sgm_workspace_bytes(H: int, W: int, D: int) -> int:
    return int(lib().sf_sgm_workspace_bytes(H, W, D))


def sgm_set_epilogue(mode: int) -> None:
    """0 = automatic, 1 = per-direction u8 slabs + sum, 2 = packed atomics into S."""
    check(lib().sf_sgm_set_epilogue(mode))


def sgm_aggregate(cost_vol, P1: int, P2: int, path_mask: int = 0xFF, out=None, workspace=None,
                  stream=None):
    """Aggregated costs S (int16 container of uint16 values) [H][W][D]."""
    H, W, D = cost_vol.shape
    if out is None:
        out = torch.empty((H, W, D), dtype=torch.int16, device=cost_vol.device)
    if workspace is None:
        workspace = torch.empty(sgm_workspace_bytes(H, W, D), dtype=torch.uint8,
                                device=cost_vol.device)
    check(lib().sf_sgm_aggregate(_ptr(cost_vol), H, W, D, P1, P2, path_mask, _ptr(out),
                                 _ptr(workspace), workspace.numel(), _stream(stream)))
    return out


def sgm_aggregate_census(cen_base, cen_match, D: int, base_is_right: bool, P1: int, P2: int,
                         path_mask: int = 0xFF, out=None, workspace=None, stream=None):
    """Aggregated costs S [H][W][D] with the Hamming costs computed inside the
    aggregation from the two census images (no cost volume); equal to
    sgm_aggregate(cost(cen_base, cen_match, D, base_is_right), P1, P2, path_mask)."""
    H, W = cen_base.shape
    if out is None:
        out = torch.empty((H, W, D), dtype=torch.int16, device=cen_base.device)
    if workspace is None:
        workspace = torch.empty(sgm_workspace_bytes(H, W, D), dtype=torch.uint8,
                                device=cen_base.device)
    check(lib().sf_sgm_aggregate_census(_ptr(cen_base), _ptr(cen_match), H, W, D, int(base_is_right), P1,
                                        P2, path_mask, _ptr(out), _ptr(workspace), workspace.numel(),
                                        _stream(stream)))
    return out


def wta_lr(S_left, S_right=None, img_left=None, P2: int = 120, lr_tol: int = 1, want_feat=False,
           out=None, stream=None):
    """WTA + sub-pixel + LR check (+ features).

    Returns dict with wta_left int16, wta_right int16 (or None), disp float32,
    valid uint8, feat float32 [H][W][4] (or None)."""
    H, W, D = S_left.shape
    dev = S_left.device
    o = out or {}
    wl = o.get("wta_left")
    if wl is None:
        wl = torch.empty((H, W), dtype=torch.int16, device=dev)
    wr = o.get("wta_right")
    if S_right is not None and wr is None:
        wr = torch.empty((H, W), dtype=torch.int16, device=dev)
    disp = o.get("disp")
    if disp is None:
        disp = torch.empty((H, W), dtype=torch.float32, device=dev)
    valid = o.get("valid")
    if valid is None:
        valid = torch.empty((H, W), dtype=torch.uint8, device=dev)
    feat = o.get("feat")
    if want_feat and feat is None:
        feat = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
    if not want_feat:
        feat = None
    pitch = img_left.stride(0) if img_left is not None else W
    check(lib().sf_wta_lr(_ptr(S_left), _ptr(S_right), _ptr(img_left), pitch, H, W, D, P2, lr_tol,
                          _ptr(wl), _ptr(wr) if S_right is not None else None, _ptr(disp),
                          _ptr(valid), _ptr(feat), _stream(stream)))
    return {"wta_left": wl, "wta_right": wr if S_right is not None else None, "disp": disp,
            "valid": valid, "feat": feat}


def combine(disp0, valid0, disp1, valid1, flow, cam=None, out=None, stream=None):
    """Scene-flow map (Sec. 3.3) and, with cam = (f, B, cx, cy), 3-D points / motion."""
    H, W = disp0.shape
    dev = disp0.device
    o = out or {}
    sf4 = o.get("sf4")
    if sf4 is None:
        sf4 = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
    valid = o.get("valid")
    if valid is None:
        valid = torch.empty((H, W), dtype=torch.uint8, device=dev)
    xyz0 = motion = None
    camp = None
    if cam is not None:
        xyz0 = o.get("xyz0")
        if xyz0 is None:
            xyz0 = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
        motion = o.get("motion")
        if motion is None:
            motion = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
        camp = ct.byref(SfCamera(*[float(c) for c in cam]))
    check(lib().sf_combine(_ptr(disp0), _ptr(valid0), _ptr(disp1), _ptr(valid1), _ptr(flow), H, W,
                           camp, _ptr(sf4), _ptr(valid), _ptr(xyz0), _ptr(motion),
                           _stream(stream)))
    return {"sf4": sf4, "valid": valid, "xyz0": xyz0, "motion": motion}


class Plan:
    """Owner of an sf_plan handle (destroyed with the object)."""

    def __init__(self, handle: ct.c_void_p):
        self.handle = handle

    def workspace_bytes(self) -> int:
        return int(lib().sf_plan_workspace_bytes(self.handle))

    def close(self):
        if self.handle:
            lib().sf_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sgm_aggregate_adaptive(cost_vol, img, P1: int, P2: int, path_mask: int = 0xFF, out=None,
                           workspace=None, stream=None):
    """S with the intensity-adaptive large-jump penalty (img = the base image)."""
    H, W, D = cost_vol.shape
    if out is None:
        out = torch.empty((H, W, D), dtype=torch.int16, device=cost_vol.device)
    if workspace is None:
        workspace = torch.empty(sgm_workspace_bytes(H, W, D), dtype=torch.uint8,
                                device=cost_vol.device)
    check(lib().sf_sgm_aggregate_adaptive(_ptr(cost_vol), _ptr(img), img.stride(0), H, W, D, P1,
                                          P2, path_mask, _ptr(out), _ptr(workspace),
                                          workspace.numel(), _stream(stream)))
    return out


def wta_right_diag(S_left, out=None, stream=None):
    """Right-view d* by the diagonal search in the left volume (no right aggregation)."""
    H, W, D = S_left.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.int16, device=S_left.device)
    check(lib().sf_wta_right_diag(_ptr(S_left), H, W, D, _ptr(out), _stream(stream)))
    return out


def lr_check(wta_left, wta_right, dsub, lr_tol: int = 1, out=None, stream=None):
    """LR check of given maps -> {"valid", "disp"}."""
    H, W = wta_left.shape
    if out is None:
        out = {"valid": torch.empty((H, W), dtype=torch.uint8, device=wta_left.device),
               "disp": torch.empty((H, W), dtype=torch.float32, device=wta_left.device)}
    check(lib().sf_lr_check(_ptr(wta_left), _ptr(wta_right), _ptr(dsub), H, W, lr_tol,
                            _ptr(out["valid"]), _ptr(out["disp"]), _stream(stream)))
    return out


def median3x3(m, mask=None, out=None, stream=None):
    """3x3 median (clamp-to-edge) of a float [H][W] map; -1 where mask == 0."""
    H, W = m.shape
    if out is None:
        out = torch.empty_like(m)
    check(lib().sf_median3x3(_ptr(m), _ptr(mask), H, W, _ptr(out), _stream(stream)))
    return out


def densify(sf4, valid, out=None, stream=None):
    """Dense scene-flow map -> {"sf4": [H][W][4] float, "fill": [H][W] uint8}."""
    H, W = valid.shape
    dev = valid.device
    o = out or {}
    dense = o.get("sf4")
    if dense is None:
        dense = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
    fill = o.get("fill")
    if fill is None:
        fill = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ws = o.get("workspace")
    if ws is None:
        ws = torch.empty(max(1, lib().sf_densify_workspace_bytes(H)), dtype=torch.uint8, device=dev)
    check(lib().sf_densify(_ptr(sf4), _ptr(valid), H, W, _ptr(dense), _ptr(fill), _ptr(ws), ws.numel(),
                           _stream(stream)))
    return {"sf4": dense, "fill": fill}


def temporal_check(sf4_a, valid_a, sf4_b, valid_b, tau_f: float = 2.0, tau_d: float = 1.0,
                   out=None, stream=None):
    """uint8 [H][W]: 1 where S_a is kept by the check against S_b along its flow."""
    H, W = valid_a.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=valid_a.device)
    check(lib().sf_temporal_check(_ptr(sf4_a), _ptr(valid_a), _ptr(sf4_b), _ptr(valid_b), H, W,
                                  float(tau_f), float(tau_d), _ptr(out), _stream(stream)))
    return out


def flow(L0, L1, levels: int = 5, iters: int = 6, R: int = 128, seed: int = 1801, tol: int = 1,
         fine_radius: int = 0, out=None, stream=None):
    """Optical-flow stand-in -> {"flow": [H][W][2] float (NaN where the
    forward-backward check drops it), "F", "B": [H][W][2] int16}."""
    H, W = L0.shape
    dev = L0.device
    o = out or {}
    F = o.get("F")
    if F is None:
        F = torch.empty((H, W, 2), dtype=torch.int16, device=dev)
    B = o.get("B")
    if B is None:
        B = torch.empty((H, W, 2), dtype=torch.int16, device=dev)
    fl = o.get("flow")
    if fl is None:
        fl = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
    ws = o.get("workspace")
    if ws is None:
        ws = torch.empty(lib().sf_flow_workspace_bytes(H, W, levels), dtype=torch.uint8, device=dev)
    check(lib().sf_flow(_ptr(L0), _ptr(L1), L0.stride(0), H, W, levels, iters, R, fine_radius, seed, tol, _ptr(F),
                        _ptr(B), _ptr(fl), _ptr(ws), ws.numel(), _stream(stream)))
    return {"flow": fl, "F": F, "B": B, "workspace": ws}


def mask_agreement(a, b, out=None, stream=None):
    """Device u32 count of the pixels where masks a and b agree (sf_mask_agreement)."""
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=a.device)
    assert a.numel() == b.numel()
    check(lib().sf_mask_agreement(_ptr(a), _ptr(b), a.numel(), _ptr(out), _stream(stream)))
    return out


FRAME_PERSISTENT, FRAME_LEARNED, FRAME_DIAG, FRAME_MEDIAN, FRAME_ADAPTIVE_P2 = 1, 2, 4, 8, 16


def frame_plan(H: int, W: int, D: int, P1: int = 10, P2: int = 120, lr_tol: int = 1,
               persistent: bool = False, learned: bool = False, tuning=None, diag: bool = False,
               median: bool = False, adaptive_p2: bool = False) -> Plan:
    """tuning: an _lib.SfAggTuning for the aggregation launch (None = default).
    diag: right maps by the diagonal search (plain frames); median: 3x3 median of
    the left sub-pixel maps before the mask."""
    h = ct.c_void_p()
    flags = ((FRAME_PERSISTENT if persistent else 0) | (FRAME_LEARNED if learned else 0) |
             (FRAME_DIAG if diag else 0) | (FRAME_MEDIAN if median else 0) |
             (FRAME_ADAPTIVE_P2 if adaptive_p2 else 0))
    tp = ct.byref(tuning) if tuning is not None else None
    check(lib().sf_frame_plan_create(H, W, D, P1, P2, lr_tol, flags, tp, ct.byref(h)))
    return Plan(h)


def frame_run(plan: Plan, L0, R0, L1, R1, flow, cam, out: dict, workspace, stream=None):
    """Fused plain frame; `out` holds disp0, valid0, disp1, valid1, sf4, valid, xyz0, motion."""
    camp = ct.byref(SfCamera(*[float(c) for c in cam])) if cam is not None else None
    check(lib().sf_frame_run(plan.handle, _ptr(L0), _ptr(R0), _ptr(L1), _ptr(R1), L0.stride(0),
                             _ptr(flow), camp, _ptr(out["disp0"]), _ptr(out["valid0"]),
                             _ptr(out["disp1"]), _ptr(out["valid1"]), _ptr(out["sf4"]),
                             _ptr(out["valid"]), _ptr(out.get("xyz0")), _ptr(out.get("motion")),
                             _ptr(workspace), workspace.numel(), _stream(stream)))
    return out


def frame_run_learned(plan: Plan, L0, R0, L1, R1, flow, cam, params, out: dict, workspace,
                      stream=None):
    """Learned frame: right views skipped, validity from the network's mask."""
    camp = ct.byref(SfCamera(*[float(c) for c in cam])) if cam is not None else None
    check(lib().sf_frame_run_learned(plan.handle, _ptr(L0), _ptr(R0), _ptr(L1), _ptr(R1),
                                     L0.stride(0), _ptr(flow), camp, _ptr(params),
                                     _ptr(out["disp0"]), _ptr(out["valid0"]), _ptr(out["disp1"]),
                                     _ptr(out["valid1"]), _ptr(out["sf4"]), _ptr(out["valid"]),
                                     _ptr(out.get("xyz0")), _ptr(out.get("motion")),
                                     _ptr(workspace), workspace.numel(), _stream(stream)))
    return out
