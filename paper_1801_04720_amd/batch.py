"""Binding of the batched plain SGM (sf_batch_*) and of the aggregation autotuner.

Marshalling only: the plan, the waves, the task tables, the graph capture and
every kernel are in libsf.so.  The autotuner's choices are cached in a JSON
file keyed by GPU architecture and H x W x D."""
from __future__ import annotations

import ctypes as ct
import json
import os

import torch

from ._lib import SfAggTuning, SfPair, check, lib
from .api import Plan, _stream

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                             "autotune_cache.json")


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def tuning_dict(t: SfAggTuning) -> dict:
    return {"chains_per_block": t.chains_per_block, "prefetch": t.prefetch, "order": t.order,
            "persistent_per_cu": t.persistent_per_cu, "packed": t.packed}


def _from_cache(e: dict) -> SfAggTuning:
    return SfAggTuning(e["chains_per_block"], e["prefetch"], e["order"], e["persistent_per_cu"],
                       e.get("packed", 0))


def autotune(H: int, W: int, D: int, P1: int = 10, P2: int = 120, cache: str | None = DEFAULT_CACHE,
             stream=None, refresh: bool = False, nviews: int = 2) -> tuple[SfAggTuning, float | None]:
    """Fastest aggregation tuning for nviews views of H x W x D (2 = a stereo pair,
    4 = a scene-flow frame), cached per arch, size and view count."""
    key = f"{_arch()}:{H}x{W}x{D}:P1={P1}:P2={P2}" + (f":views={nviews}" if nviews != 2 else "")
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
    if key in db and not refresh:
        e = db[key]
        return _from_cache(e), e.get("ms")
    best = SfAggTuning()
    ms = ct.c_float(0.0)
    check(lib().sf_agg_autotune(H, W, D, P1, P2, nviews, _stream(stream), ct.byref(best), ct.byref(ms)))
    if cache:
        db[key] = dict(tuning_dict(best), ms=float(ms.value))
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best, float(ms.value)


def frame_autotune(H: int, W: int, D: int, P1: int = 10, P2: int = 120, lr_tol: int = 1, flags: int = 0,
                   cache: str | None = DEFAULT_CACHE, stream=None,
                   refresh: bool = False) -> tuple[SfAggTuning, float | None]:
    """Aggregation tuning with the fastest whole frame (sf_frame_autotune) for a
    frame plan of this size, penalties and flags, cached per arch and key."""
    key = f"{_arch()}:frame:{H}x{W}x{D}:P1={P1}:P2={P2}:tol={lr_tol}:flags={flags}"
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
    if key in db and not refresh:
        e = db[key]
        return _from_cache(e), e.get("ms")
    best = SfAggTuning()
    ms = ct.c_float(0.0)
    check(lib().sf_frame_autotune(H, W, D, P1, P2, lr_tol, flags, _stream(stream), ct.byref(best), ct.byref(ms)))
    if cache:
        db[key] = dict(tuning_dict(best), ms=float(ms.value))
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best, float(ms.value)


class Batch:
    """A batch of stereo pairs (dicts with uint8 'left', 'right' tensors on the GPU
    and 'D'); outputs per pair: wta int16, disp float32, valid uint8."""

    def __init__(self, pairs, P1=10, P2=120, lr_tol=1, tunings=None, mem_budget=0,
                 device="cuda:0"):
        self.pairs = pairs
        self.out = []
        arr = (SfPair * len(pairs))()
        for i, p in enumerate(pairs):
            L, R = p["left"], p["right"]
            H, W = L.shape
            o = {"wta": torch.empty((H, W), dtype=torch.int16, device=device),
                 "disp": torch.empty((H, W), dtype=torch.float32, device=device),
                 "valid": torch.empty((H, W), dtype=torch.uint8, device=device)}
            self.out.append(o)
            arr[i] = SfPair(H, W, int(p["D"]), L.stride(0), L.data_ptr(), R.data_ptr(),
                            o["wta"].data_ptr(), o["disp"].data_ptr(), o["valid"].data_ptr())
        classes = []
        for p in pairs:
            k = (p["left"].shape[0], p["left"].shape[1], int(p["D"]))
            if k not in classes:
                classes.append(k)
        self.classes = classes
        tun = None
        ntun = 0
        if tunings is not None:
            tun = (SfAggTuning * len(classes))()
            for c, k in enumerate(classes):
                t = tunings.get(k) if isinstance(tunings, dict) else tunings[c]
                tun[c] = t if t is not None else SfAggTuning(16, 8, 0, 0, 0)
            ntun = len(classes)
        h = ct.c_void_p()
        check(lib().sf_batch_plan_create(arr, len(pairs), P1, P2, lr_tol, tun, ntun, mem_budget,
                                         ct.byref(h)))
        self.plan = Plan(h)
        self._arr = arr
        self.ws = torch.empty(self.plan.workspace_bytes(), dtype=torch.uint8, device=device)
        nw, nc = ct.c_int(), ct.c_int()
        check(lib().sf_batch_plan_info(h, ct.byref(nw), ct.byref(nc)))
        self.nwaves, self.nclasses = nw.value, nc.value
        self.captured = False

    def run(self, stream=None):
        check(lib().sf_batch_run(self.plan.handle, ct.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                 _stream(stream)))
        return self.out

    def capture(self, stream):
        check(lib().sf_batch_capture(self.plan.handle, ct.c_void_p(self.ws.data_ptr()),
                                     self.ws.numel(), ct.c_void_p(stream.cuda_stream)))
        self.captured = True

    def launch(self, stream=None):
        check(lib().sf_batch_launch(self.plan.handle, _stream(stream)))
        return self.out
