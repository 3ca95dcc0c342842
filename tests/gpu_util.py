"""Helpers shared by the GPU tests: host<->device moves and the tolerance of
FP32 outputs (|gpu - oracle| <= 1e-5 * max(|oracle|, scale))."""
import numpy as np
import torch

DEV = "cuda:0"


def dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to(DEV)


def host(t: torch.Tensor, as_dtype=None) -> np.ndarray:
    a = t.detach().cpu().numpy()
    if as_dtype is not None:
        a = a.view(as_dtype)
    return a


def assert_close_rel(gpu, ref, scale=1.0, rel=1e-5, what=""):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    nan_g, nan_r = np.isnan(gpu), np.isnan(ref)
    assert np.array_equal(nan_g, nan_r), f"{what}: NaN pattern differs at {np.argwhere(nan_g != nan_r)[:5]}"
    ok = ~nan_r
    scale = np.broadcast_to(np.asarray(scale, np.float64), ref.shape)
    tol = rel * np.maximum(np.abs(ref[ok]), scale[ok])
    err = np.abs(gpu[ok] - ref[ok])
    bad = err > tol
    assert not bad.any(), f"{what}: {bad.sum()} values beyond tolerance, max err {err.max()}"
