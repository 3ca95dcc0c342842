"""Binding and training loop of the learned stand-in for the LR check.

Marshalling only: forward, loss/gradient and the Adam step are HIP kernels of
libsf.so (sf_lrnet_forward / sf_lrnet_grad / sf_lrnet_backward / sf_lrnet_adam)."""
from __future__ import annotations

import numpy as np
import torch

from ._lib import check, lib
from .api import _ptr, _stream

NPARAM = 5377
OFFSETS = {"W1": 0, "b1": 576, "W2": 592, "b2": 2896, "W3": 2912, "b3": 5216, "W4": 5232, "b4": 5376}


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation of the flat FP32 parameter vector."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, np.float32)
    p[0:576] = rng.standard_normal(576) * np.sqrt(2.0 / 36)
    p[576:592] = 0.01
    p[592:2896] = rng.standard_normal(2304) * np.sqrt(2.0 / 144)
    p[2896:2912] = 0.01
    p[2912:5216] = rng.standard_normal(2304) * np.sqrt(2.0 / 144)
    p[5216:5232] = 0.01
    p[5232:5376] = rng.standard_normal(144) * np.sqrt(1.0 / 144)
    p[5376] = 2.0  # most pixels pass the check
    return p


def workspace_bytes(B: int, H: int, W: int, train: bool) -> int:
    return int(lib().sf_lrnet_workspace_bytes(B, H, W, int(train)))


def forward(params, feat, logits=None, workspace=None, stream=None):
    B, H, W, _ = feat.shape
    if logits is None:
        logits = torch.empty((B, H, W), dtype=torch.float32, device=feat.device)
    if workspace is None:
        workspace = torch.empty(workspace_bytes(B, H, W, False), dtype=torch.uint8, device=feat.device)
    check(lib().sf_lrnet_forward(_ptr(params), _ptr(feat), B, H, W, _ptr(logits), _ptr(workspace),
                                 workspace.numel(), _stream(stream)))
    return logits


def mask(logits, wta, dsub, valid=None, disp=None, stream=None):
    H, W = wta.shape
    if valid is None:
        valid = torch.empty((H, W), dtype=torch.uint8, device=wta.device)
    if disp is None:
        disp = torch.empty((H, W), dtype=torch.float32, device=wta.device)
    check(lib().sf_lrnet_mask(_ptr(logits), _ptr(wta), _ptr(dsub), H, W, _ptr(valid), _ptr(disp),
                              _stream(stream)))
    return valid, disp


def grad(params, feat, label, grad_out=None, loss_out=None, workspace=None, stream=None):
    B, H, W, _ = feat.shape
    dev = feat.device
    if grad_out is None:
        grad_out = torch.empty(NPARAM, dtype=torch.float32, device=dev)
    if loss_out is None:
        loss_out = torch.empty(1, dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = torch.empty(workspace_bytes(B, H, W, True), dtype=torch.uint8, device=dev)
    check(lib().sf_lrnet_grad(_ptr(params), _ptr(feat), _ptr(label), B, H, W, _ptr(grad_out),
                              _ptr(loss_out), _ptr(workspace), workspace.numel(), _stream(stream)))
    return grad_out, loss_out


def backward(params, feat, dz4, grad_out=None, workspace=None, stream=None):
    """Parameter gradient for a given dL/dz4 [B][H][W] (sf_lrnet_backward)."""
    B, H, W, _ = feat.shape
    dev = feat.device
    if grad_out is None:
        grad_out = torch.empty(NPARAM, dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = torch.empty(workspace_bytes(B, H, W, True), dtype=torch.uint8, device=dev)
    check(lib().sf_lrnet_backward(_ptr(params), _ptr(feat), _ptr(dz4), B, H, W, _ptr(grad_out),
                                  _ptr(workspace), workspace.numel(), _stream(stream)))
    return grad_out


def adam(params, m, v, g, lr, b1, b2, eps, step, stream=None):
    """One Adam step in place; b1^step, b2^step formed in FP32 by repeated products."""
    b1t = np.float32(1.0)
    b2t = np.float32(1.0)
    for _ in range(step):
        b1t = np.float32(b1t * np.float32(b1))
        b2t = np.float32(b2t * np.float32(b2))
    check(lib().sf_lrnet_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(g), params.numel(), lr, b1, b2,
                              eps, float(b1t), float(b2t), _stream(stream)))


class Trainer:
    """Adam on the GPU: FP32 master weights, optimizer moments, step count."""

    def __init__(self, params: np.ndarray, lr=2e-3, b1=0.9, b2=0.999, eps=1e-8, device="cuda:0"):
        self.params = torch.from_numpy(np.ascontiguousarray(params, np.float32)).to(device)
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=device)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=device)
        self.g = torch.empty(NPARAM, dtype=torch.float32, device=device)
        self.loss = torch.empty(1, dtype=torch.float32, device=device)
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.step_count = 0
        self.ws = None
        self.ws_shape = None

    def step(self, feat, label):
        B, H, W, _ = feat.shape
        if self.ws_shape != (B, H, W):
            self.ws = torch.empty(workspace_bytes(B, H, W, True), dtype=torch.uint8, device=feat.device)
            self.ws_shape = (B, H, W)
        grad(self.params, feat, label, self.g, self.loss, self.ws)
        self.step_count += 1
        adam(self.params, self.m, self.v, self.g, self.lr, self.b1, self.b2, self.eps, self.step_count)
        return self.loss

    def state(self) -> dict:
        """Checkpoint: master weights, moments and step count (numpy)."""
        return {"params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "step": self.step_count,
                "hyper": np.array([self.lr, self.b1, self.b2, self.eps], np.float64)}

    def load_state(self, st: dict) -> None:
        dev = self.params.device
        self.params = torch.from_numpy(np.ascontiguousarray(st["params"], np.float32)).to(dev)
        self.m = torch.from_numpy(np.ascontiguousarray(st["m"], np.float32)).to(dev)
        self.v = torch.from_numpy(np.ascontiguousarray(st["v"], np.float32)).to(dev)
        self.step_count = int(st["step"])
