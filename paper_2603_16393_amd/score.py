"""The score network of the reverse-diffusion loop (Algorithm 2) through the C ABI.

``ScoreNet`` wraps the library's noise-prediction network (layers in
include/fwi.h): forward with a per-sample output map (noise, score or the
clean estimate of Eq. v0hat), its vector-Jacobian product (for the clean
estimate, the chain rule h = (d v0hat / d x_i)^T g of Eq. chain_rule), one
denoising score-matching Adam step, and the parameter / optimiser state for
checkpoints.  Argument marshalling only: every computation runs in the HIP
kernels.  ``vp_schedule`` gives the discrete variance-preserving schedule
(beta_i linear from 1e-4 to 0.02, abar_i = prod (1 - beta_j)) that the
reverse step of Algorithm 2 uses.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check

__all__ = ["ScoreNet", "vp_schedule", "output_map"]

NZ = NX = 70


def vp_schedule(N: int = 1000):
    """(beta [N], abar [N]) of the discrete VP schedule, index i = 1..N stored at i - 1."""
    beta = np.linspace(1e-4, 0.02, N)
    return beta, np.cumprod(1.0 - beta)


def output_map(kind: str, abar):
    """(skip, scale) arrays of the output map out = skip x + scale eps for abar [B]:
    'eps' the noise, 'score' s = -eps / sqrt(1 - abar), 'clean' v0hat = (x - sqrt(1 - abar) eps) / sqrt(abar)."""
    ab = np.asarray(abar, np.float64).reshape(-1)
    if kind == "eps":
        return np.zeros_like(ab), np.ones_like(ab)
    if kind == "score":
        return np.zeros_like(ab), -1.0 / np.sqrt(1.0 - ab)
    if kind == "clean":
        return 1.0 / np.sqrt(ab), -np.sqrt(1.0 - ab) / np.sqrt(ab)
    raise ValueError(kind)


def _p(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class ScoreNet:
    def __init__(self, max_batch: int, device=None):
        L = _lib.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.max_batch = int(max_batch)
        self.n_params = int(L.fwi_score_param_count())
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.fwi_score_create(self.max_batch, ctypes.byref(h)), "fwi_score_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fwi_score_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state --------------------------------------------------------------
    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(np.asarray(params, np.float32).reshape(-1))
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        check(_lib.load().fwi_score_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)), "fwi_score_set_params")

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, np.float32)
        check(_lib.load().fwi_score_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p)), "fwi_score_get_params")
        return p

    def get_grads(self) -> np.ndarray:
        g = np.empty(self.n_params, np.float32)
        check(_lib.load().fwi_score_get_grads(self._h, g.ctypes.data_as(ctypes.c_void_p)), "fwi_score_get_grads")
        return g

    def get_adam(self):
        m = np.empty(self.n_params, np.float32)
        v = np.empty(self.n_params, np.float32)
        step = ctypes.c_int()
        check(_lib.load().fwi_score_get_adam(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                             v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(step)),
              "fwi_score_get_adam")
        return m, v, step.value

    def set_adam(self, m: np.ndarray, v: np.ndarray, step: int):
        m = np.ascontiguousarray(np.asarray(m, np.float32))
        v = np.ascontiguousarray(np.asarray(v, np.float32))
        if m.size != self.n_params or v.size != self.n_params:
            raise ValueError("Adam moments of the wrong size")
        check(_lib.load().fwi_score_set_adam(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                             v.ctypes.data_as(ctypes.c_void_p), int(step)), "fwi_score_set_adam")

    # -- compute ------------------------------------------------------------
    def _check(self, t: torch.Tensor, name: str, shape):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device == self.device and t.dtype == torch.float32
                and tuple(t.shape) == tuple(shape) and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 tensor of shape {tuple(shape)} on {self.device}")

    def forward(self, x: torch.Tensor, tcond: torch.Tensor, skip: Optional[torch.Tensor] = None,
                scale: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        B = x.shape[0]
        self._check(x, "x", (B, NZ, NX))
        self._check(tcond, "tcond", (B,))
        for name, t in (("skip", skip), ("scale", scale)):
            if t is not None:
                self._check(t, name, (B,))
        if out is None:
            out = torch.empty_like(x)
        self._check(out, "out", (B, NZ, NX))
        check(_lib.load().fwi_score_forward(self._h, B, _p(x), _p(tcond), _p(skip), _p(scale), _p(out), _stream()),
              "fwi_score_forward")
        return out

    def backward(self, dout: torch.Tensor, dx: Optional[torch.Tensor] = None, want_input: bool = True,
                 weight_grads: bool = False) -> Optional[torch.Tensor]:
        B = dout.shape[0]
        self._check(dout, "dout", (B, NZ, NX))
        if want_input and dx is None:
            dx = torch.empty_like(dout)
        if dx is not None:
            self._check(dx, "dx", (B, NZ, NX))
        check(_lib.load().fwi_score_backward(self._h, B, _p(dout), _p(dx), int(bool(weight_grads)), _stream()),
              "fwi_score_backward")
        return dx

    def train_step(self, x0: torch.Tensor, noise: torch.Tensor, tcond: torch.Tensor, sqrt_abar: torch.Tensor,
                   sqrt_1m_abar: torch.Tensor, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                   loss_out: Optional[torch.Tensor] = None):
        B = x0.shape[0]
        self._check(x0, "x0", (B, NZ, NX))
        self._check(noise, "noise", (B, NZ, NX))
        for name, t in (("tcond", tcond), ("sqrt_abar", sqrt_abar), ("sqrt_1m_abar", sqrt_1m_abar)):
            self._check(t, name, (B,))
        if loss_out is not None:
            self._check(loss_out, "loss_out", (1,))
        p = _lib.ScoreTrainParams(float(lr), float(beta1), float(beta2), float(eps))
        check(_lib.load().fwi_score_train_step(self._h, B, _p(x0), _p(noise), _p(tcond), _p(sqrt_abar),
                                               _p(sqrt_1m_abar), ctypes.byref(p), _p(loss_out), _stream()),
              "fwi_score_train_step")
        return loss_out
