"""Python face of the learned trace surrogate and the judge.

The network, its backward pass and its Adam training step run in the
library's HIP kernels (fwi_sur_* of include/fwi.h); this module only moves
parameters between host and device and passes tensors through.  Shapes are
fixed: v [B, 70, 70] m/s -> traces [B, 5, 70, 1000] (the layout of
FwiPlan.forward), B <= max_batch.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check
from .fwi import _need, _ptr, _stream

__all__ = ["Surrogate", "PARAM_SPEC", "pack", "unpack", "init_params", "judge", "mf_predict"]

NZ = NX = 70
NS, NR, NT = 5, 70, 1000
Z = X = 72
C, CH, T, S = 64, 128, 256, 8
NBLK = 4


def _spec():
    spec = [("lift_w", (3, C)), ("lift_b", (C,))]
    for i in range(NBLK):
        q = f"enc{i}_"
        spec += [(q + "dw_k", (C, 3, 3)), (q + "dw_b", (C,)), (q + "w1", (C, CH)), (q + "b1", (CH,)),
                 (q + "w2", (CH, C)), (q + "b2", (C,))]
    spec.append(("d2t", (T, Z)))
    for i in range(NBLK):
        q = f"dec{i}_"
        spec += [(q + "xm", (X, X)), (q + "dw_k", (C, 3, 3)), (q + "dw_b", (C,)), (q + "w1", (C, CH)),
                 (q + "b1", (CH,)), (q + "w2", (CH, C)), (q + "b2", (C,))]
    spec += [("proj_w", (C, S)), ("proj_b", (S,)), ("up", (NT, T)), ("out_scale", ())]
    return spec


#: (name, shape) of every parameter, in the order of the FP32 parameter vector.
PARAM_SPEC = _spec()


def pack(params: dict) -> np.ndarray:
    """Parameter dict (names of PARAM_SPEC) -> contiguous FP32 vector."""
    parts = [np.asarray(params[n], np.float64).reshape(-1) for n, _ in PARAM_SPEC]
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def unpack(vec: np.ndarray) -> dict:
    out, o = {}, 0
    for n, shp in PARAM_SPEC:
        k = int(np.prod(shp)) if shp else 1
        a = np.asarray(vec[o:o + k], np.float64)
        out[n] = a.reshape(shp) if shp else float(a[0])
        o += k
    return out


def init_params(seed: int = 0, out_scale: float = 1.0) -> dict:
    """Training initialisation: fan-in scaled weights, near-identity depthwise
    kernels, small residual branches, and a time up-sampling that starts as
    linear interpolation from the 256-row grid to the 1000 trace samples."""
    rng = np.random.default_rng(seed)
    p = {"lift_w": rng.standard_normal((3, C)) * 0.5, "lift_b": rng.standard_normal(C) * 0.1}
    for name in ("enc", "dec"):
        for i in range(NBLK):
            q = f"{name}{i}_"
            k = rng.standard_normal((C, 3, 3)) * 0.1
            k[:, 1, 1] += 1.0
            p[q + "dw_k"] = k
            p[q + "dw_b"] = np.zeros(C)
            p[q + "w1"] = rng.standard_normal((C, CH)) * np.sqrt(2.0 / C)
            p[q + "b1"] = np.zeros(CH)
            p[q + "w2"] = rng.standard_normal((CH, C)) * np.sqrt(1.0 / CH) * 0.2
            p[q + "b2"] = np.zeros(C)
            if name == "dec":
                p[q + "xm"] = rng.standard_normal((X, X)) * np.sqrt(1.0 / X) * 0.2
    p["d2t"] = rng.standard_normal((T, Z)) * np.sqrt(1.0 / Z)
    p["proj_w"] = rng.standard_normal((C, S)) * np.sqrt(1.0 / C)
    p["proj_b"] = np.zeros(S)
    up = np.zeros((NT, T))
    pos = np.arange(NT) * (T - 1) / (NT - 1)
    lo = np.minimum(np.floor(pos).astype(int), T - 2)
    fr = pos - lo
    up[np.arange(NT), lo] = 1.0 - fr
    up[np.arange(NT), lo + 1] = fr
    p["up"] = up
    p["out_scale"] = float(out_scale)
    return p


class Surrogate:
    """Device-resident surrogate network (parameters, Adam state, activations)."""

    def __init__(self, max_batch: int, device: Optional[torch.device] = None):
        L = _lib.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.fwi_sur_create(self.max_batch, ctypes.byref(h)), "fwi_sur_create")
        self._h = h
        self.n_params = int(L.fwi_sur_param_count())
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fwi_sur_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fused_mlp(self, fused: bool) -> None:
        """One kernel per pointwise MLP (default) or two GEMMs; identical results."""
        check(_lib.load().fwi_sur_set_fused_mlp(self._h, int(bool(fused))), "fwi_sur_set_fused_mlp")

    # parameters ---------------------------------------------------------
    def set_params(self, params) -> None:
        vec = pack(params) if isinstance(params, dict) else np.ascontiguousarray(params, np.float32)
        if vec.shape != (self.n_params,):
            raise ValueError(f"expected {self.n_params} parameters, got {vec.shape}")
        check(_lib.load().fwi_sur_set_params(self._h, vec.ctypes.data_as(ctypes.c_void_p)), "fwi_sur_set_params")

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        check(_lib.load().fwi_sur_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)), "fwi_sur_get_params")
        return out

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        check(_lib.load().fwi_sur_get_grads(self._h, out.ctypes.data_as(ctypes.c_void_p)), "fwi_sur_get_grads")
        return out

    def get_adam(self):
        """(m, v, step) of the Adam optimiser."""
        m = np.empty(self.n_params, np.float32)
        v = np.empty(self.n_params, np.float32)
        step = ctypes.c_int()
        check(_lib.load().fwi_sur_get_adam(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                           v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(step)), "fwi_sur_get_adam")
        return m, v, step.value

    def set_adam(self, m: np.ndarray, v: np.ndarray, step: int) -> None:
        m = np.ascontiguousarray(m, np.float32)
        v = np.ascontiguousarray(v, np.float32)
        if m.shape != (self.n_params,) or v.shape != (self.n_params,):
            raise ValueError("Adam moments of the wrong size")
        check(_lib.load().fwi_sur_set_adam(self._h, m.ctypes.data_as(ctypes.c_void_p),
                                           v.ctypes.data_as(ctypes.c_void_p), int(step)), "fwi_sur_set_adam")

    # compute ------------------------------------------------------------
    def forward(self, v: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        B = v.shape[0]
        _need(v, "v", (B, NZ, NX), device=self.device)
        if out is None:
            out = torch.empty((B, NS, NR, NT), dtype=torch.float32, device=self.device)
        _need(out, "traces", (B, NS, NR, NT), device=self.device)
        check(_lib.load().fwi_sur_forward(self._h, B, _ptr(v), _ptr(out), _stream()), "fwi_sur_forward")
        return out

    def backward(self, dtraces: torch.Tensor, want_input_grad: bool = True, want_weight_grads: bool = False,
                 out: Optional[torch.Tensor] = None) -> Optional[torch.Tensor]:
        B = dtraces.shape[0]
        _need(dtraces, "dtraces", (B, NS, NR, NT), device=self.device)
        dv = None
        if want_input_grad:
            dv = out if out is not None else torch.empty((B, NZ, NX), dtype=torch.float32, device=self.device)
            _need(dv, "dv", (B, NZ, NX), device=self.device)
        check(_lib.load().fwi_sur_backward(self._h, B, _ptr(dtraces), _ptr(dv), int(want_weight_grads), _stream()),
              "fwi_sur_backward")
        return dv

    def train_step(self, v: torch.Tensor, target: torch.Tensor, lr: float = 1e-3, beta1: float = 0.9,
                   beta2: float = 0.999, eps: float = 1e-8, loss_k: float = 0.0, pair_weight: float = 0.0,
                   loss_out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """One Adam step on the weighted trace MSE; returns the loss (device scalar, before the step).

        With pair_weight > 0 the batch is (v, v + delta) stacked (even B) and the
        loss also matches the surrogate's finite differences to the target's."""
        B = v.shape[0]
        _need(v, "v", (B, NZ, NX), device=self.device)
        _need(target, "target", (B, NS, NR, NT), device=self.device)
        lo = loss_out if loss_out is not None else self._loss
        tp = _lib.SurTrainParams(lr, beta1, beta2, eps, loss_k, pair_weight)
        check(_lib.load().fwi_sur_train_step(self._h, B, _ptr(v), _ptr(target), ctypes.byref(tp), _ptr(lo), _stream()),
              "fwi_sur_train_step")
        return lo


def judge(g_a: torch.Tensor, g_b: torch.Tensor, J_a: Optional[torch.Tensor] = None,
          J_b: Optional[torch.Tensor] = None, cos_out=None, jerr_out=None):
    """Per-sample cosine between two gradient batches and, with J_a, J_b
    (float64 [B]), the relative misfit error |J_a - J_b| / |J_b|."""
    B = g_a.shape[0]
    n = int(np.prod(g_a.shape[1:]))
    _need(g_a, "g_a", tuple(g_a.shape), device=g_a.device)
    _need(g_b, "g_b", tuple(g_a.shape), device=g_a.device)
    cos = cos_out if cos_out is not None else torch.empty(B, dtype=torch.float32, device=g_a.device)
    jerr = None
    if J_a is not None:
        _need(J_a, "J_a", (B,), dtype=torch.float64, device=g_a.device)
        _need(J_b, "J_b", (B,), dtype=torch.float64, device=g_a.device)
        jerr = jerr_out if jerr_out is not None else torch.empty(B, dtype=torch.float32, device=g_a.device)
    check(_lib.load().fwi_judge(B, n, _ptr(g_a), _ptr(g_b), _ptr(J_a), _ptr(J_b), _ptr(cos), _ptr(jerr), _stream()),
          "fwi_judge")
    return cos, jerr


def mf_predict(g_anchor: torch.Tensor, s_now: torch.Tensor, s_anchor: torch.Tensor, out: torch.Tensor,
               J_anchor: Optional[torch.Tensor] = None, Js_now: Optional[torch.Tensor] = None,
               Js_anchor: Optional[torch.Tensor] = None, J_out: Optional[torch.Tensor] = None):
    """out = g_anchor + (s_now - s_anchor); J_out = J_anchor + (Js_now - Js_anchor) if given."""
    B = g_anchor.shape[0]
    n = int(np.prod(g_anchor.shape[1:]))
    for t, nm in ((g_anchor, "g_anchor"), (s_now, "s_now"), (s_anchor, "s_anchor"), (out, "out")):
        _need(t, nm, tuple(g_anchor.shape), device=g_anchor.device)
    if J_out is not None:
        for t, nm in ((J_anchor, "J_anchor"), (Js_now, "Js_now"), (Js_anchor, "Js_anchor"), (J_out, "J_out")):
            _need(t, nm, (B,), dtype=torch.float64, device=g_anchor.device)
    check(_lib.load().fwi_mf_predict(B, n, _ptr(g_anchor), _ptr(s_now), _ptr(s_anchor), _ptr(out), _ptr(J_anchor),
                                     _ptr(Js_now), _ptr(Js_anchor), _ptr(J_out), _stream()), "fwi_mf_predict")
    return out, J_out
