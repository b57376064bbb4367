"""Python face of the guidance path: a plan object, the misfit as a
torch.autograd.Function, and the preconditioned guidance update.

PyTorch supplies device memory and the current HIP stream; every step runs in
the library's HIP kernels through the C ABI (see _lib.py).  Inputs must be
contiguous float32 tensors on the plan's GPU.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check

__all__ = ["FwiPlan", "FwiW2Loss", "guidance_step", "DEFAULT_W2", "DEFAULT_GUIDANCE"]

# Paper settings: Sec. 6.2 (W2 numerics), Sec. 6.3 fixed values and Table
# 'parameter' (CurveVel-A column for gamma and rho0).
DEFAULT_W2 = dict(k=100.0, eps_prime=1e-9, n_xi=1000, c_factor=1.1, squared=False, reduction=0)
DEFAULT_GUIDANCE = dict(rho0=1.15, c=0.1, tau=0.0, gamma=0.55, eps=1e-4, kappa_max=0.0, unit_scale=1.0)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t: torch.Tensor, name: str, shape: tuple, dtype=torch.float32, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if device is not None and t.device != device:
        raise ValueError(f"{name} must be on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class FwiPlan:
    """Plan for one acquisition (grid, time axis, shots, receivers).

    ``acq`` is any object with the fields nz, nx, dz, dx, dt, nt, nb,
    free_surface, v_max, src_iz, src_ix, rec_iz, rec_ix (model-grid indices).
    """

    def __init__(self, acq, max_batch: int, mem_budget_bytes: int = 0, force_path: int = -1, ckpt_every: int = 0,
                 device: Optional[torch.device] = None, lds_tile: tuple = (0, 0), timing: bool = False,
                 split: int = 0):
        L = _lib.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.nz, self.nx, self.nt = int(acq.nz), int(acq.nx), int(acq.nt)
        self._idx = [np.ascontiguousarray(np.asarray(a, dtype=np.int32)) for a in
                     (acq.src_iz, acq.src_ix, acq.rec_iz, acq.rec_ix)]
        self.ns, self.nr = len(self._idx[0]), len(self._idx[2])
        ip = [a.ctypes.data_as(_lib.c_int_p) for a in self._idx]
        self._geom = _lib.Geometry(self.nz, self.nx, float(acq.dz), float(acq.dx), float(acq.dt), self.nt,
                                   int(acq.nb), int(bool(acq.free_surface)), float(acq.v_max), self.ns, ip[0], ip[1],
                                   self.nr, ip[2], ip[3], int(bool(getattr(acq, "pml", False))))
        self.max_batch = int(max_batch)
        opts = _lib.PlanOptions(int(force_path), int(ckpt_every), int(lds_tile[0]), int(lds_tile[1]), int(bool(timing)),
                                int(split))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.fwi_plan_create_ex(ctypes.byref(self._geom), self.max_batch, int(mem_budget_bytes),
                                       ctypes.byref(opts), ctypes.byref(h)), "fwi_plan_create")
        self._h = h
        info = _lib.PlanInfo()
        check(L.fwi_plan_get_info(self._h, ctypes.byref(info)), "fwi_plan_get_info")
        self.info = {f: getattr(info, f) for f, _ in _lib.PlanInfo._fields_}
        self.obs_shape = (self.ns, self.nr, self.nt)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fwi_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points -----------------------------------------------------
    def set_obs(self, d_obs: torch.Tensor, k=100.0, eps_prime=1e-9, n_xi=1000, c_factor=1.1, squared=False,
                reduction=0):
        _need(d_obs, "d_obs", self.obs_shape, device=self.device)
        p = _lib.W2Params(float(k), float(eps_prime), int(n_xi), float(c_factor), int(bool(squared)), int(reduction))
        check(_lib.load().fwi_set_obs(self._h, _ptr(d_obs), ctypes.byref(p), _stream()), "fwi_set_obs")

    def forward(self, v: torch.Tensor, wavelet: torch.Tensor, keep_for_adjoint: bool = True,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        B = v.shape[0]
        _need(v, "v", (B, self.nz, self.nx), device=self.device)
        _need(wavelet, "wavelet", (self.nt,), device=self.device)
        if out is None:
            out = torch.empty((B, self.ns, self.nr, self.nt), dtype=torch.float32, device=self.device)
        _need(out, "out", (B, self.ns, self.nr, self.nt), device=self.device)
        check(_lib.load().fwi_forward(self._h, B, _ptr(v), _ptr(wavelet), _ptr(out), int(bool(keep_for_adjoint)),
                                      _stream()), "fwi_forward")
        return out

    def w2_misfit(self, d_syn: torch.Tensor, want_adjoint: bool = True, J_out=None, adj_out=None):
        B = d_syn.shape[0]
        _need(d_syn, "d_syn", (B, self.ns, self.nr, self.nt), device=self.device)
        J = J_out if J_out is not None else torch.empty(B, dtype=torch.float64, device=self.device)
        _need(J, "J", (B,), dtype=torch.float64, device=self.device)
        adj = None
        if want_adjoint:
            adj = adj_out if adj_out is not None else torch.empty_like(d_syn)
            _need(adj, "adj", tuple(d_syn.shape), device=self.device)
        check(_lib.load().fwi_w2_misfit(self._h, B, _ptr(d_syn), _ptr(J), _ptr(adj), _stream()), "fwi_w2_misfit")
        return J, adj

    def l2_misfit(self, d_syn: torch.Tensor, d_obs: torch.Tensor, sigma: float = 0.05, k: float = 0.0,
                  normalize: bool = False, want_adjoint: bool = True, J_out=None, adj_out=None):
        """Least-squares potential (1/2) sum (w (d_syn - d_obs))^2 / S per sample and dJ/dd_syn
        (baseline DPS: k = 0, S = sigma^2; the ablation's enhanced form: k > 0, normalize)."""
        B = d_syn.shape[0]
        _need(d_syn, "d_syn", (B, self.ns, self.nr, self.nt), device=self.device)
        _need(d_obs, "d_obs", self.obs_shape, device=self.device)
        J = J_out if J_out is not None else torch.empty(B, dtype=torch.float64, device=self.device)
        _need(J, "J", (B,), dtype=torch.float64, device=self.device)
        adj = None
        if want_adjoint:
            adj = adj_out if adj_out is not None else torch.empty_like(d_syn)
            _need(adj, "adj", tuple(d_syn.shape), device=self.device)
        p = _lib.L2Params(float(sigma), float(k), int(bool(normalize)))
        check(_lib.load().fwi_l2_misfit(self._h, B, _ptr(d_syn), _ptr(d_obs), ctypes.byref(p), _ptr(J), _ptr(adj),
                                        _stream()), "fwi_l2_misfit")
        return J, adj

    def history(self) -> int:
        """Number of the forward call whose history the plan keeps (0 = none)."""
        h = ctypes.c_ulonglong()
        check(_lib.load().fwi_plan_history(self._h, ctypes.byref(h)), "fwi_plan_history")
        return h.value

    def adjoint_gradient(self, v: torch.Tensor, adj: torch.Tensor, scale: Optional[torch.Tensor] = None,
                         out: Optional[torch.Tensor] = None, history: Optional[int] = None) -> torch.Tensor:
        """dJ/dv for the kept forward history; with `history` (from history() after that forward call) the call
        fails with FWI_ESTATE if a later forward call has replaced it."""
        B = v.shape[0]
        _need(v, "v", (B, self.nz, self.nx), device=self.device)
        _need(adj, "adj", (B, self.ns, self.nr, self.nt), device=self.device)
        if scale is not None:
            _need(scale, "scale", (B,), device=self.device)
        if out is None:
            out = torch.empty((B, self.nz, self.nx), dtype=torch.float32, device=self.device)
        _need(out, "out", (B, self.nz, self.nx), device=self.device)
        if history is None:
            check(_lib.load().fwi_adjoint_gradient(self._h, B, _ptr(v), _ptr(adj), _ptr(scale), _ptr(out),
                                                   _stream()), "fwi_adjoint_gradient")
        else:
            check(_lib.load().fwi_adjoint_gradient_of(self._h, int(history), B, _ptr(v), _ptr(adj), _ptr(scale),
                                                      _ptr(out), _stream()), "fwi_adjoint_gradient_of")
        return out

    def sweep_ms(self):
        """(forward, adjoint) mean device ms of the sweeps since the previous call; needs timing=True."""
        f, a = ctypes.c_float(), ctypes.c_float()
        check(_lib.load().fwi_plan_sweep_ms(self._h, ctypes.byref(f), ctypes.byref(a)), "fwi_plan_sweep_ms")
        return f.value, a.value

    def status(self) -> int:
        """Synchronises and returns the device-side status code (0 = ok)."""
        return _lib.load().fwi_status(self._h)


class FwiW2Loss(torch.autograd.Function):
    """J(v) per sample (m/s in, W2 objective out); backward runs the adjoint sweep.

    Usage: ``J = FwiW2Loss.apply(v, plan, wavelet)`` with v [B, nz, nx].
    """

    @staticmethod
    def forward(ctx, v, plan: FwiPlan, wavelet):
        v = v.detach().contiguous()
        d = plan.forward(v, wavelet, keep_for_adjoint=True)
        J, adj = plan.w2_misfit(d, want_adjoint=True)
        ctx.plan = plan
        ctx.history = plan.history()
        ctx.save_for_backward(v, adj)
        return J

    @staticmethod
    def backward(ctx, gJ):
        v, adj = ctx.saved_tensors
        scale = gJ.detach().to(torch.float32).contiguous()
        # raises FwiError (FWI_ESTATE) if another forward call on the plan replaced this one's history
        g = ctx.plan.adjoint_gradient(v, adj, scale=scale, history=ctx.history)
        return g, None, None


def guidance_step(v_prop, h, g, v0hat, rho0=1.15, c=0.1, tau=0.0, gamma=0.55, eps=1e-4, kappa_max=0.0,
                  unit_scale=1.0, out=None, rho_out=None):
    """v_{i-1} = v'_{i-1} - rho kappa (s h) with rho from TV(v0hat) and kappa from s g (Sec. 5.2)."""
    B, nz, nx = v_prop.shape
    dev = v_prop.device
    for name, t in (("v_prop", v_prop), ("h", h), ("g", g), ("v0hat", v0hat)):
        _need(t, name, (B, nz, nx), device=dev)
    if out is None:
        out = torch.empty_like(v_prop)
    if rho_out is None:
        rho_out = torch.empty(B, dtype=torch.float32, device=dev)
    _need(out, "out", (B, nz, nx), device=dev)
    _need(rho_out, "rho_out", (B,), device=dev)
    p = _lib.GuidanceParams(float(rho0), float(c), float(tau), float(gamma), float(eps), float(kappa_max),
                            float(unit_scale))
    check(_lib.load().fwi_guidance_step(B, nz, nx, _ptr(v_prop), _ptr(h), _ptr(g), _ptr(v0hat), ctypes.byref(p),
                                        _ptr(out), _ptr(rho_out), _stream()), "fwi_guidance_step")
    return out, rho_out


def tv_subgradient(v: torch.Tensor, g: Optional[torch.Tensor] = None, alpha: float = 1.0,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g + alpha q with q a subgradient of TV(v) (Eq. tv, sign(0) = 0), per sample of [B, nz, nx]."""
    B, nz, nx = v.shape
    _need(v, "v", (B, nz, nx), device=v.device)
    if g is not None:
        _need(g, "g", (B, nz, nx), device=v.device)
    if out is None:
        out = torch.empty_like(v)
    _need(out, "out", (B, nz, nx), device=v.device)
    check(_lib.load().fwi_tv_subgradient(B, nz, nx, _ptr(v), _ptr(g), float(alpha), _ptr(out), _stream()),
          "fwi_tv_subgradient")
    return out


def ddpm_step(v: torch.Tensor, beta: float, abar: float, abar_prev: float, score: Optional[torch.Tensor] = None,
              v0hat: Optional[torch.Tensor] = None, z: Optional[torch.Tensor] = None, sigma: float = 0.0,
              out: Optional[torch.Tensor] = None):
    """Reverse DDPM step of Algorithm 2 before its guidance term: returns (v0hat, v_prop) with
    v0hat = (v + (1 - abar) score) / sqrt(abar) when `score` is given (else the given v0hat) and
    v_prop = sqrt(1 - beta)(1 - abar_prev)/(1 - abar) v + sqrt(abar_prev) beta/(1 - abar) v0hat + sigma z."""
    shape = tuple(v.shape)
    _need(v, "v", shape, device=v.device)
    if score is not None:
        _need(score, "score", shape, device=v.device)
        v0hat = torch.empty_like(v) if v0hat is None else v0hat
    elif v0hat is None:
        raise ValueError("ddpm_step needs a score or a clean estimate v0hat")
    _need(v0hat, "v0hat", shape, device=v.device)
    if z is not None:
        _need(z, "z", shape, device=v.device)
    if out is None:
        out = torch.empty_like(v)
    _need(out, "out", shape, device=v.device)
    check(_lib.load().fwi_ddpm_step(v.numel(), _ptr(v), _ptr(score), _ptr(z), float(beta), float(abar),
                                    float(abar_prev), float(sigma), _ptr(v0hat), _ptr(out), _stream()),
          "fwi_ddpm_step")
    return v0hat, out
