"""Guidance gradients for a batch of reverse-diffusion samples, from the
exact solver or from the learned surrogate under the solver's judgement.

The exact gradient of one step is rows forward -> W2 misfit -> adjoint of
the guidance path (Sec. 5.1, Sec. 5.2).  Following the outlook of Sec. 7
(multi-fidelity surrogate strategies), above a noise level ``t_switch`` the
gradient may instead be predicted as

    g(v) ~ g_exact(v_a) + (g_S(v) - g_S(v_a)),   J(v) ~ J_exact(v_a) + (J_S(v) - J_S(v_a)),

where v_a is the last anchor (a step where the solver ran) and g_S, J_S are
the gradient and misfit computed through the surrogate's traces and its VJP.
After ``k`` predicted steps the solver runs again and judges the prediction
it would have replaced: if the gradient cosine of any sample falls below
``cos_min`` or its relative misfit error exceeds ``jerr_max``, k is halved
(down to 0: the solver on every step, still judging); if all samples pass,
k doubles (from 0 to 1) up to ``k_max``.  The judged step itself always returns the exact values and
becomes the new anchor.

``predictor="anchor"`` is the same schedule without the network (the
anchor's exact values are reused unchanged between judged steps); it is the
baseline that shows what the trained surrogate adds.

The decision is made for the whole batch: on MI355X one solver launch holds
one workgroup per (sample, shot), so any batch of up to about 50 samples
costs the same as one sample and a per-sample fallback would save nothing.
All arithmetic runs in the library's kernels; this class only schedules.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import torch

from .fwi import FwiPlan
from .surrogate import Surrogate, judge, mf_predict

__all__ = ["GuidanceGradients", "GuidanceStats"]


@dataclass
class GuidanceStats:
    exact_batches: int = 0       # solver gradient evaluations (batches)
    surrogate_batches: int = 0   # surrogate gradient evaluations (batches)
    served_exact: int = 0        # steps whose returned gradient is the solver's
    served_predicted: int = 0    # steps whose returned gradient is a prediction
    judged: int = 0
    passed: int = 0
    judge_cos: List[float] = field(default_factory=list)   # per sample, at judged steps
    judge_jerr: List[float] = field(default_factory=list)
    k_trace: List[int] = field(default_factory=list)


class GuidanceGradients:
    """Per-step gradient source for a batch of B samples.

    ``plan`` must hold the observations (set_obs) and have max_batch >= B.
    ``surrogate`` may be None (plain solver guidance).
    """

    def __init__(self, plan: FwiPlan, wavelet: torch.Tensor, B: int, surrogate: Optional[Surrogate] = None,
                 t_switch: float = 0.5, cos_min: float = 0.95, jerr_max: float = 0.05, k0: int = 4,
                 k_max: int = 32, predictor: str = "surrogate", adapt: bool = True):
        if predictor not in ("surrogate", "anchor"):
            raise ValueError("predictor must be 'surrogate' or 'anchor'")
        if predictor == "surrogate" and surrogate is None:
            predictor = "none"
        self.plan, self.w, self.B, self.sur = plan, wavelet, B, surrogate
        self.predictor, self.adapt = predictor, adapt
        self.t_switch, self.cos_min, self.jerr_max = t_switch, cos_min, jerr_max
        self.k, self.k_max = max(0, k0), max(1, k_max)
        dev = plan.device
        shp = (B, plan.nz, plan.nx)
        tr = (B, plan.ns, plan.nr, plan.nt)
        f32 = dict(dtype=torch.float32, device=dev)
        f64 = dict(dtype=torch.float64, device=dev)
        self.d = torch.empty(tr, **f32)
        self.adj = torch.empty(tr, **f32)
        self.g = torch.empty(shp, **f32)
        self.J = torch.empty(B, **f64)
        self.gs = torch.empty(shp, **f32)
        self.Js = torch.empty(B, **f64)
        self.ga = torch.empty(shp, **f32)
        self.gsa = torch.empty(shp, **f32)
        self.Ja = torch.empty(B, **f64)
        self.Jsa = torch.empty(B, **f64)
        self.gp = torch.empty(shp, **f32)
        self.Jp = torch.empty(B, **f64)
        self.cos = torch.empty(B, **f32)
        self.jerr = torch.empty(B, **f32)
        self.have_anchor = False
        self.since = 0
        self.stats = GuidanceStats()

    # building blocks ----------------------------------------------------
    def _exact(self, v):
        self.plan.forward(v, self.w, keep_for_adjoint=True, out=self.d)
        self.plan.w2_misfit(self.d, want_adjoint=True, J_out=self.J, adj_out=self.adj)
        self.plan.adjoint_gradient(v, self.adj, out=self.g)
        self.stats.exact_batches += 1

    def _surrogate(self, v):
        self.sur.forward(v, out=self.d)
        self.plan.w2_misfit(self.d, want_adjoint=True, J_out=self.Js, adj_out=self.adj)
        self.sur.backward(self.adj, out=self.gs)
        self.stats.surrogate_batches += 1

    def _anchor(self):
        self.ga.copy_(self.g)
        self.Ja.copy_(self.J)
        if self.predictor == "surrogate":
            self.gsa.copy_(self.gs)
            self.Jsa.copy_(self.Js)
        self.have_anchor = True
        self.since = 0

    # one step -----------------------------------------------------------
    def __call__(self, t: float, v: torch.Tensor):
        """(J [B] float64, g [B, nz, nx] float32) for the models v at noise level t.
        The returned tensors are owned by this object and overwritten by the next call."""
        if self.predictor == "none" or t <= self.t_switch:
            self._exact(v)
            self.stats.served_exact += 1
            self.have_anchor = False
            return self.J, self.g
        use_net = self.predictor == "surrogate"
        if self.have_anchor and self.since < self.k:
            self.since += 1
            self.stats.served_predicted += 1
            if not use_net:
                return self.Ja, self.ga
            self._surrogate(v)
            mf_predict(self.ga, self.gs, self.gsa, self.gp, self.Ja, self.Js, self.Jsa, self.Jp)
            return self.Jp, self.gp
        # judge step: exact values, the prediction they replace, new anchor
        self._exact(v)
        if use_net:
            self._surrogate(v)
        if self.have_anchor:
            if use_net:
                mf_predict(self.ga, self.gs, self.gsa, self.gp, self.Ja, self.Js, self.Jsa, self.Jp)
                judge(self.gp, self.g, self.Jp, self.J, cos_out=self.cos, jerr_out=self.jerr)
            else:
                judge(self.ga, self.g, self.Ja, self.J, cos_out=self.cos, jerr_out=self.jerr)
            cos = self.cos.tolist()
            jerr = self.jerr.tolist()
            ok = all(c >= self.cos_min for c in cos) and all(e <= self.jerr_max for e in jerr)
            self.stats.judged += 1
            self.stats.passed += int(ok)
            self.stats.judge_cos += cos
            self.stats.judge_jerr += jerr
            if self.adapt:
                self.k = min(max(1, 2 * self.k), self.k_max) if ok else self.k // 2
        self.stats.k_trace.append(self.k)
        self._anchor()
        self.stats.served_exact += 1
        return self.J, self.g
