"""The reverse-diffusion loop of Algorithm 2 (OT-WE-PDPS) on the GPU.

One reverse step for a batch of B states x_i (normalised velocity, [-1, 1]):

    v0hat   = (x_i - sqrt(1 - abar_i) eps_theta(x_i, i/N)) / sqrt(abar_i)     Eq. v0hat (score network)
    v'      = sqrt(alpha) (1 - abar_prev)/(1 - abar_i) x_i
              + sqrt(abar_prev) beta / (1 - abar_i) v0hat + sigma z           DDPM posterior mean + noise
    g       = dJ/dv0hat  (forward modelling, W2 misfit, adjoint gradient)      the guidance gradient
    h       = (d v0hat / d x_i)^T g                                           Eq. chain_rule (network VJP)
    x_{i-1} = v' - rho(TV(v0hat)) kappa(g) h                                   Eqs. precond_step, rho, kappa

on a respaced schedule of n steps over the N = 1000 VP steps (beta and abar of
vp_schedule; a respaced step from i to i_prev uses beta = 1 - abar_i /
abar_prev and sigma^2 = beta (1 - abar_prev)/(1 - abar_i)).  The clean
estimate enters the solver in m/s, v = 1500 + 1500 (v0hat + 1), clipped to
1500-4500 m/s; the gradient passes the clip unchanged (straight through).
Each line runs in the library's kernels: fwi_score_forward / fwi_score_backward,
fwi_ddpm_step, fwi_forward / fwi_w2_misfit / fwi_adjoint_gradient,
fwi_guidance_step; this module only sequences them (the unit change and the
clip are torch element-wise operations on the 16 x 70 x 70 batch).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from .fwi import FwiPlan, ddpm_step, guidance_step
from .score import ScoreNet, output_map, vp_schedule

__all__ = ["respaced_steps", "ReverseLoop", "LoopStats"]

V_LO, V_HI = 1500.0, 4500.0


def respaced_steps(n: int, N: int = 1000) -> np.ndarray:
    """n step indices from N down to 1, evenly spaced."""
    return np.unique(np.round(np.linspace(1, N, n)).astype(int))[::-1]


@dataclass
class LoopStats:
    J: List[np.ndarray] = field(default_factory=list)      # per step, misfit of the clean estimate (guided)
    rho: List[np.ndarray] = field(default_factory=list)


class ReverseLoop:
    """Algorithm 2 for B samples; plan=None runs the unguided reverse process."""

    def __init__(self, net: ScoreNet, B: int, n_steps: int, plan: Optional[FwiPlan] = None,
                 wavelet: Optional[torch.Tensor] = None, guidance: Optional[dict] = None, N: int = 1000):
        self.net, self.plan, self.w, self.B = net, plan, wavelet, B
        self.dev = net.device
        self.steps = respaced_steps(n_steps, N)
        _, self.abar = vp_schedule(N)
        self.N = N
        self.gp = dict(rho0=1.15, c=0.1, tau=0.0, gamma=0.55, eps=1e-4, kappa_max=0.0)
        if guidance:
            self.gp.update(guidance)
        shp = (B, 70, 70)
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.v0 = torch.empty(shp, **f32)
        self.vprop = torch.empty(shp, **f32)
        self.vphys = torch.empty(shp, **f32)
        self.h = torch.empty(shp, **f32)
        self.xn = torch.empty(shp, **f32)
        self.rho = torch.empty(B, **f32)
        if plan is not None:
            self.d = torch.empty((B, plan.ns, plan.nr, plan.nt), **f32)
            self.adj = torch.empty_like(self.d)
            self.J = torch.empty(B, dtype=torch.float64, device=self.dev)
            self.g = torch.empty(shp, **f32)
        # per-step scalars on the device (output map of the clean estimate, conditioning time)
        self._coef = []
        for k, i in enumerate(self.steps):
            ab = float(self.abar[i - 1])
            ab_prev = float(self.abar[self.steps[k + 1] - 1]) if k + 1 < len(self.steps) else 1.0
            skip, scale = output_map("clean", np.full(B, ab))
            beta = 1.0 - ab / ab_prev
            sigma = float(np.sqrt(beta * (1.0 - ab_prev) / (1.0 - ab))) if k + 1 < len(self.steps) else 0.0
            self._coef.append(dict(i=int(i), ab=ab, ab_prev=ab_prev, beta=beta, sigma=sigma,
                                   t=torch.full((B,), i / N, **f32),
                                   skip=torch.tensor(skip, **f32), scale=torch.tensor(scale, **f32)))

    def step(self, x: torch.Tensor, k: int, z: Optional[torch.Tensor], stats: Optional[LoopStats] = None):
        """One reverse step k of the schedule; returns x_{i-1} (a buffer owned by the loop)."""
        c = self._coef[k]
        self.net.forward(x, c["t"], c["skip"], c["scale"], out=self.v0)                      # Eq. v0hat
        ddpm_step(x, c["beta"], c["ab"], c["ab_prev"], v0hat=self.v0, z=z if c["sigma"] > 0 else None,
                  sigma=c["sigma"], out=self.vprop)
        if self.plan is None:
            self.xn.copy_(self.vprop)
            return self.xn
        torch.add(self.v0, 1.0, out=self.vphys).mul_(0.5 * (V_HI - V_LO)).add_(V_LO).clamp_(V_LO, V_HI)
        self.plan.forward(self.vphys, self.w, keep_for_adjoint=True, out=self.d)
        self.plan.w2_misfit(self.d, want_adjoint=True, J_out=self.J, adj_out=self.adj)
        self.plan.adjoint_gradient(self.vphys, self.adj, out=self.g)
        self.net.backward(self.g, dx=self.h)                                                 # Eq. chain_rule
        guidance_step(self.vprop, self.h, self.g, self.v0, unit_scale=0.5 * (V_HI - V_LO), out=self.xn,
                      rho_out=self.rho, **self.gp)
        if stats is not None:
            stats.J.append(self.J.cpu().numpy())
            stats.rho.append(self.rho.cpu().numpy())
        return self.xn

    def step_noise(self, seed: int) -> torch.Tensor:
        """Seeded standard normal noise for every step, [n_steps, B, 70, 70] on the device."""
        rng = np.random.default_rng(seed)
        z = rng.standard_normal((len(self.steps), self.B, 70, 70)).astype(np.float32)
        return torch.from_numpy(z).to(self.dev)

    def run(self, x_init: torch.Tensor, noise_seed: int = 0, stats: Optional[LoopStats] = None,
            noise: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Runs every step from x_init (B x 70 x 70 standard normal for sampling); the step noise is `noise`
        (from step_noise) or drawn from noise_seed."""
        zs = self.step_noise(noise_seed) if noise is None else noise
        x = x_init.clone()
        for k in range(len(self.steps)):
            x.copy_(self.step(x, k, zs[k], stats))
        return x
