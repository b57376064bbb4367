"""MI355X (gfx950) likelihood-guidance path of physics-guided diffusion FWI.

Forward modelling, W2 misfit with its adjoint source, adjoint-state gradient
and the preconditioned guidance update, all in hand-written HIP kernels
behind the C ABI of include/fwi.h (libfwi.so, built in-tree).
"""
from .fwi import DEFAULT_GUIDANCE, DEFAULT_W2, FwiPlan, FwiW2Loss, ddpm_step, guidance_step, tv_subgradient  # noqa: F401
