"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generation only: velocity models, acquisition
geometry, the source wavelet and the stand-in denoised estimates.  It contains
none of the method's arithmetic (no wave propagation, no misfit, no gradient,
no guidance), so both the FP64 oracle and the HIP path may consume it.

The paper evaluates on OpenFWI (CurveVel, FlatFault, CurveFault) and
Marmousi2 with a trained score network (Sec. 6); none of those are available
here, so seeded layered / faulted models with the same grid (70 x 70,
dx = dz = 10 m), velocity range (1500-4500 m/s) and acquisition (surface
shots, one receiver per surface column; Sec. 6.3.1) stand in for them.
All randomness is numpy PCG64 with explicit seeds; models are produced in
float64 and callers cast as needed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Acquisition",
    "ricker",
    "even_shot_columns",
    "surface_acquisition",
    "layered_model",
    "blob_perturbation",
    "faulted_model",
    "large_lens_model",
    "smooth_noise",
    "to_normalised",
    "prior_model",
    "from_normalised",
    "V_LO",
    "V_HI",
]

# Velocity range of the stand-in models (m/s); the diffusion state maps
# [-1, 1] onto it.
V_LO = 1500.0
V_HI = 4500.0


@dataclasses.dataclass
class Acquisition:
    """Grid, time axis and surface acquisition of one experiment.

    Indices are model-grid indices: row 0 is the surface (the reflecting top
    boundary), x is the fast axis.  Every shot sees the same receiver spread.
    """

    nz: int
    nx: int
    dz: float
    dx: float
    dt: float
    nt: int
    nb: int
    free_surface: bool
    v_max: float
    src_iz: np.ndarray
    src_ix: np.ndarray
    rec_iz: np.ndarray
    rec_ix: np.ndarray
    f_peak: float = 15.0
    pml: bool = False  # the nb-cell absorbing layer is a PML instead of the damping sponge

    @property
    def ns(self) -> int:
        return int(len(self.src_iz))

    @property
    def nr(self) -> int:
        return int(len(self.rec_iz))

    @property
    def padded_shape(self) -> tuple[int, int]:
        nzp = self.nz + self.nb + (0 if self.free_surface else self.nb)
        return nzp, self.nx + 2 * self.nb

    def subset_shots(self, shots) -> "Acquisition":
        shots = np.asarray(shots, dtype=np.int64)
        return dataclasses.replace(self, src_iz=self.src_iz[shots].copy(), src_ix=self.src_ix[shots].copy())


def ricker(nt: int, dt: float, f_peak: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet sampled at t_n = n dt (Sec. 6.1), t0 = 1.1 / f_peak by default."""
    if t0 is None:
        t0 = 1.1 / f_peak
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f_peak * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def even_shot_columns(nx: int, ns: int) -> np.ndarray:
    """Shot columns k * floor(nx / ns), the placement rule of Sec. 6.3.1
    (ten shots at 0, 7, ..., 63 on a 70-wide grid)."""
    step = nx // ns
    return np.arange(ns, dtype=np.int32) * step


def surface_acquisition(
    nz: int = 70,
    nx: int = 70,
    ns: int = 5,
    *,
    shot_cols=None,
    dx: float = 10.0,
    dz: float | None = None,
    dt: float = 1e-3,
    nt: int = 1000,
    nb: int = 40,
    free_surface: bool = True,
    v_max: float = V_HI,
    f_peak: float = 15.0,
    src_row: int = 0,
    rec_row: int = 0,
    rec_cols=None,
) -> Acquisition:
    """Surface shots and one receiver per surface column (Sec. 6.3.1)."""
    if shot_cols is None:
        shot_cols = even_shot_columns(nx, ns)
    shot_cols = np.asarray(shot_cols, dtype=np.int32)
    if rec_cols is None:
        rec_cols = np.arange(nx, dtype=np.int32)
    rec_cols = np.asarray(rec_cols, dtype=np.int32)
    return Acquisition(
        nz=nz,
        nx=nx,
        dz=float(dx if dz is None else dz),
        dx=float(dx),
        dt=float(dt),
        nt=int(nt),
        nb=int(nb),
        free_surface=bool(free_surface),
        v_max=float(v_max),
        src_iz=np.full(len(shot_cols), src_row, dtype=np.int32),
        src_ix=shot_cols.copy(),
        rec_iz=np.full(len(rec_cols), rec_row, dtype=np.int32),
        rec_ix=rec_cols.copy(),
        f_peak=float(f_peak),
    )


def layered_model(nz: int, nx: int, seed: int, n_layers: int = 3, v_lo: float = V_LO, v_hi: float = V_HI,
                  depth_range=(10, 59)) -> np.ndarray:
    """Flat layers, interface rows drawn from U{depth_range}, velocities drawn
    from U(v_lo, v_hi) and sorted to increase with depth."""
    rng = np.random.default_rng(seed)
    lo, hi = depth_range
    hi = min(hi, nz - 1)
    depths = np.sort(rng.choice(np.arange(lo, hi + 1), size=n_layers - 1, replace=False))
    vel = np.sort(rng.uniform(v_lo, v_hi, size=n_layers))
    v = np.empty((nz, nx), dtype=np.float64)
    z = np.arange(nz)[:, None]
    layer = np.searchsorted(depths, z, side="right")
    v[:] = vel[layer]
    return v


def blob_perturbation(v: np.ndarray, seed: int, amp: float = 0.1, radius: float = 6.0,
                      centre_range=(20, 50)) -> np.ndarray:
    """v * (1 + amp * sign * exp(-r^2 / (2 radius^2))) with a seeded sign and centre."""
    rng = np.random.default_rng(seed)
    sign = 1.0 if rng.integers(0, 2) == 1 else -1.0
    cz, cx = rng.uniform(centre_range[0], centre_range[1], size=2)
    nz, nx = v.shape
    z = np.arange(nz)[:, None]
    x = np.arange(nx)[None, :]
    r2 = (z - cz) ** 2 + (x - cx) ** 2
    return v * (1.0 + amp * sign * np.exp(-r2 / (2.0 * radius * radius)))


def faulted_model(nz: int, nx: int, seed: int, v_lo: float = V_LO, v_hi: float = V_HI) -> np.ndarray:
    """Dipping layers (2-4 interfaces, dips in +-10 deg) cut by one normal fault
    (surface trace in U[15, 55] scaled to nx, dip 60-80 deg, throw 3-10 cells);
    velocities sorted to increase with depth."""
    rng = np.random.default_rng(seed)
    n_if = int(rng.integers(2, 5))
    z0 = np.sort(rng.uniform(0.12 * nz, 0.88 * nz, size=n_if))
    theta = np.deg2rad(rng.uniform(-10.0, 10.0, size=n_if))
    vel = np.sort(rng.uniform(v_lo, v_hi, size=n_if + 1))
    xf = rng.uniform(15.0 / 70.0 * nx, 55.0 / 70.0 * nx)
    dip = np.deg2rad(rng.uniform(60.0, 80.0))
    throw = int(rng.integers(3, 11))
    z = np.arange(nz, dtype=np.float64)[:, None] * np.ones((1, nx))
    x = np.ones((nz, 1)) * np.arange(nx, dtype=np.float64)[None, :]
    hanging = x > xf + z / math.tan(dip)
    zs = np.where(hanging, z - throw, z)
    layer = np.zeros((nz, nx), dtype=np.int64)
    for i in range(n_if):
        layer += (zs >= z0[i] + math.tan(theta[i]) * (x - nx / 2.0)).astype(np.int64)
    return vel[layer]


def large_lens_model(nz: int = 400, nx: int = 800, seed: int = 0, v_top: float = 1500.0,
                     v_bottom: float = 4000.0, lens_dv: float = 1000.0, v_cap: float = 5000.0) -> np.ndarray:
    """Smooth depth gradient plus three flat layer steps and an elliptical
    high-velocity lens, capped at v_cap."""
    rng = np.random.default_rng(seed)
    z = np.arange(nz, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    v = v_top + (v_bottom - v_top) * z / max(nz - 1, 1) * np.ones((1, nx))
    steps = np.sort(rng.uniform(0.15 * nz, 0.85 * nz, size=3))
    jumps = rng.uniform(100.0, 300.0, size=3)
    for s, j in zip(steps, jumps):
        v = v + j * (z >= s)
    cz = rng.uniform(0.35 * nz, 0.65 * nz)
    cx = rng.uniform(0.3 * nx, 0.7 * nx)
    az = rng.uniform(0.06 * nz, 0.12 * nz)
    ax = rng.uniform(0.1 * nx, 0.2 * nx)
    inside = ((z - cz) / az) ** 2 + ((x - cx) / ax) ** 2 <= 1.0
    v = np.where(inside, v + lens_dv, v)
    return np.minimum(v, v_cap)


def smooth_noise(nz: int, nx: int, seed: int, sigma_cells: float = 3.0, std: float = 600.0) -> np.ndarray:
    """White noise smoothed by a separable Gaussian of sigma_cells and scaled to std."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, nx))
    r = int(math.ceil(3 * sigma_cells))
    k = np.exp(-0.5 * (np.arange(-r, r + 1) / sigma_cells) ** 2)
    k /= k.sum()
    from scipy.ndimage import convolve1d

    # zero-padded 'same' convolution along each axis (the kernel is symmetric)
    w = convolve1d(w, k, axis=0, mode="constant", cval=0.0)
    w = convolve1d(w, k, axis=1, mode="constant", cval=0.0)
    return w * (std / w.std())


def to_normalised(v: np.ndarray) -> np.ndarray:
    """Physical velocity (m/s) -> diffusion state in [-1, 1]."""
    return (v - V_LO) / (0.5 * (V_HI - V_LO)) - 1.0


def from_normalised(x: np.ndarray) -> np.ndarray:
    """Diffusion state in [-1, 1] -> physical velocity (m/s)."""
    return V_LO + (x + 1.0) * 0.5 * (V_HI - V_LO)


def stand_in_estimate(v_true: np.ndarray, t: float, zeta: np.ndarray) -> np.ndarray:
    """Stand-in for a denoiser's clean estimate at noise level t (no score network
    is part of this build): clip(v_true + t zeta, V_LO, V_HI)."""
    return np.clip(v_true + t * zeta, V_LO, V_HI)


def stand_in_zeta(nz: int, nx: int, sample: int) -> np.ndarray:
    """Per-sample smooth perturbation of the stand-in estimates: white noise
    smoothed by a 3-cell Gaussian, std 600 m/s (seed 7000 + sample)."""
    return smooth_noise(nz, nx, 7000 + sample, sigma_cells=3.0, std=600.0)


def prior_model(seed: int, nz: int = 70, nx: int = 70) -> np.ndarray:
    """One draw from the stand-in prior the score network learns: a faulted
    model of dipping layers (even seeds) or flat layers with 2-5 layers and
    interfaces in rows 5..64 (odd seeds), 1500-4500 m/s increasing with depth."""
    if seed % 2 == 0:
        return faulted_model(nz, nx, seed)
    return layered_model(nz, nx, seed, n_layers=2 + (seed // 2) % 4, depth_range=(5, min(64, nz - 1)))


def surrogate_training_pair(seed: int, nz: int = 70, nx: int = 70):
    """One training input for the trace surrogate and a perturbation of it.

    v: a dipping-layer faulted model (seed 10^6 + seed) plus t zeta with
    t ~ U(0, 1) and zeta smooth noise (3-cell Gaussian, std 600 m/s), the
    distribution of the stand-in estimates; delta: smooth noise (Gaussian of
    U(2, 8) cells, std U(30, 100) m/s), clipped so v + delta stays in range.
    Returns (v, v + delta) as float64 [nz, nx]."""
    rng = np.random.default_rng(2_000_000 + seed)
    base = faulted_model(nz, nx, 1_000_000 + seed)
    t = rng.uniform(0.0, 1.0)
    v = np.clip(base + t * smooth_noise(nz, nx, 3_000_000 + seed, 3.0, 600.0), V_LO, V_HI)
    d = smooth_noise(nz, nx, 4_000_000 + seed, rng.uniform(2.0, 8.0), rng.uniform(30.0, 100.0))
    return v, np.clip(v + d, V_LO, V_HI)


OPERATORS = ("Init", "Freq10", "Depth2", "Shot17", "AllChange", "Marmousi-P1", "Marmousi-P3")


def operator_acquisition(name: str, nz: int = 70, nx: int = 70, nb: int = 40) -> Acquisition:
    """Forward-operator configurations of the robustness study (Sec. 6.5, on a 70 x 70 grid with ten
    sources at columns 7k as Init): Freq10 (10 Hz Ricker), Depth2 (sources and receivers two grid
    intervals below the surface), Shot17 (17 evenly placed sources), AllChange (all three); and the
    anisotropic grids of the Marmousi2 crops (table of local models: dx = 10 m or 100/7 m, dz = 2.5 m),
    whose dz needs dt = 0.4 ms (2500 samples for 1 s) by the CFL bound."""
    base = dict(ns=10, shot_cols=even_shot_columns(nx, 10), nt=1000, nb=nb)
    cfg = {
        "Init": {},
        "Freq10": dict(f_peak=10.0),
        "Depth2": dict(src_row=2, rec_row=2),
        "Shot17": dict(ns=17, shot_cols=even_shot_columns(nx, 17)),
        "AllChange": dict(f_peak=10.0, src_row=2, rec_row=2, ns=17, shot_cols=even_shot_columns(nx, 17)),
        "Marmousi-P1": dict(dx=10.0, dz=2.5, dt=4e-4, nt=2500),
        "Marmousi-P3": dict(dx=100.0 / 7.0, dz=2.5, dt=4e-4, nt=2500),
    }[name]
    return surface_acquisition(nz, nx, **{**base, **cfg})


def uneven_requests(n: int = 64, seed0: int = 2000, nb: int = 40, sizes=(70, 140, 256), nts=(1000, 1500, 2500),
                    shots=(5, 10)):
    """Requests of an uneven guidance batch: request r (seed seed0 + r) draws a
    square grid size from `sizes`, a trace length from `nts` and U{shots}
    surface shots placed evenly, one receiver per surface column, dt = 1 ms,
    15 Hz Ricker, dx = 10 m, an nb-cell sponge, and a faulted (even r) or
    layered (odd r) model in 1500-4500 m/s.  Returns [(acq, v, wavelet)]."""
    out = []
    for r in range(n):
        rng = np.random.default_rng(seed0 + r)
        size = int(sizes[int(rng.integers(0, len(sizes)))])
        nt = int(nts[int(rng.integers(0, len(nts)))])
        ns = int(rng.integers(shots[0], shots[1] + 1))
        acq = surface_acquisition(size, size, ns=ns, nt=nt, nb=nb)
        v = faulted_model(size, size, seed0 + r) if r % 2 == 0 else layered_model(
            size, size, seed0 + r, n_layers=2 + r % 3, depth_range=(size // 7, size - size // 7))
        out.append((acq, v, ricker(nt, acq.dt, acq.f_peak)))
    return out
