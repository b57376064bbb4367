"""FP64 CPU oracle for the likelihood-guidance path (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark are the only callers.  The product library
never imports this package, and this package never imports the product.

The arithmetic lives in ``fwi_oracle.c`` (plain C, double precision, OpenMP
across independent (sample, shot) units only); this module marshals numpy
arrays through ctypes.  Functions and the passages they follow:

* :func:`forward`      -- forward operator F(v) (Sec. 2.1 Eq. solving, Sec. 6.1); with
                          ``acq.pml`` the absorbing layer is a PML (Sec. 2.1, Sec. 6.1)
                          instead of the damping sponge
* :func:`gradient`     -- reverse-mode dJ/dv of the discrete objective (either layer)
* :func:`w2_prepare`   -- omega, c', Q_obs, S_obs (Sec. 5.1 (I)-(III), Sec. 6.2)
* :func:`w2_misfit`    -- J (Eq. final_objective) and dJ/dd_syn
* :func:`guidance`     -- TV, rho, kappa and the update (Sec. 5.2, Algorithm 2)
* :func:`l2_misfit`    -- least-squares potential Phi_l2 of baseline DPS (Sec. 4,
                          Algorithm 1) and its weighted / normalised ablation form
* :func:`tv_subgradient` -- g + alpha dTV (Eq. tv) for the TV-regularised baselines (Sec. 6)
* :func:`ddpm_step`    -- clean estimator and DDPM posterior mean + noise of Algorithm 2 (numpy)

Every function is pinned by the CPU tests in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fwi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str) -> str:
    """Compile the same source with AddressSanitizer and UndefinedBehaviorSanitizer (host code) into `path`;
    load it by setting ORACLE_LIB=path in a process started with the ASan runtime preloaded."""
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", path, "-lm"]
    subprocess.run(cmd, check=True)
    return path


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB")
        if not path:
            path = _LIB_PATH
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
        L = ctypes.CDLL(path)
        i, d = ctypes.c_int, ctypes.c_double
        geo = [i, i, d, d, d, i, i, i, d, i, _ip, _ip, i, _ip, _ip]
        L.orc_forward.argtypes = geo + [i, _dp, _dp, _dp]
        L.orc_gradient.argtypes = geo + [i, _dp, _dp, _dp, _dp, _dp]
        L.orc_forward_pml.argtypes = geo + [i, _dp, _dp, _dp]
        L.orc_gradient_pml.argtypes = geo + [i, _dp, _dp, _dp, _dp]
        L.orc_w2_prepare.argtypes = [i, i, d, _dp, d, d, i, d, i, _dp, _dp, _dp, _dp]
        L.orc_w2_misfit.argtypes = [i, i, i, d, _dp, _dp, _dp, _dp, d, d, i, i, i, _dp, _dp, _dp]
        L.orc_quantiles.argtypes = [i, d, _dp, d, i, _dp, _dp]
        L.orc_guidance.argtypes = [i, i, i, _dp, _dp, _dp, _dp, d, d, d, d, d, d, d, _dp, _dp, _dp, _dp]
        L.orc_l2_misfit.argtypes = [i, i, i, _dp, _dp, d, d, i, _dp, _dp]
        L.orc_tv_subgradient.argtypes = [i, i, i, _dp, _dp, d, _dp]
        L.orc_stencil_weights.argtypes = [_dp]
        L.orc_stencil_weights.restype = None
        L.orc_apply_laplacian.argtypes = [i, i, d, d, i, _dp, _dp, i]
        L.orc_sponge.argtypes = [i, i, d, d, d, i, i, d, _dp]
        L.orc_wavefield.argtypes = [i, i, d, d, d, i, i, i, d, i, i, _dp, _dp, i, i, _dp]
        L.orc_cfl_number.argtypes = [d, d, d, d]
        L.orc_cfl_number.restype = d
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        names = {-1: "EINVAL", -2: "ECFL", -3: "ENOMEM"}
        super().__init__(f"{what}: oracle status {code} ({names.get(code, '?')})")
        self.code = code


def _chk(code: int, what: str):
    if code != 0:
        raise OracleError(code, what)


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a: np.ndarray):
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    return a.ctypes.data_as(_ip)


def _geo_args(acq):
    keep = [_i(acq.src_iz), _i(acq.src_ix), _i(acq.rec_iz), _i(acq.rec_ix)]
    args = [acq.nz, acq.nx, acq.dz, acq.dx, acq.dt, acq.nt, acq.nb, int(acq.free_surface), acq.v_max,
            len(keep[0]), _p(keep[0]), _p(keep[1]), len(keep[2]), _p(keep[2]), _p(keep[3])]
    return args, keep


def forward(acq, v: np.ndarray, wavelet: np.ndarray) -> np.ndarray:
    """Traces d[b, s, r, n] = u^n(receiver r) for every sample b and shot s."""
    v = _d(v)
    single = v.ndim == 2
    if single:
        v = v[None]
    B = v.shape[0]
    w = _d(wavelet)
    out = np.zeros((B, acq.ns, acq.nr, acq.nt))
    args, keep = _geo_args(acq)
    if getattr(acq, "pml", False):
        _chk(lib().orc_forward_pml(*args, B, _p(v), _p(w), _p(out)), "orc_forward_pml")
    else:
        _chk(lib().orc_forward(*args, B, _p(v), _p(w), _p(out)), "orc_forward")
    return out[0] if single else out


def gradient(acq, v: np.ndarray, wavelet: np.ndarray, adj: np.ndarray, want_wavelet_grad: bool = False):
    """dJ/dv for a given data-space adjoint a = dJ/dd (reverse mode of the
    discrete time stepping), optionally also dJ/df per shot."""
    v = _d(v)
    single = v.ndim == 2
    if single:
        v = v[None]
        adj = np.asarray(adj)[None]
    B = v.shape[0]
    a = _d(adj)
    assert a.shape == (B, acq.ns, acq.nr, acq.nt)
    g = np.zeros((B, acq.nz, acq.nx))
    gw = np.zeros((B, acq.ns, acq.nt)) if want_wavelet_grad else None
    args, keep = _geo_args(acq)
    if getattr(acq, "pml", False):
        if want_wavelet_grad:
            raise ValueError("the wavelet gradient is not provided with the PML")
        _chk(lib().orc_gradient_pml(*args, B, _p(v), _p(_d(wavelet)), _p(a), _p(g)), "orc_gradient_pml")
    else:
        _chk(lib().orc_gradient(*args, B, _p(v), _p(_d(wavelet)), _p(a), _p(g),
                                _p(gw) if gw is not None else None), "orc_gradient")
    if single:
        g = g[0]
        gw = gw[0] if gw is not None else None
    return (g, gw) if want_wavelet_grad else g


def w2_prepare(d_obs: np.ndarray, dt: float, k: float = 100.0, eps_prime: float = 1e-9, n_xi: int = 1000,
               c_factor: float = 1.1, squared: bool = False) -> dict:
    """Observation-side cache: omega, c', Q_obs and S_obs."""
    d = _d(d_obs)
    shape = d.shape
    nt = shape[-1]
    ntr = int(np.prod(shape[:-1]))
    om = np.zeros(ntr * nt)
    cp = np.zeros(ntr)
    Q = np.zeros(ntr * n_xi)
    S = np.zeros(1)
    _chk(lib().orc_w2_prepare(ntr, nt, dt, _p(d), k, eps_prime, n_xi, c_factor, int(squared), _p(om), _p(cp), _p(Q),
                              _p(S)), "orc_w2_prepare")
    return dict(omega=om.reshape(shape), cprime=cp.reshape(shape[:-1]), Qobs=Q.reshape(shape[:-1] + (n_xi,)),
                S_obs=float(S[0]), dt=dt, eps_prime=eps_prime, n_xi=n_xi, squared=bool(squared), k=k,
                c_factor=c_factor)


def w2_misfit(obs: dict, d_syn: np.ndarray, reduction: int = 0, want_adjoint: bool = True):
    """J per sample and (optionally) the adjoint source dJ/dd_syn, plus per-pair W2."""
    d = _d(d_syn)
    tr_shape = obs["cprime"].shape
    single = d.ndim == len(tr_shape) + 1
    if single:
        d = d[None]
    B = d.shape[0]
    ntr = int(np.prod(tr_shape))
    nt = d.shape[-1]
    J = np.zeros(B)
    adj = np.zeros(d.shape) if want_adjoint else None
    w2 = np.zeros((B,) + tr_shape)
    _chk(lib().orc_w2_misfit(B, ntr, nt, obs["dt"], _p(d), _p(_d(obs["omega"])), _p(_d(obs["cprime"])),
                             _p(_d(obs["Qobs"])), obs["S_obs"], obs["eps_prime"], obs["n_xi"], int(obs["squared"]),
                             int(reduction), _p(J), _p(adj) if adj is not None else None, _p(w2)),
         "orc_w2_misfit")
    if single:
        return J[0], (adj[0] if adj is not None else None), w2[0]
    return J, adj, w2


def quantiles(h: np.ndarray, dt: float, eps_prime: float = 1e-9, n_xi: int = 1000):
    """Quantile function (and CDF) of one shifted trace h >= 0."""
    h = _d(h)
    Q = np.zeros(n_xi)
    F = np.zeros(len(h))
    _chk(lib().orc_quantiles(len(h), dt, _p(h), eps_prime, n_xi, _p(Q), _p(F)), "orc_quantiles")
    return Q, F


def objective(acq, v, wavelet, obs, reduction: int = 0):
    """J(v) through the forward operator and the misfit."""
    d = forward(acq, v, wavelet)
    J, _, _ = w2_misfit(obs, d, reduction=reduction, want_adjoint=False)
    return J


def objective_and_gradient(acq, v, wavelet, obs, reduction: int = 0):
    """J(v) and dJ/dv (m/s units), composing forward, misfit and reverse mode."""
    d = forward(acq, v, wavelet)
    J, adj, _ = w2_misfit(obs, d, reduction=reduction, want_adjoint=True)
    g = gradient(acq, v, wavelet, adj)
    return J, g, d, adj


def guidance(v_prop, h, g, v0hat, rho0=1.15, c=0.1, tau=0.0, gamma=0.55, eps=1e-4, kappa_max=0.0,
             unit_scale=1.0):
    """Preconditioned guidance update; returns (v_next, rho, tv, kappa)."""
    vp, hh, gg, x0 = (_d(a) for a in (v_prop, h, g, v0hat))
    single = vp.ndim == 2
    if single:
        vp, hh, gg, x0 = vp[None], hh[None], gg[None], x0[None]
    B, nz, nx = vp.shape
    vn = np.zeros_like(vp)
    rho = np.zeros(B)
    tv = np.zeros(B)
    kap = np.zeros_like(vp)
    _chk(lib().orc_guidance(B, nz, nx, _p(vp), _p(hh), _p(gg), _p(x0), rho0, c, tau, gamma, eps, kappa_max,
                            unit_scale, _p(vn), _p(rho), _p(tv), _p(kap)), "orc_guidance")
    if single:
        return vn[0], rho[0], tv[0], kap[0]
    return vn, rho, tv, kap


def l2_misfit(d_syn: np.ndarray, d_obs: np.ndarray, sigma: float = 0.05, k: float = 0.0, normalize: bool = False,
              want_adjoint: bool = True):
    """J per sample and dJ/dd_syn of (1/2) sum (w (d_syn - d_obs))^2 / S, with
    w = 1/(1 + k |d_obs| / max|d_obs|) and S = sigma^2 or sum (w d_obs)^2."""
    o = _d(d_obs)
    d = _d(d_syn)
    single = d.ndim == o.ndim
    if single:
        d = d[None]
    B = d.shape[0]
    assert d.shape[1:] == o.shape
    nt = o.shape[-1]
    ntr = int(np.prod(o.shape[:-1]))
    J = np.zeros(B)
    adj = np.zeros(d.shape) if want_adjoint else None
    _chk(lib().orc_l2_misfit(B, ntr, nt, _p(d), _p(o), float(sigma), float(k), int(bool(normalize)), _p(J),
                             _p(adj) if adj is not None else None), "orc_l2_misfit")
    if single:
        return J[0], (adj[0] if adj is not None else None)
    return J, adj


def tv_subgradient(x: np.ndarray, g: np.ndarray | None = None, alpha: float = 1.0) -> np.ndarray:
    """g + alpha q with q a subgradient of TV (Eq. tv) at x (sign(0) = 0)."""
    xx = _d(x)
    single = xx.ndim == 2
    if single:
        xx = xx[None]
    B, nz, nx = xx.shape
    gg = None
    if g is not None:
        gg = _d(g).reshape(B, nz, nx)
    out = np.zeros_like(xx)
    _chk(lib().orc_tv_subgradient(B, nz, nx, _p(xx), _p(gg) if gg is not None else None, float(alpha), _p(out)),
         "orc_tv_subgradient")
    return out[0] if single else out


def stencil_weights() -> np.ndarray:
    w = np.zeros(5)
    lib().orc_stencil_weights(_p(w))
    return w


def apply_laplacian(u: np.ndarray, dz: float, dx: float, free_surface: bool, transpose: bool = False) -> np.ndarray:
    u = _d(u)
    out = np.zeros_like(u)
    _chk(lib().orc_apply_laplacian(u.shape[0], u.shape[1], dz, dx, int(free_surface), _p(u), _p(out),
                                   int(transpose)), "orc_apply_laplacian")
    return out


def sponge(acq) -> np.ndarray:
    """Velocity-damping factor a of every padded node (1 in the model)."""
    nzp, nxp = acq.padded_shape
    a = np.zeros((nzp, nxp))
    _chk(lib().orc_sponge(acq.nz, acq.nx, acq.dz, acq.dx, acq.dt, acq.nb, int(acq.free_surface), acq.v_max, _p(a)),
         "orc_sponge")
    return a


def wavefield(acq, v, wavelet, shot: int = 0, nsteps: int | None = None, check_cfl: bool = True) -> np.ndarray:
    """Padded wavefield u^nsteps of one shot."""
    nzp, nxp = acq.padded_shape
    out = np.zeros((nzp, nxp))
    nsteps = acq.nt - 1 if nsteps is None else nsteps
    w = _d(wavelet)
    _chk(lib().orc_wavefield(acq.nz, acq.nx, acq.dz, acq.dx, acq.dt, len(w), acq.nb, int(acq.free_surface), acq.v_max,
                             int(acq.src_iz[shot]), int(acq.src_ix[shot]), _p(_d(v)), _p(w), int(nsteps),
                             int(check_cfl), _p(out)), "orc_wavefield")
    return out


def cfl_number(v_max: float, dt: float, dz: float, dx: float) -> float:
    """Courant ratio; the scheme is stable iff it is below 1."""
    return float(lib().orc_cfl_number(v_max, dt, dz, dx))


def ddpm_step(v, beta, abar, abar_prev, score=None, v0hat=None, z=None, sigma=0.0):
    """One reverse DDPM step of Algorithm 2 without the guidance term (Sec. 5.3): the clean estimator
    Eq. v0hat, v0hat = (v + (1 - abar_i) s) / sqrt(abar_i), when a score s is given (else the caller's
    v0hat), and the posterior mean plus noise
    v' = sqrt(alpha_i) (1 - abar_{i-1}) / (1 - abar_i) v + sqrt(abar_{i-1}) beta_i / (1 - abar_i) v0hat + sigma z,
    alpha_i = 1 - beta_i.  FP64.  Returns (v0hat, v')."""
    v = np.asarray(v, np.float64)
    if score is not None:
        v0hat = (v + (1.0 - abar) * np.asarray(score, np.float64)) / np.sqrt(abar)
    v0hat = np.asarray(v0hat, np.float64)
    alpha = 1.0 - beta
    vp = np.sqrt(alpha) * (1.0 - abar_prev) / (1.0 - abar) * v + np.sqrt(abar_prev) * beta / (1.0 - abar) * v0hat
    if z is not None:
        vp = vp + sigma * np.asarray(z, np.float64)
    return v0hat, vp
