"""Pins of the oracle's forward operator against mathematics it must satisfy.

Each check is chosen so that a plausible slip in the oracle (a wrong stencil
weight, a missing 1/dx^2, a misplaced mirror ghost, a source scaled or timed
wrongly, a transposition error in the reverse sweep) fails at least one test.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import fwi_inputs as fi


def test_stencil_polynomial_exactness(orc):
    """Central weights differentiate x^p exactly for p <= 9 (8th order), not p = 10."""
    w = orc.stencil_weights()
    h = 0.37
    x0 = 0.83
    for p in range(0, 11):
        approx = w[0] * x0**p + sum(w[k] * ((x0 + k * h) ** p + (x0 - k * h) ** p) for k in range(1, 5))
        approx /= h * h
        exact = p * (p - 1) * x0 ** (p - 2) if p >= 2 else 0.0
        if p <= 9:
            assert abs(approx - exact) <= 1e-9 * max(1.0, abs(exact)), p
        else:
            assert abs(approx - exact) > 1e-6 * abs(exact)


def test_stencil_nyquist_symbol():
    """The weights' symbol peaks at theta = pi with magnitude 2048/315 (the CFL constant)."""
    import oracle

    w = oracle.stencil_weights()
    th = np.linspace(0, math.pi, 20001)
    sym = w[0] + 2 * sum(w[k] * np.cos(k * th) for k in range(1, 5))
    assert np.argmin(sym) == len(th) - 1
    assert abs(-sym[-1] - 2048.0 / 315.0) < 1e-12


def test_laplacian_2d_polynomial_and_spacings(orc):
    """L applied to a 2-D polynomial of degree <= 9 per axis is exact away from
    the edges, with distinct dz and dx."""
    nzp, nxp, dz, dx = 30, 34, 2.5, 10.0
    z = np.arange(nzp)[:, None] * dz
    x = np.arange(nxp)[None, :] * dx
    zs, xs = z / 50.0, x / 200.0
    u = zs**7 - 3 * zs**3 + xs**9 + 2 * xs**2 * zs**2
    lap = orc.apply_laplacian(u, dz, dx, free_surface=False)
    uzz = (42 * zs**5 - 18 * zs + 4 * xs**2) / 50.0**2
    uxx = (72 * xs**7 + 4 * zs**2) / 200.0**2
    exact = uzz + uxx
    inner = (slice(4, nzp - 4), slice(4, nxp - 4))
    assert np.max(np.abs(lap[inner] - exact[inner])) <= 1e-10 * np.max(np.abs(exact[inner]))


def test_reflecting_top_mirror(orc):
    """With the reflecting top, an even-in-z polynomial (d_z u = 0 at row 0) is
    differentiated exactly on the top rows too; an odd one is not."""
    nzp, nxp, dz, dx = 20, 20, 10.0, 10.0
    z = np.arange(nzp)[:, None] * dz / 100.0
    u_even = (z**2 + 0.5 * z**4 - z**8) * np.ones((1, nxp))
    lap = orc.apply_laplacian(u_even, dz, dx, free_surface=True)
    exact = (2 + 6 * z**2 - 56 * z**6) / 100.0**2
    cols = slice(4, nxp - 4)
    assert np.allclose(lap[:8, cols], np.broadcast_to(exact[:8], lap[:8, cols].shape), rtol=1e-9, atol=1e-12)
    u_odd = z * np.ones((1, nxp))
    lap_odd = orc.apply_laplacian(u_odd, dz, dx, free_surface=True)
    assert np.max(np.abs(lap_odd[:4, cols])) > 1e-6


@pytest.mark.parametrize("fs", [False, True])
def test_laplacian_transpose_and_weighted_symmetry(orc, fs):
    """The scatter transpose is the matrix transpose, and with the top mirror
    diag(1/2 on row 0, 1 elsewhere) L is symmetric."""
    rng = np.random.default_rng(3)
    nzp, nxp = 17, 13
    a = rng.standard_normal((nzp, nxp))
    b = rng.standard_normal((nzp, nxp))
    La = orc.apply_laplacian(a, 7.0, 5.0, fs)
    LTb = orc.apply_laplacian(b, 7.0, 5.0, fs, transpose=True)
    assert abs(np.sum(La * b) - np.sum(a * LTb)) <= 1e-12 * np.sum(np.abs(La * b))
    W = np.ones((nzp, 1))
    if fs:
        W[0] = 0.5
    Lb = orc.apply_laplacian(b, 7.0, 5.0, fs)
    lhs = np.sum(W * La * b)
    rhs = np.sum(a * W * Lb)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(W * La * b))
    if fs:  # without the weight the mirrored operator is not symmetric
        assert abs(np.sum(La * b) - np.sum(a * Lb)) > 1e-6 * np.sum(np.abs(La * b))


def test_sponge_absorbs(orc):
    """With the sponge the field energy left after the wave has crossed the
    model is a small fraction of that without it (reflecting edges)."""
    v = np.full((40, 40), 2000.0)
    w = fi.ricker(400, 1e-3, 15.0)
    e = {}
    for nb in (0, 30):
        acq = fi.surface_acquisition(40, 40, ns=1, shot_cols=[20], nt=400, nb=nb, free_surface=False)
        acq.src_iz = np.array([20], np.int32)
        u = orc.wavefield(acq, v, w, nsteps=399)
        sl = (slice(nb, nb + 40), slice(nb, nb + 40))
        e[nb] = np.sum(u[sl] ** 2)
    assert e[30] < 0.02 * e[0]


def _green_trace(r, v, t, f):
    """2-D Green's function of (1/v^2) d_tt - Laplacian convolved with f:
    u(r,t) = 1/(2 pi) int_0^{acosh(v t / r)} f(t - (r/v) cosh a) da."""
    out = np.zeros_like(t)
    for i, ti in enumerate(t):
        if v * ti <= r:
            continue
        th = math.acosh(v * ti / r)
        out[i] = quad(lambda a: f(ti - (r / v) * math.cosh(a)), 0, th, limit=200)[0] / (2 * math.pi)
    return out


def test_homogeneous_green_function_second_order_in_time(orc):
    """A surface source in a homogeneous medium with the mirror top is the
    full-space point source; traces match the analytic 2-D Green's function
    (before any edge reflection) and the error falls ~4x when dt halves."""
    v0, fp = 2000.0, 15.0
    t0 = 1.1 / fp

    def f(t):
        a = (math.pi * fp * (t - t0)) ** 2
        return (1 - 2 * a) * math.exp(-a)

    errs = []
    for dt in (5e-4, 2.5e-4):
        nt = int(round(0.2 / dt)) + 1
        acq = fi.surface_acquisition(60, 120, ns=1, shot_cols=[60], nt=nt, nb=0, dx=5.0, dt=dt,
                                     rec_cols=[40, 80], v_max=v0)
        acq.rec_iz = np.array([0, 20], dtype=np.int32)  # one surface receiver, one 100 m deep
        acq.rec_ix = np.array([40, 60], dtype=np.int32)
        d = orc.forward(acq, np.full((60, 120), v0), fi.ricker(nt, dt, fp))
        t = np.arange(nt) * dt
        g = _green_trace(100.0, v0, t, f)
        e = [np.linalg.norm(d[0, k] - g) / np.linalg.norm(g) for k in range(2)]
        errs.append(e)
    assert max(errs[0]) < 2e-3
    assert max(errs[1]) < 5e-4
    for k in range(2):
        assert 3.0 < errs[0][k] / errs[1][k] < 5.0


def _one_pair(acq, s, r):
    import dataclasses

    return dataclasses.replace(acq, src_iz=np.array([s[0]], np.int32), src_ix=np.array([s[1]], np.int32),
                               rec_iz=np.array([r[0]], np.int32), rec_ix=np.array([r[1]], np.int32))


def test_reciprocity(orc):
    """Swapping source and receiver leaves the trace unchanged when both lie on
    the surface or both in the interior (heterogeneous medium, sponge).  With
    W = diag(1/2 on the surface row, 1 elsewhere), W(M - L) is symmetric for the
    time-stepping operator M - L, so G_rs / G_sr = w_s / w_r: a surface-interior
    swap scales the trace by exactly 2."""
    rng = np.random.default_rng(11)
    nz, nx = 24, 30
    v = 1800 + 1500 * rng.random((nz, nx))
    acq = fi.surface_acquisition(nz, nx, ns=1, nt=400, nb=8, dx=10.0, dt=1e-3)
    w = fi.ricker(acq.nt, acq.dt, 15.0)
    pairs = [((0, 4), (0, 23)), ((7, 5), (18, 21))]
    for a, b in pairs:
        dab = orc.forward(_one_pair(acq, a, b), v, w)[0, 0]
        dba = orc.forward(_one_pair(acq, b, a), v, w)[0, 0]
        assert np.linalg.norm(dab - dba) <= 1e-12 * np.linalg.norm(dab)
    s_surf, r_int = (0, 6), (15, 20)
    d1 = orc.forward(_one_pair(acq, s_surf, r_int), v, w)[0, 0]  # recorded in the interior
    d2 = orc.forward(_one_pair(acq, r_int, s_surf), v, w)[0, 0]  # recorded on the surface
    assert np.linalg.norm(d2 - 2.0 * d1) <= 1e-12 * np.linalg.norm(d2)


def test_linearity_in_source(orc):
    acq = fi.surface_acquisition(20, 20, ns=2, nt=200, nb=6)
    v = fi.layered_model(20, 20, 4, depth_range=(3, 16))
    w = fi.ricker(acq.nt, acq.dt, 15.0)
    d1 = orc.forward(acq, v, w)
    d2 = orc.forward(acq, v, -2.5 * w)
    assert np.allclose(d2, -2.5 * d1, rtol=1e-13, atol=1e-13 * np.abs(d1).max())


def test_cfl_bound_and_rejection(orc):
    """Stable for 10^4 steps just below the leapfrog bound, explosive just above,
    and the modelling call refuses a declared v_max beyond it."""
    nz = nx = 32
    dx = 10.0
    vcrit = 2.0 / math.sqrt(2048.0 / 315.0 * 2.0 / dx**2) / 1e-3  # dt = 1 ms
    assert orc.cfl_number(vcrit, 1e-3, dx, dx) == pytest.approx(1.0, rel=1e-14)
    w = fi.ricker(40, 1e-3, 15.0)
    res = {}
    for fac in (0.99, 1.01):
        vv = vcrit * fac
        acq = fi.surface_acquisition(nz, nx, ns=1, shot_cols=[16], nt=40, nb=0, free_surface=False, dx=dx,
                                     v_max=vv)
        acq.src_iz = np.array([16], np.int32)
        u = orc.wavefield(acq, np.full((nz, nx), vv), w, nsteps=10000, check_cfl=False)
        res[fac] = np.max(np.abs(u)) if np.all(np.isfinite(u)) else np.inf
    assert res[0.99] < 1.0
    assert res[1.01] > 1e6
    acq = fi.surface_acquisition(nz, nx, ns=1, nt=40, nb=0, dx=dx, v_max=vcrit * 1.001)
    with pytest.raises(orc.OracleError) as e:
        orc.forward(acq, np.full((nz, nx), vcrit), w)
    assert e.value.code == -2


def test_adjoint_dot_product(orc):
    """<S f, a> = <f, S^T a> for the linear map wavelet -> traces, with S^T the
    oracle's reverse sweep (heterogeneous medium, sponge, mirror top)."""
    rng = np.random.default_rng(5)
    nz, nx = 18, 22
    acq = fi.surface_acquisition(nz, nx, ns=2, nt=250, nb=7)
    acq.rec_iz = np.array([0, 0, 3, 9, 17], np.int32)
    acq.rec_ix = np.array([0, 10, 21, 4, 12], np.int32)
    v = 1700 + 2500 * rng.random((nz, nx))
    f = rng.standard_normal(acq.nt)
    a = rng.standard_normal((acq.ns, acq.nr, acq.nt))
    d = orc.forward(acq, v, f)
    _, gw = orc.gradient(acq, v, f, a, want_wavelet_grad=True)
    lhs = np.sum(d * a)
    rhs = np.sum(gw * f[None, :])
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(d) * np.linalg.norm(a))


def _small_problem(seed=0, nz=16, nx=16, nt=300):
    rng = np.random.default_rng(seed)
    acq = fi.surface_acquisition(nz, nx, ns=2, shot_cols=[3, 11], nt=nt, nb=6)
    v = 2000 + 600 * rng.random((nz, nx))
    vt = v * (1 + 0.05 * rng.standard_normal((nz, nx)))
    w = fi.ricker(acq.nt, acq.dt, 15.0)
    return acq, v, vt, w


def test_gradient_fd_least_squares(orc):
    """Reverse-mode dJ/dv equals central finite differences of the smooth
    J = 1/2 ||F(v) - d||^2 (second-order FD error ~1e-10 at h = 1e-5 v),
    including edge cells whose sponge copies fold back and the source column."""
    acq, v, vt, w = _small_problem()
    dobs = orc.forward(acq, vt, w)
    d = orc.forward(acq, v, w)
    g = orc.gradient(acq, v, w, d - dobs)

    def J(vv):
        return 0.5 * np.sum((orc.forward(acq, vv, w) - dobs) ** 2)

    for iz, ix in [(0, 0), (3, 5), (15, 15), (0, 3), (10, 0), (0, 15), (15, 7)]:
        h = 1e-5 * v[iz, ix]
        vp = v.copy()
        vp[iz, ix] += h
        vm = v.copy()
        vm[iz, ix] -= h
        fd = (J(vp) - J(vm)) / (2 * h)
        assert abs(g[iz, ix] - fd) <= 1e-7 * abs(fd), (iz, ix, g[iz, ix], fd)


def test_gradient_fd_w2_objective(orc):
    """Full chain: forward, W2 misfit, adjoint source and reverse sweep agree
    with central differences of J(v) at h = 1e-6 v, to 1e-5 of max|g| (the
    quantile brackets make J only piecewise smooth)."""
    acq, v, vt, w = _small_problem(seed=1)
    dobs = orc.forward(acq, vt, w)
    obs = orc.w2_prepare(dobs, acq.dt)
    J, g, _, _ = orc.objective_and_gradient(acq, v, w, obs)
    for iz, ix in [(0, 0), (8, 8), (0, 7), (12, 3)]:
        h = 1e-6 * v[iz, ix]
        vp = v.copy()
        vp[iz, ix] += h
        vm = v.copy()
        vm[iz, ix] -= h
        fd = (orc.objective(acq, vp, w, obs) - orc.objective(acq, vm, w, obs)) / (2 * h)
        assert abs(g[iz, ix] - fd) <= 1e-5 * np.max(np.abs(g)), (iz, ix, g[iz, ix], fd)
