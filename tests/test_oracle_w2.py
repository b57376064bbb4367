"""Pins of the oracle's Wasserstein-2 misfit (Sec. 5.1 and Sec. 6.2).

Closed forms (integer shift, Gaussians), a brute-force quantile search on
tiny traces, invariances of the normalised objective, the weight's bounds
and finite differences of the adjoint source.
"""
import math

import numpy as np
import pytest


def _bump(nt, centre, width):
    t = np.arange(nt, dtype=np.float64)
    x = (t - centre) / width
    return np.where(np.abs(x) < 1, np.cos(0.5 * math.pi * x) ** 2, 0.0)


def _pair_w2(orc, dobs, dsyn, dt, k=0.0, n_xi=1000, eps=1e-9):
    obs = orc.w2_prepare(dobs[None, None], dt, k=k, n_xi=n_xi, eps_prime=eps)
    J, adj, w2 = orc.w2_misfit(obs, dsyn[None, None])
    return float(w2[0, 0]), obs


@pytest.mark.parametrize("shift", [1, 7, -13, 40])
def test_integer_shift_closed_form(orc, shift):
    """A compact nonnegative density shifted by s samples: every interior
    quantile moves by s dt and the xi = 0 node stays at 0, so
    W2^2 = (s dt)^2 (1 - 1/(2 (N_xi - 1))) exactly (c' = 0 since min = 0, k = 0)."""
    nt, dt, nxi = 600, 1e-3, 1000
    dobs = _bump(nt, 250.0, 30.0)
    dsyn = np.roll(dobs, shift)
    w2, obs = _pair_w2(orc, dobs, dsyn, dt, n_xi=nxi)
    assert obs["cprime"][0, 0] == 0.0
    exact = (shift * dt) ** 2 * (1.0 - 1.0 / (2 * (nxi - 1)))
    assert w2**2 == pytest.approx(exact, rel=1e-9)


def test_gaussian_closed_form(orc):
    """W2^2 between Gaussians = (mu1 - mu2)^2 + (s1 - s2)^2; the quadrature
    error (quantile tails on the xi grid) is below 3e-5 s^2 at N_xi = 1000 and
    shrinks at least 3x at N_xi = 4000."""
    nt, dt = 1000, 1e-3
    t = np.arange(nt) * dt
    for (m1, s1, m2, s2) in [(0.4, 0.03, 0.55, 0.05), (0.3, 0.06, 0.32, 0.02), (0.5, 0.04, 0.5, 0.07)]:
        a = np.exp(-0.5 * ((t - m1) / s1) ** 2)
        b = np.exp(-0.5 * ((t - m2) / s2) ** 2)
        exact = (m1 - m2) ** 2 + (s1 - s2) ** 2
        w2a, _ = _pair_w2(orc, a, b, dt, n_xi=1000)
        w2b, _ = _pair_w2(orc, a, b, dt, n_xi=4000)
        assert abs(w2a**2 - exact) < 3e-5
        assert abs(w2b**2 - exact) < abs(w2a**2 - exact) / 3.0


def test_identity_and_symmetry(orc):
    rng = np.random.default_rng(2)
    nt, dt = 500, 1e-3
    a = np.abs(rng.standard_normal(nt)) * _bump(nt, 200, 150)
    b = np.abs(rng.standard_normal(nt)) * _bump(nt, 260, 150)
    w_aa, _ = _pair_w2(orc, a, a, dt)
    assert w_aa == 0.0
    w_ab, _ = _pair_w2(orc, a, b, dt)
    w_ba, _ = _pair_w2(orc, b, a, dt)
    assert w_ab > 0 and w_ab == pytest.approx(w_ba, rel=1e-12)


def _brute_quantile(h, dt, eps, xi):
    """inf{t : F(t) >= xi} of the piecewise-linear trapezoid CDF, by scanning
    segments and solving the linear crossing -- written independently of the
    oracle's pointer search."""
    nt = len(h)
    Z = sum(dt * (h[k] + h[k + 1]) / 2 for k in range(nt - 1))
    rho = [x / (Z + eps) for x in h]
    F = [0.0]
    for k in range(nt - 1):
        F.append(F[-1] + dt * (rho[k] + rho[k + 1]) / 2)
    x = min(xi, max(F))
    if F[0] >= x:
        return 0.0
    for k in range(1, nt):
        if F[k] >= x:  # crossing on [t_{k-1}, t_k]
            lo, hi = (k - 1) * dt, k * dt
            # bisection on the linear interpolant (independent of the closed form)
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                fm = F[k - 1] + (F[k] - F[k - 1]) * (mid - (k - 1) * dt) / dt
                if fm >= x:
                    hi = mid
                else:
                    lo = mid
            return hi
    raise AssertionError("unreachable")


def test_quantiles_brute_force_tiny(orc):
    """Tiny traces, including one whose density dips negative (non-monotone
    CDF) and one with flat zero stretches: quantiles equal the brute-force
    first crossing, with xi clamped to max F."""
    dt, eps, nxi = 0.1, 1e-9, 9
    traces = [
        np.array([0.0, 1.0, 3.0, 0.5, 2.0, 0.0]),
        np.array([0.2, 2.0, -0.9, -0.8, 1.5, 0.3, 0.1]),  # negative stretch
        np.array([0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 2.0, 0.0]),
        np.array([1.0, 1.0, 1.0, 1.0]),
    ]
    for h in traces:
        Q, F = orc.quantiles(h, dt, eps, nxi)
        for j in range(nxi):
            xi = j / (nxi - 1)
            assert Q[j] == pytest.approx(_brute_quantile(list(h), dt, eps, xi), abs=1e-12), (h, j)


def test_weight_bounds_and_monotone(orc):
    """omega = 1/(1 + k a) lies in [1/(1+k), 1], equals 1/(1+k) at the global
    peak of |d_obs| and 1 at zeros, and decreases with |d_obs| (Eq. omega_def)."""
    rng = np.random.default_rng(4)
    d = rng.standard_normal((3, 4, 200))
    k = 100.0
    obs = orc.w2_prepare(d, 1e-3, k=k)
    om = obs["omega"]
    assert om.min() >= 1 / (1 + k) - 1e-15 and om.max() <= 1.0
    i = np.unravel_index(np.argmax(np.abs(d)), d.shape)
    assert om[i] == pytest.approx(1 / (1 + k), rel=1e-14)
    flat_a = np.abs(d).ravel()
    order = np.argsort(flat_a)
    assert np.all(np.diff(om.ravel()[order]) <= 1e-15)
    d2 = d.copy()
    d2[0, 0, 5] = 0.0
    assert orc.w2_prepare(d2, 1e-3, k=k)["omega"][0, 0, 5] == 1.0


def test_shift_constant_makes_obs_density_nonnegative(orc):
    """c' = 1.1 |min_t omega d_obs| per trace, so min(omega d_obs + c') = 0.1 |min| >= 0."""
    rng = np.random.default_rng(6)
    d = rng.standard_normal((2, 3, 150))
    obs = orc.w2_prepare(d, 1e-3)
    wd = obs["omega"] * d
    mn = wd.min(axis=-1)
    assert np.allclose(obs["cprime"], 1.1 * np.abs(mn), rtol=1e-14)
    assert np.all((wd + obs["cprime"][..., None]).min(axis=-1) >= 0)


def test_objective_invariances(orc):
    """J is unchanged (up to eps') by a joint amplitude scale of d_obs and d_syn
    and by a change of time unit; S_obs depends on observations only."""
    rng = np.random.default_rng(7)
    nt = 400
    t = np.arange(nt)
    base = np.sin(t / 9.0) * np.exp(-((t - 150) / 60.0) ** 2)
    dobs = np.stack([np.roll(base, s) for s in (0, 20, 40)])[None] + 0.01 * rng.standard_normal((1, 3, nt))
    dsyn = np.stack([np.roll(base, s + 5) for s in (0, 20, 40)])[None]
    o1 = orc.w2_prepare(dobs, 1e-3, eps_prime=0.0)
    J1 = orc.w2_misfit(o1, dsyn, want_adjoint=False)[0]
    o2 = orc.w2_prepare(37.0 * dobs, 1e-3, eps_prime=0.0)
    J2 = orc.w2_misfit(o2, 37.0 * dsyn, want_adjoint=False)[0]
    o3 = orc.w2_prepare(dobs, 4e-3, eps_prime=0.0)
    J3 = orc.w2_misfit(o3, dsyn, want_adjoint=False)[0]
    assert J2 == pytest.approx(J1, rel=1e-12)
    assert J3 == pytest.approx(J1, rel=1e-12)
    assert o3["S_obs"] == pytest.approx(4 * o1["S_obs"], rel=1e-12)


def test_reduction_and_power_variants(orc):
    """Sum / S_obs (Eq. final_objective), average over pairs, and the squared
    form sum W2^2 / sum int Q_obs^2 of the raw-trace baseline agree with the
    per-pair distances."""
    rng = np.random.default_rng(8)
    nt = 300
    dobs = rng.standard_normal((2, 5, nt)) * _bump(nt, 120, 100)
    dsyn = np.roll(dobs, 6, axis=-1) + 0.05 * rng.standard_normal((2, 5, nt))
    o = orc.w2_prepare(dobs, 1e-3)
    J0, _, w2 = orc.w2_misfit(o, dsyn, reduction=0, want_adjoint=False)
    J1, _, _ = orc.w2_misfit(o, dsyn, reduction=1, want_adjoint=False)
    assert J0 == pytest.approx(w2.sum() / o["S_obs"], rel=1e-13)
    assert J1 == pytest.approx(w2.mean(), rel=1e-13)
    osq = orc.w2_prepare(dobs, 1e-3, k=0.0, squared=True)
    Jsq, _, w2sq = orc.w2_misfit(osq, dsyn, want_adjoint=False)
    qn = (osq["Qobs"] ** 2)
    wts = np.full(o["n_xi"], 1.0 / (o["n_xi"] - 1))
    wts[0] = wts[-1] = 0.5 / (o["n_xi"] - 1)
    assert osq["S_obs"] == pytest.approx(np.sum(qn * wts), rel=1e-12)
    assert Jsq == pytest.approx(np.sum(w2sq**2) / osq["S_obs"], rel=1e-12)


@pytest.mark.parametrize("squared", [False, True])
def test_adjoint_source_finite_differences(orc, squared):
    """dJ/dd_syn equals central differences in FP64 (away from bracket kinks)."""
    rng = np.random.default_rng(9)
    nt = 400
    t = np.arange(nt)
    dobs = np.stack([np.sin(t / (7.0 + s)) * np.exp(-((t - 150 - 10 * s) / 50.0) ** 2) for s in range(4)])[None]
    dsyn = np.roll(dobs, 4, axis=-1) * 1.1 + 0.02 * rng.standard_normal(dobs.shape)
    o = orc.w2_prepare(dobs, 1e-3, squared=squared)
    J, adj, _ = orc.w2_misfit(o, dsyn)
    scale = np.abs(adj).max()
    for idx in [(0, 0, 150), (0, 1, 170), (0, 2, 10), (0, 3, 390), (0, 3, 200)]:
        e = 1e-7 * np.abs(dsyn).max()
        dp = dsyn.copy()
        dp[idx] += e
        dm = dsyn.copy()
        dm[idx] -= e
        fd = (orc.w2_misfit(o, dp, want_adjoint=False)[0] - orc.w2_misfit(o, dm, want_adjoint=False)[0]) / (2 * e)
        assert abs(adj[idx] - fd) <= 1e-5 * scale, (idx, adj[idx], fd)


def test_gradient_is_the_local_slope_between_jumps(orc):
    """Full-size batch acquisition (70 x 70, 5 shots, 1000 samples): synthetic
    densities omega d + c' go negative (c' is fixed from the observations), so
    the first-crossing quantile makes J jump at isolated points.  Along a
    smooth direction J's slope over 0.01 m/s segments equals the reverse-mode
    directional derivative on every segment but a few (the jumps)."""
    from scipy.ndimage import gaussian_filter

    import fwi_inputs as fi

    acq = fi.surface_acquisition(70, 70, ns=5, nt=1000, nb=40)
    w = fi.ricker(acq.nt, acq.dt, acq.f_peak)
    obs = orc.w2_prepare(orc.forward(acq, fi.faulted_model(70, 70, 1000), w), acq.dt)
    v0 = fi.faulted_model(70, 70, 0)
    dsyn = orc.forward(acq, v0, w)
    dens = obs["omega"].reshape(dsyn.shape) * dsyn + obs["cprime"].reshape(dsyn.shape[:-1])[..., None]
    assert (dens < 0).any()  # the premise: the weighted synthetic density is not nonnegative
    _, g, _, _ = orc.objective_and_gradient(acq, v0[None], w, obs)
    blk = gaussian_filter(np.random.default_rng(0).standard_normal((16, 16)), 2.0)
    d = np.zeros((70, 70))
    d[4:20, 27:43] = blk / np.abs(blk).max()
    an = float(np.sum(g[0] * d))
    hs = np.linspace(-0.05, 0.05, 11)
    J = orc.objective(acq, np.stack([v0 + h * d for h in hs]), w, obs)
    slopes = np.diff(J) / np.diff(hs)
    close = np.abs(slopes - an) <= 1e-3 * abs(an)
    assert close.sum() >= len(slopes) - 2, (an, slopes)
