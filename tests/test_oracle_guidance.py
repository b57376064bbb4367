"""Pins of the oracle's preconditioned guidance update (Sec. 5.2, Algorithm 2).

Special cases that reduce to the baseline DPS step, closed forms of the TV
indicator, properties of rho and kappa, and the descent property that
motivates the preconditioner (Eq. descent_lemma) on a small FWI problem.
"""
import json
import math
import os

import numpy as np
import pytest

import fwi_inputs as fi

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_settings.json")


def _rand(seed, shape=(2, 12, 15)):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(shape) for _ in range(4)]


def test_reduces_to_baseline_dps(orc):
    """gamma = 0 makes kappa = 1 and tau = inf makes rho = rho0, so the step is
    v' - rho0 h: P_i = zeta I (Eq. precond_step)."""
    vp, h, g, x0 = _rand(0)
    vn, rho, tv, kap = orc.guidance(vp, h, g, x0, rho0=0.7, gamma=0.0, tau=1e30)
    assert np.all(kap == 1.0)
    assert np.all(rho == 0.7)
    assert np.allclose(vn, vp - 0.7 * h, rtol=0, atol=1e-15)


def test_tv_closed_forms(orc):
    """TV of a constant field is 0; one flat interface of jump a contributes
    a * nx / (nz nx); a checkerboard of +-1 gives 2 (2 nz nx - nz - nx)/(nz nx)."""
    nz, nx = 10, 14
    const = np.full((1, nz, nx), 0.3)
    z = np.zeros((1, nz, nx))
    _, rho, tv, _ = orc.guidance(z, z, z + 1, const, rho0=2.0, c=0.1, tau=0.0)
    assert tv[0] == 0.0 and rho[0] == 2.0
    step = np.zeros((1, nz, nx))
    step[:, 6:, :] = 0.45
    _, rho, tv, _ = orc.guidance(z, z, z + 1, step, rho0=2.0, c=0.1, tau=0.0)
    assert tv[0] == pytest.approx(0.45 * nx / (nz * nx), rel=1e-14)
    assert rho[0] == pytest.approx(2.0 * math.exp(-tv[0] / 0.1), rel=1e-14)
    cb = np.where((np.add.outer(np.arange(nz), np.arange(nx)) % 2) == 0, 1.0, -1.0)[None]
    _, _, tv, _ = orc.guidance(z, z, z + 1, cb, tau=0.0)
    assert tv[0] == pytest.approx(2 * (2 * nz * nx - nz - nx) / (nz * nx), rel=1e-14)


def test_rho_schedule_properties(orc):
    """rho in (0, rho0], rho = rho0 when TV <= tau, monotone decreasing in TV
    beyond tau (Eq. rho)."""
    nz, nx = 8, 8
    z = np.zeros((1, nz, nx))
    rhos = []
    for a in [0.0, 0.05, 0.1, 0.2, 0.4]:
        step = np.zeros((1, nz, nx))
        step[:, 4:, :] = a
        _, rho, tv, _ = orc.guidance(z, z, z + 1, step, rho0=1.5, c=0.1, tau=0.02)
        rhos.append(rho[0])
        if tv[0] <= 0.02:
            assert rho[0] == 1.5
    assert all(0 < r <= 1.5 for r in rhos)
    assert all(rhos[i + 1] <= rhos[i] for i in range(len(rhos) - 1))


def test_kappa_properties(orc):
    """kappa >= 1 everywhere, = 1 at argmax |g|, equals the closed form at a
    zero of g, and is capped by kappa_max when given (Eq. kappa)."""
    vp, h, g, x0 = _rand(1, (1, 9, 11))
    g[0, 3, 4] = 0.0
    eps, gamma = 1e-4, 0.55
    _, _, _, kap = orc.guidance(vp, h, g, x0, gamma=gamma, eps=eps)
    assert np.all(kap >= 1.0)
    i = np.unravel_index(np.argmax(np.abs(g[0])), g[0].shape)
    assert kap[0][i] == 1.0
    gmax = np.abs(g).max()
    assert kap[0, 3, 4] == pytest.approx(((gmax + eps) / eps) ** gamma, rel=1e-14)
    _, _, _, kc = orc.guidance(vp, h, g, x0, gamma=gamma, eps=eps, kappa_max=5.0)
    assert kc.max() == 5.0 and np.all(kc <= kap)


def test_unit_scale_is_a_chain_factor(orc):
    """Gradients given per m/s and a chain factor s equal gradients given
    already in diffusion-state units."""
    vp, h, g, x0 = _rand(2)
    s = 1500.0
    a = orc.guidance(vp, h, g, x0, unit_scale=s)
    b = orc.guidance(vp, s * h, s * g, x0, unit_scale=1.0)
    assert np.allclose(a[0], b[0], rtol=1e-14, atol=1e-14)
    assert np.allclose(a[3], b[3], rtol=1e-14)


def test_paper_settings_fixture_defaults(orc):
    """The fixed settings of Sec. 6.3 and the CurveVel-A column of Table
    'parameter' are the defaults the oracle's wrapper uses."""
    gold = json.load(open(GOLD))
    import inspect

    sig = inspect.signature(orc.guidance)
    assert sig.parameters["eps"].default == gold["fixed"]["eps"]
    assert sig.parameters["c"].default == gold["fixed"]["c"]
    assert sig.parameters["tau"].default == gold["fixed"]["tau"]
    assert sig.parameters["gamma"].default == gold["ours"]["CurveVel-A"]["gamma"]
    assert sig.parameters["rho0"].default == gold["ours"]["CurveVel-A"]["rho0"]
    sigw = inspect.signature(orc.w2_prepare)
    assert sigw.parameters["k"].default == gold["fixed"]["k"]
    assert sigw.parameters["eps_prime"].default == gold["w2_numerics"]["eps_prime"]
    assert sigw.parameters["n_xi"].default == gold["w2_numerics"]["n_xi"]
    assert sigw.parameters["c_factor"].default == gold["w2_numerics"]["c_prime_factor"]
    assert list(fi.even_shot_columns(70, 10)) == gold["acquisition"]["shot_columns_10"]


def test_descent_for_small_step(orc):
    """For a small rho0 the preconditioned step v - rho kappa g lowers J
    (Eq. descent_lemma with ||P|| small), on a small FWI problem with h = g."""
    rng = np.random.default_rng(3)
    nz, nx = 16, 16
    acq = fi.surface_acquisition(nz, nx, ns=2, shot_cols=[3, 11], nt=300, nb=6, v_max=5000.0)
    vt = fi.layered_model(nz, nx, 1, depth_range=(4, 12), v_hi=4000.0)
    v = vt + 150.0 * rng.standard_normal((nz, nx))
    w = fi.ricker(acq.nt, acq.dt, 15.0)
    obs = orc.w2_prepare(orc.forward(acq, vt, w), acq.dt)
    J0, g, _, _ = orc.objective_and_gradient(acq, v, w, obs)
    x0 = fi.to_normalised(v)
    gn = g  # J per m/s
    step_scale = 5.0 / np.abs(gn).max()  # a 5 m/s change at the largest entry before kappa
    vn, rho, tv, kap = orc.guidance(v, gn, gn, x0, rho0=step_scale, gamma=0.55, c=0.1, tau=0.0)
    J1 = orc.objective(acq, vn, w, obs)
    pred = -np.sum(rho * kap * gn * gn)
    assert J1 < J0
    assert (J1 - J0) == pytest.approx(pred, rel=0.2)
